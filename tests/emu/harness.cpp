// Host harness for the CPU emulation of the library's kernels (built by
// tests/test_emulated_kernels.py with clang++ and AddressSanitizer against the
// shim in tests/emu/hip).  It calls the library's internal entry points (the
// C ABI wrappers in capi.hip are not linked), whose kernels then run on the
// host:
//
//   harness fsg D.bin Q.bin gx gy gz d t0 t1 out.bin              -> "status n"
//   harness search D.bin Q.bin layout prec d t0 t1 cap out.bin [bins] -> "status n ftests"
//   harness selfjoin D.bin layout prec d t0 t1 cap out.bin        -> "status n ftests"
//   harness merge recs.bin capacity out.bin                       -> "status n"
//   harness hostsearch D.bin Q.bin d t0 t1 out.bin                -> "status n candidates"
//   harness fill seed W C K frac add align prefix                 -> "status count cap T holes R"
//   harness filtercheck seed n                                    -> "status accepted misses naive"
//   harness cvt in.bin out.bin                                    -> "status n"
//
// D.bin / Q.bin: 9 float64 columns (xs ys zs ts xe ye ze te traj), column
// after column.  recs.bin: tds_result records.  out.bin: the records or
// intervals written.
//
// "fill" runs the direct-output fill pass (k_fill_plan, k_fill_copy) alone on
// a synthetic reservation pattern: W waves append random runs of 1..64
// results in chunks of C positions, as the distance kernel's direct output
// does, in a random interleaving (K runs per wave at most); the capacity is
// floor(count * frac) + add (rounded down to a multiple of C if align).  It
// writes prefix.all (every result: id in q_seg, position in e_seg, e_traj 1 if
// its position was kept in the output or scratch), prefix.before and
// prefix.after (the first T = min(count, capacity) output records before and
// after the fill; holes are 0xFFFFFFFF).
//
// "filtercheck" draws n grazing pairs at random scales (coordinates, lengths
// and d from 1e-3 to 1e9, separations of d (1 + eps) with eps down to 0) and
// counts the pairs that the canonical evaluation accepts but the FP32
// filter (sphere32 spheres and sphere_pass, the outward-rounded time
// extents, seg_box32 boxes and box_overlap, built as the kernels build them)
// would drop: "misses", which must be 0.  "naive" counts the accepted pairs
// that boxes without margins (end points rounded to nearest, grown by d in
// FP32) would drop, which shows that the pairs are close enough to the
// boundary to matter.
//
// "cvt" converts the float64 values of in.bin to float32 rounded downwards
// and upwards (f32_rd, f32_ru) and writes them as pairs.
//
// search.hip is part of this translation unit (not compiled on its own), so
// that the fill kernels in its anonymous namespace can be launched directly.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <numeric>
#include <random>
#include <vector>

#include "search.hip"

long emu_launches = 0;

namespace tds {
int build_impl(const tds_segments* D, const tds_build_params* p, hipStream_t stream,
               tds_index** out);
void destroy_index(tds_index* idx);
int search_impl(tds_index* idx, const tds_segments* Q, double d, double t_start, double t_end,
                tds_result* out, uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
                hipStream_t stream, tds_stats* stats);
int self_join_impl(tds_index* idx, double d, double t_start, double t_end, tds_result* out,
                   uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
                   hipStream_t stream, tds_stats* stats);
int fsg_build(const tds_index* idx, uint32_t gx, uint32_t gy, uint32_t gz, hipStream_t s,
              tds_fsg** out);
void fsg_destroy(tds_fsg* f);
int fsg_search(const tds_fsg* f, const tds_segments* Q, double d, double t_start, double t_end,
               tds_result* out, uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
               hipStream_t s, tds_stats* stats);
int merge_impl(const tds_result* recs, uint64_t n, bool recs_dev, tds_traj_interval* out,
               uint64_t capacity, bool out_dev, uint64_t* n_out, hipStream_t s);
}  // namespace tds

// As in the C ABI (capi.hip, not linked here).
extern "C" void tds_search_params_default(tds_search_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->precision = TDS_PREC_FP32_RECHECK;
}

namespace {

std::vector<char> read_file(const char* path) {
    std::ifstream f(path, std::ios::binary);
    f.seekg(0, std::ios::end);
    const size_t bytes = (size_t)f.tellg();
    f.seekg(0);
    std::vector<char> v(bytes);
    f.read(v.data(), (std::streamsize)bytes);
    return v;
}

struct Columns {
    std::vector<double> v;
    size_t n = 0;
    const double* col(int k) const { return v.data() + (size_t)k * n; }
};

Columns read_columns(const char* path) {
    const std::vector<char> raw = read_file(path);
    Columns c;
    c.v.resize(raw.size() / sizeof(double));
    std::memcpy(c.v.data(), raw.data(), c.v.size() * sizeof(double));
    c.n = c.v.size() / 9;
    return c;
}

// Segment view of the columns (host memory) with trajectory ids.
struct SegSet {
    std::vector<uint32_t> traj;
    tds_segments s{};
    explicit SegSet(const Columns& c) : traj(c.n) {
        for (size_t i = 0; i < c.n; ++i) traj[i] = (uint32_t)c.col(8)[i];
        s.xs = c.col(0);
        s.ys = c.col(1);
        s.zs = c.col(2);
        s.ts = c.col(3);
        s.xe = c.col(4);
        s.ye = c.col(5);
        s.ze = c.col(6);
        s.te = c.col(7);
        s.traj_id = traj.data();
        s.n = c.n;
        s.on_device = 0;
    }
};

void write_records(const char* path, const std::vector<tds_result>& out, uint64_t n) {
    FILE* fo = fopen(path, "wb");
    fwrite(out.data(), sizeof(tds_result), std::min<uint64_t>(n, out.size()), fo);
    fclose(fo);
}

tds_index* build(const Columns& D, uint32_t layout, uint32_t num_bins = 0) {
    SegSet S(D);
    tds_build_params bp{};
    bp.layout = layout;
    bp.num_bins = num_bins;
    tds_index* idx = nullptr;
    const int st = tds::build_impl(&S.s, &bp, nullptr, &idx);
    if (st != TDS_OK) {
        printf("%d 0 0\n", st);
        exit(0);
    }
    return idx;
}

int run_fsg(char** argv) {
    const Columns D = read_columns(argv[2]);
    const Columns Qc = read_columns(argv[3]);
    const uint32_t g[3] = {(uint32_t)atoi(argv[4]), (uint32_t)atoi(argv[5]),
                           (uint32_t)atoi(argv[6])};
    const double d = atof(argv[7]), t0 = atof(argv[8]), t1 = atof(argv[9]);
    tds_index* idx = build(D, TDS_LAYOUT_DEFAULT);
    tds_fsg* f = nullptr;
    int st = tds::fsg_build(idx, g[0], g[1], g[2], nullptr, &f);
    if (st != TDS_OK) {
        printf("%d 0\n", st);
        return 0;
    }
    SegSet Q(Qc);
    std::vector<tds_result> out(1u << 20);
    uint64_t n = 0;
    st = tds::fsg_search(f, &Q.s, d, t0, t1, out.data(), out.size(), &n, nullptr, nullptr, nullptr);
    write_records(argv[10], out, n);
    tds::fsg_destroy(f);
    tds::destroy_index(idx);
    printf("%d %llu\n", st, (unsigned long long)n);
    return 0;
}

// search / self-join: layout and precision by their C ABI values
int run_search(int argc, char** argv, bool self_join) {
    int a = 2;
    const Columns D = read_columns(argv[a++]);
    Columns Qc;
    if (!self_join) Qc = read_columns(argv[a++]);
    const uint32_t layout = (uint32_t)atoi(argv[a++]);
    const int prec = atoi(argv[a++]);
    const double d = atof(argv[a++]), t0 = atof(argv[a++]), t1 = atof(argv[a++]);
    const uint64_t cap = strtoull(argv[a++], nullptr, 10);
    const char* path = argv[a++];
    const uint32_t num_bins = (a < argc) ? (uint32_t)atoi(argv[a++]) : 0u;  // 0: automatic
    const uint32_t refine = (a < argc) ? (uint32_t)atoi(argv[a++]) : 0u;    // TDS_REFINE_*
    const uint32_t tile = (a < argc) ? (uint32_t)atoi(argv[a++]) : 0u;
    const uint32_t output = (a < argc) ? (uint32_t)atoi(argv[a++]) : 0u;  // TDS_OUTPUT_*
    tds_index* idx = build(D, layout, num_bins);
    tds_search_params p;
    tds_search_params_default(&p);
    p.precision = prec;
    p.refine = refine;
    p.tile = tile;
    p.output = output;
    p.grid_waves = 64;  // 16 persistent workgroups: fewer idle host threads
    std::vector<tds_result> out(std::max<uint64_t>(cap, 1));
    uint64_t n = 0;
    tds_stats st{};
    int status;
    if (self_join) {
        status = tds::self_join_impl(idx, d, t0, t1, out.data(), cap, &n, &p, nullptr, &st);
    } else {
        SegSet Q(Qc);
        status = tds::search_impl(idx, &Q.s, d, t0, t1, out.data(), cap, &n, &p, nullptr, &st);
    }
    write_records(path, out, n);
    tds::destroy_index(idx);
    printf("%d %llu %llu %llu\n", status, (unsigned long long)n, (unsigned long long)st.filter_tests,
           (unsigned long long)st.stage_flushes);
    return 0;
}

// The serving loop's host route: the index built by the (emulated) kernels,
// copied to host memory, searched on the host.
int run_hostsearch(char** argv) {
    const Columns D = read_columns(argv[2]);
    const Columns Qc = read_columns(argv[3]);
    const double d = atof(argv[4]), t0 = atof(argv[5]), t1 = atof(argv[6]);
    tds_index* idx = build(D, TDS_LAYOUT_DEFAULT);
    tds::HostIndex h;
    const int st = tds::host_index_load(idx, &h);
    SegSet Q(Qc);
    std::vector<tds_result> out;
    uint64_t cand = 0;
    if (st == TDS_OK) {
        cand = tds::host_candidates(h, Qc.col(0), Qc.n, t0, t1, ~0ull);
        tds::host_search(h, Qc.col(0), Q.traj.data(), Qc.n, d, t0, t1, &out);
    }
    write_records(argv[7], out, out.size());
    tds::destroy_index(idx);
    printf("%d %llu %llu\n", st, (unsigned long long)out.size(), (unsigned long long)cand);
    return 0;
}

int run_fill(char** argv) {
    std::mt19937_64 rng(strtoull(argv[2], nullptr, 10));
    const uint32_t W = (uint32_t)atoi(argv[3]), C = (uint32_t)atoi(argv[4]),
                   K = (uint32_t)atoi(argv[5]);
    const double frac = atof(argv[6]);
    const int64_t add = strtoll(argv[7], nullptr, 10);
    const bool align = atoi(argv[8]) != 0;
    const std::string prefix = argv[9];
    if (W == 0 || W > tds::kMaxDirectWaves || C < 64 || C > 2048 || C % 64) {
        printf("%d 0 0 0 0 0\n", TDS_E_INVALID);
        return 0;
    }
    // the runs of each wave, then a random interleaving of them
    std::vector<std::vector<uint32_t>> runs(W);
    std::vector<uint32_t> order;
    for (uint32_t w = 0; w < W; ++w) {
        const uint32_t nr = (uint32_t)(rng() % (K + 1));
        for (uint32_t r = 0; r < nr; ++r) {
            runs[w].push_back(1 + (uint32_t)(rng() % 64));
            order.push_back(w);
        }
    }
    std::shuffle(order.begin(), order.end(), rng);
    // positions: a wave fills its chunk from the front and reserves the next
    // chunk from the shared counter when a run does not fit
    struct Placed {
        uint64_t id, pos;
    };
    std::vector<Placed> placed;
    std::vector<uint64_t> dpos(W, 0), dend(W, 0);
    std::vector<size_t> next(W, 0);
    uint64_t ctr = 0;
    for (uint32_t w : order) {
        const uint32_t nhit = runs[w][next[w]++];
        const uint64_t room = dend[w] - dpos[w];
        uint64_t b = 0;
        if (nhit > room) {
            b = ctr;
            ctr += C;
        }
        for (uint32_t r = 0; r < nhit; ++r) {
            const uint64_t pos = r < room ? dpos[w] + r : b + (r - room);
            placed.push_back({placed.size(), pos});
        }
        if (nhit > room) {
            dpos[w] = b + (nhit - room);
            dend[w] = b + C;
        } else {
            dpos[w] += nhit;
        }
    }
    const uint64_t count = placed.size();
    int64_t capi = (int64_t)std::floor((double)count * frac) + add;
    if (capi < 0) capi = 0;
    uint64_t cap = (uint64_t)capi;
    if (align) cap -= cap % C;
    const uint64_t scap = (uint64_t)W * C;
    const uint64_t T = std::min(count, cap);
    constexpr uint32_t kHole = 0xFFFFFFFFu;
    tds_result blank{};
    blank.q_seg = blank.e_seg = kHole;
    std::vector<tds_result> out(std::max<uint64_t>(cap, 1), blank), scratch(scap, blank);
    std::vector<tds_result> all(count);
    for (const Placed& p : placed) {
        tds_result r{};
        r.q_seg = (uint32_t)p.id;
        r.e_seg = (uint32_t)p.pos;
        r.e_traj = p.pos < cap + scap ? 1u : 0u;
        all[p.id] = r;
        r.e_traj = 0;
        if (p.pos < cap) out[p.pos] = r;
        else if (p.pos - cap < scap) scratch[p.pos - cap] = r;
    }
    std::vector<uint64_t> dlast(W);
    uint64_t holes = 0;
    for (uint32_t w = 0; w < W; ++w) {
        dlast[w] = dend[w] ? ((dend[w] / C - 1) << 16) | (C - (dend[w] - dpos[w])) : ~0ull;
        if (dend[w] && dpos[w] < T) holes += std::min(dend[w], T) - dpos[w];
    }
    write_records((prefix + ".all").c_str(), all, count);
    write_records((prefix + ".before").c_str(), out, T);
    // the pass as the library launches it, on buffers of the sizes it
    // allocates (W + 2, W + 1, W and 4 entries)
    tds::Request req{};
    req.q_count = 1;
    req.out_capacity = cap;
    tds::ReqCounter rc{count, 0};
    unsigned long long R = ctr;
    std::vector<uint64_t> s_pre((size_t)W + 2), d_pre((size_t)W + 1), d_start(W), plan(4);
    hipLaunchKernelGGL(tds::k_fill_plan, dim3(1), dim3(1024), 0, nullptr, &req, &rc, &R,
                       dlast.data(), W, C, s_pre.data(), d_pre.data(), d_start.data(),
                       plan.data());
    hipLaunchKernelGGL(tds::k_fill_copy, dim3(1024), dim3(256), 0, nullptr, plan.data(),
                       s_pre.data(), d_pre.data(), d_start.data(), W, C, &req, out.data(),
                       scratch.data());
    write_records((prefix + ".after").c_str(), out, T);
    printf("%d %llu %llu %llu %llu %llu\n", TDS_OK, (unsigned long long)count,
           (unsigned long long)cap, (unsigned long long)T, (unsigned long long)holes,
           (unsigned long long)R);
    return 0;
}

int run_filtercheck(char** argv) {
    using tds::Box32;
    using tds::QCanon;
    std::mt19937_64 rng(strtoull(argv[2], nullptr, 10));
    const uint64_t n = strtoull(argv[3], nullptr, 10);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::normal_distribution<double> N(0.0, 1.0);
    const double eps_set[] = {0.0, 1e-15, -1e-15, 1e-12, -1e-12, 1e-9, -1e-9, 1e-6, -1e-6};
    uint64_t accepted = 0, misses = 0, naive = 0;
    for (uint64_t k = 0; k < n; ++k) {
        const double S = std::pow(10.0, -3.0 + 12.0 * U(rng));     // length scale
        const double off = std::pow(10.0, -3.0 + 12.0 * U(rng));   // coordinate magnitude
        const double d = S * std::pow(10.0, -3.0 + 4.0 * U(rng));
        double o[3], ve[3], w[3], nv[3];
        for (int a = 0; a < 3; ++a) {
            o[a] = off * (2.0 * U(rng) - 1.0);
            ve[a] = S * N(rng);
            w[a] = (k % 5 == 0) ? 0.0 : S * N(rng);
            nv[a] = N(rng);
        }
        // n perpendicular to w, unit length
        const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
        const double nw = nv[0] * w[0] + nv[1] * w[1] + nv[2] * w[2];
        for (int a = 0; a < 3; ++a) nv[a] -= ww > 0 ? nw / ww * w[a] : 0.0;
        const double nn = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        for (int a = 0; a < 3; ++a) nv[a] /= nn;
        const double ets = 20.0 * U(rng) - 10.0, ete = ets + std::pow(10.0, -2.0 + 3.0 * U(rng));
        const double qts = ets + (ete - ets) * (U(rng) - 0.5);
        const double qte = qts + (ete - ets) * (0.2 + U(rng));
        const double lo = std::max(ets, qts), hi = std::min(ete, qte);
        if (!(lo < hi)) continue;
        const double tau = lo + (hi - lo) * U(rng);
        const double eps = (k % 10 == 9) ? 1e-3 * (2.0 * U(rng) - 1.0) : eps_set[k % 9];
        double e0[3], e1[3], q0[3], q1[3];
        for (int a = 0; a < 3; ++a) {
            e0[a] = o[a];
            e1[a] = o[a] + ve[a] * (ete - ets);
            const double at_tau = o[a] + ve[a] * (tau - ets) + nv[a] * d * (1.0 + eps);
            q0[a] = at_tau + (ve[a] + w[a]) * (qts - tau);
            q1[a] = at_tau + (ve[a] + w[a]) * (qte - tau);
        }
        // canonical data: velocity = displacement / duration, window unbounded
        QCanon q;
        q.x = q0[0];
        q.y = q0[1];
        q.z = q0[2];
        q.vx = (q1[0] - q0[0]) / (qte - qts);
        q.vy = (q1[1] - q0[1]) / (qte - qts);
        q.vz = (q1[2] - q0[2]) / (qte - qts);
        q.ts = qts;
        q.aq = qts;
        q.bq = qte;
        q.d = d;
        const double edt = ete - ets;
        const double evx = (e1[0] - e0[0]) / edt, evy = (e1[1] - e0[1]) / edt,
                     evz = (e1[2] - e0[2]) / edt;
        double t_lo, t_hi;
        if (!tds::canon_eval<false>(q, e0[0], e0[1], e0[2], evx, evy, evz, ets, ete, &t_lo, &t_hi))
            continue;
        ++accepted;
        // the FP32 filter as the kernels build it: entry sphere from the data
        // end points, entry box from the canonical end points, query sphere
        // and box from the clipped end points
        float ecx, ecy, ecz, er;
        tds::sphere32(e0[0], e0[1], e0[2], e1[0], e1[1], e1[2], 0.0, ecx, ecy, ecz, er);
        const Box32 eb = tds::seg_box32(e0[0], e0[1], e0[2], e0[0] + evx * edt, e0[1] + evy * edt,
                                   e0[2] + evz * edt, 0.0);
        const double pa[3] = {q.x + q.vx * (q.aq - q.ts), q.y + q.vy * (q.aq - q.ts),
                              q.z + q.vz * (q.aq - q.ts)};
        const double pb[3] = {q.x + q.vx * (q.bq - q.ts), q.y + q.vy * (q.bq - q.ts),
                              q.z + q.vz * (q.bq - q.ts)};
        float qcx, qcy, qcz, qR;
        tds::sphere32(pa[0], pa[1], pa[2], pb[0], pb[1], pb[2], d, qcx, qcy, qcz, qR);
        const Box32 qb = tds::seg_box32(pa[0], pa[1], pa[2], pb[0], pb[1], pb[2], d);
        const bool time_ok = tds::f32_rd(q.aq) < tds::f32_ru(ete) && tds::f32_rd(ets) < tds::f32_ru(q.bq);
        if (!(tds::sphere_pass(qcx, qcy, qcz, qR, ecx, ecy, ecz, er) && time_ok &&
              tds::box_overlap(eb, qb)))
            ++misses;
        const float df = (float)d;
        const Box32 nb = {(float)std::min(e0[0], e1[0]), (float)std::min(e0[1], e1[1]),
                          (float)std::min(e0[2], e1[2]), (float)std::max(e0[0], e1[0]),
                          (float)std::max(e0[1], e1[1]), (float)std::max(e0[2], e1[2])};
        const Box32 nq = {(float)std::min(pa[0], pb[0]) - df, (float)std::min(pa[1], pb[1]) - df,
                          (float)std::min(pa[2], pb[2]) - df, (float)std::max(pa[0], pb[0]) + df,
                          (float)std::max(pa[1], pb[1]) + df, (float)std::max(pa[2], pb[2]) + df};
        if (!tds::box_overlap(nb, nq)) ++naive;
    }
    printf("%d %llu %llu %llu\n", TDS_OK, (unsigned long long)accepted,
           (unsigned long long)misses, (unsigned long long)naive);
    return 0;
}

int run_cvt(char** argv) {
    const std::vector<char> raw = read_file(argv[2]);
    const size_t n = raw.size() / sizeof(double);
    std::vector<double> x(n);
    if (n) std::memcpy(x.data(), raw.data(), n * sizeof(double));
    std::vector<float> out(2 * n);
    for (size_t i = 0; i < n; ++i) {
        out[2 * i] = tds::f32_rd(x[i]);
        out[2 * i + 1] = tds::f32_ru(x[i]);
    }
    FILE* fo = fopen(argv[3], "wb");
    fwrite(out.data(), sizeof(float), out.size(), fo);
    fclose(fo);
    printf("%d %llu\n", TDS_OK, (unsigned long long)n);
    return 0;
}

int run_merge(char** argv) {
    const std::vector<char> raw = read_file(argv[2]);
    const size_t n = raw.size() / sizeof(tds_result);
    std::vector<tds_result> recs(n);
    if (n) std::memcpy(recs.data(), raw.data(), n * sizeof(tds_result));
    const uint64_t cap = strtoull(argv[3], nullptr, 10);
    std::vector<tds_traj_interval> out(std::max<uint64_t>(cap, 1));
    uint64_t m = 0;
    const int st = tds::merge_impl(recs.data(), n, false, out.data(), cap, false, &m, nullptr);
    FILE* fo = fopen(argv[4], "wb");
    fwrite(out.data(), sizeof(tds_traj_interval), std::min<uint64_t>(m, cap), fo);
    fclose(fo);
    printf("%d %llu\n", st, (unsigned long long)m);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc >= 11 && std::string(argv[1]) == "fsg") return run_fsg(argv);
    if (argc >= 11 && std::string(argv[1]) == "search") return run_search(argc, argv, false);
    if (argc >= 10 && std::string(argv[1]) == "selfjoin") return run_search(argc, argv, true);
    if (argc >= 5 && std::string(argv[1]) == "merge") return run_merge(argv);
    if (argc >= 8 && std::string(argv[1]) == "hostsearch") return run_hostsearch(argv);
    if (argc >= 10 && std::string(argv[1]) == "fill") return run_fill(argv);
    if (argc >= 4 && std::string(argv[1]) == "filtercheck") return run_filtercheck(argv);
    if (argc >= 4 && std::string(argv[1]) == "cvt") return run_cvt(argv);
    fprintf(stderr, "usage: harness fsg ... | harness merge ...\n");
    return 2;
}
