// Host harness for the CPU emulation of the grid and merge kernels (built by
// tests/test_emulated_kernels.py with g++ and AddressSanitizer against the
// shim in tests/emu/hip).  It builds a tds_index by hand (entries in start
// time order; the grid does not depend on the order) and calls the library's
// grid build / search and trajectory merge, whose kernels then run on the
// host.
//
//   harness fsg D.bin Q.bin gx gy gz d t0 t1 out.bin   -> "status n"
//   harness merge recs.bin capacity out.bin            -> "status n"
//
// D.bin / Q.bin: 9 float64 columns (xs ys zs ts xe ye ze te traj), column
// after column.  recs.bin: tds_result records.  out.bin: the records or
// intervals written.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <numeric>
#include <vector>

#include "tds_internal.hpp"

long emu_launches = 0;

namespace tds {
int fsg_build(const tds_index* idx, uint32_t gx, uint32_t gy, uint32_t gz, hipStream_t s,
              tds_fsg** out);
void fsg_destroy(tds_fsg* f);
int fsg_search(const tds_fsg* f, const tds_segments* Q, double d, double t_start, double t_end,
               tds_result* out, uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
               hipStream_t s, tds_stats* stats);
int merge_impl(const tds_result* recs, uint64_t n, bool recs_dev, tds_traj_interval* out,
               uint64_t capacity, bool out_dev, uint64_t* n_out, hipStream_t s);

// The harness passes valid segment sets only.
int validate_segments_args(const tds_segments* S) {
    return (S && S->xs && S->ys && S->zs && S->ts && S->xe && S->ye && S->ze && S->te)
               ? TDS_OK
               : TDS_E_INVALID;
}
}  // namespace tds

extern "C" void tds_search_params_default(tds_search_params* p) { std::memset(p, 0, sizeof(*p)); }

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

int run_fsg(char** argv) {
    const Columns D = read_columns(argv[2]);
    const Columns Qc = read_columns(argv[3]);
    const uint32_t g[3] = {(uint32_t)atoi(argv[4]), (uint32_t)atoi(argv[5]),
                           (uint32_t)atoi(argv[6])};
    const double d = atof(argv[7]), t0 = atof(argv[8]), t1 = atof(argv[9]);
    const size_t nd = D.n, nq = Qc.n;
    std::vector<uint32_t> ord(nd);
    std::iota(ord.begin(), ord.end(), 0u);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](uint32_t a, uint32_t b) { return D.col(3)[a] < D.col(3)[b]; });
    tds_index idx;
    idx.n = nd;
    std::vector<tds::EntryF64> e64(nd);
    std::vector<uint32_t> seg_id(nd), traj(nd);
    for (size_t p = 0; p < nd; ++p) {
        const uint32_t i = ord[p];
        const double xs = D.col(0)[i], ys = D.col(1)[i], zs = D.col(2)[i], ts = D.col(3)[i];
        const double xe = D.col(4)[i], ye = D.col(5)[i], ze = D.col(6)[i], te = D.col(7)[i];
        const double dt = te - ts;
        e64[p] = tds::EntryF64{xs, ys, zs, (xe - xs) / dt, (ye - ys) / dt, (ze - zs) / dt, ts, te};
        seg_id[p] = i;
        traj[p] = (uint32_t)D.col(8)[i];
    }
    idx.e64 = e64.data();
    idx.seg_id = seg_id.data();
    idx.traj = traj.data();
    tds_fsg* f = nullptr;
    int st = tds::fsg_build(&idx, g[0], g[1], g[2], nullptr, &f);
    if (st != TDS_OK) {
        printf("%d 0\n", st);
        return 0;
    }
    std::vector<uint32_t> qtraj(nq);
    for (size_t i = 0; i < nq; ++i) qtraj[i] = (uint32_t)Qc.col(8)[i];
    tds_segments Q{};
    Q.xs = Qc.col(0);
    Q.ys = Qc.col(1);
    Q.zs = Qc.col(2);
    Q.ts = Qc.col(3);
    Q.xe = Qc.col(4);
    Q.ye = Qc.col(5);
    Q.ze = Qc.col(6);
    Q.te = Qc.col(7);
    Q.traj_id = qtraj.data();
    Q.n = nq;
    Q.on_device = 0;
    std::vector<tds_result> out(1u << 20);
    uint64_t n = 0;
    st = tds::fsg_search(f, &Q, d, t0, t1, out.data(), out.size(), &n, nullptr, nullptr, nullptr);
    FILE* fo = fopen(argv[10], "wb");
    fwrite(out.data(), sizeof(tds_result), std::min<uint64_t>(n, out.size()), fo);
    fclose(fo);
    tds::fsg_destroy(f);
    printf("%d %llu\n", st, (unsigned long long)n);
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
    if (argc >= 5 && std::string(argv[1]) == "merge") return run_merge(argv);
    fprintf(stderr, "usage: harness fsg ... | harness merge ...\n");
    return 2;
}
