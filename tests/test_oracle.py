"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's own formula: closed-form cases are
worked out by hand, membership is re-derived in exact rational arithmetic by
evaluating the quadratic at its clamped vertex (not by the oracle's
discriminant test), endpoints come from 50-digit decimal roots, positions for
the sampling test come from interpolating the end points (not from the
velocity form), and the temporal bins come from the paper's printed example.
"""
import decimal
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import trajgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def seg(ps, pe, ts, te):
    return oracle.seg_record(ps[0], ps[1], ps[2], ts, pe[0], pe[1], pe[2], te)


# ------------------------------------------------------------------ closed forms

def test_velocity_closed_form():
    r = seg((1, 2, 3), (5, -2, 3), 2.0, 4.0)
    assert list(r[3:6]) == [2.0, -2.0, 0.0]


def test_comoving_parallel_exact_contact():
    # q and l both move +1/unit in x, 5 apart in (y, z) = (3, 4): A = 0
    q = seg((0, 0, 0), (10, 0, 0), 0.0, 10.0)
    l = seg((0, 3, 4), (10, 3, 4), 0.0, 10.0)
    assert oracle.pair(q, l, 5.0) == (0.0, 10.0)
    assert oracle.pair(q, l, 4.999) is None


def test_head_on_crossing():
    # relative speed 4, closest approach 3 at t = 5: 5 -+ sqrt(25 - 9) / 4
    q = seg((-10, 0, 0), (10, 0, 0), 0.0, 10.0)
    l = seg((10, 3, 0), (-10, 3, 0), 0.0, 10.0)
    assert oracle.pair(q, l, 5.0) == (4.0, 6.0)
    assert oracle.pair(q, l, 2.999) is None
    assert oracle.pair(q, l, 3.0) == (5.0, 5.0)


def test_tangent_at_d():
    q = seg((-1, 5, 0), (1, 5, 0), 0.0, 2.0)
    l = seg((0, 0, 0), (0, 0, 0), 0.0, 2.0)
    assert oracle.pair(q, l, 5.0) == (1.0, 1.0)
    assert oracle.pair(q, l, 4.9999999) is None


def test_partial_time_overlap():
    q = seg((0, 0, 0), (10, 0, 0), 0.0, 10.0)
    l = seg((5, 1, 0), (15, 1, 0), 5.0, 15.0)
    assert oracle.pair(q, l, 2.0) == (5.0, 10.0)


def test_touch_only_is_not_a_result():
    q = seg((0, 0, 0), (0, 0, 0), 0.0, 1.0)
    l = seg((0, 0, 0), (0, 0, 0), 1.0, 2.0)
    assert oracle.pair(q, l, 100.0) is None


def test_window_clip():
    q = seg((-10, 0, 0), (10, 0, 0), 0.0, 10.0)
    l = seg((10, 3, 0), (-10, 3, 0), 0.0, 10.0)
    assert oracle.pair(q, l, 5.0, 4.5, 5.5) == (4.5, 5.5)
    assert oracle.pair(q, l, 5.0, 6.5, 9.0) is None
    # window that only touches the segments' common extent
    assert oracle.pair(q, l, 5.0, 10.0, 11.0) is None


def test_stationary_point_query_matches_point_line_distance():
    """The supernova query of Sec. 2.1: a non-moving point over a time interval.
    The closest approach of a moving point to it is the textbook point-to-line
    distance |(p - x0) x v| / |v| at time (p - x0).v / |v|^2."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        p = rng.uniform(-5, 5, 3)
        x0 = rng.uniform(-5, 5, 3)
        v = rng.uniform(-2, 2, 3)
        T = 10.0
        tstar = float(np.dot(p - x0, v) / np.dot(v, v))
        if not (0.5 < tstar < T - 0.5):
            continue
        dmin = float(np.linalg.norm(np.cross(p - x0, v)) / np.linalg.norm(v))
        q = seg(p, p, 0.0, T)
        l = seg(x0, x0 + v * T, 0.0, T)
        assert oracle.pair(q, l, dmin * (1 - 1e-7)) is None
        d = dmin + 0.3
        half = math.sqrt(d * d - dmin * dmin) / float(np.linalg.norm(v))
        r = oracle.pair(q, l, d)
        assert r is not None
        lo_ex = max(0.0, tstar - half)
        hi_ex = min(T, tstar + half)
        assert abs(r[0] - lo_ex) <= 1e-9 * max(1, abs(lo_ex))
        assert abs(r[1] - hi_ex) <= 1e-9 * max(1, abs(hi_ex))


# ------------------------------------------------------- exact rational arithmetic

def _exact_pair(qs, qe, qts, qte, ls, le, lts, lte, d, t0=None, t1=None):
    """Exact membership and the exact minimum of the squared distance, from the
    positions interpolated between end points (rationals)."""
    a = max(qts, lts) if t0 is None else max(qts, lts, t0)
    b = min(qte, lte) if t1 is None else min(qte, lte, t1)
    if not a < b:
        return None

    def pos(s, e, ts_, te_, t):
        return [s[c] + (e[c] - s[c]) * (t - ts_) / (te_ - ts_) for c in range(3)]

    def f(t):
        pq, pl = pos(qs, qe, qts, qte, t), pos(ls, le, lts, lte, t)
        return sum((pq[c] - pl[c]) ** 2 for c in range(3))

    # f is a convex quadratic in t: recover its coefficients from 3 samples
    fa, fm, fb = f(a), f((a + b) / 2), f(b)
    T = b - a
    # f(a + tau) = c0 + c1 tau + c2 tau^2
    c0 = fa
    c2 = 2 * (fb - 2 * fm + fa) / (T * T)
    c1 = (fb - fa) / T - c2 * T
    if c2 > 0:
        tau = min(max(-c1 / (2 * c2), Fraction(0)), T)
    else:
        tau = Fraction(0) if c1 >= 0 else T
    fmin = c0 + c1 * tau + c2 * tau * tau
    return dict(a=a, b=b, c0=c0, c1=c1, c2=c2, fmin=fmin, member=fmin <= d * d, T=T)


def _dyadic(rng, lo, hi, den):
    return Fraction(int(rng.integers(lo * den, hi * den + 1)), den)


def test_membership_matches_exact_rationals():
    """Random pairs with small dyadic coordinates and power-of-two durations;
    integer d so that exact ties at d occur.  Every oracle decision must equal
    the exact one."""
    rng = np.random.default_rng(1234)
    n_member = n_tie = 0
    for _ in range(6000):
        qts = _dyadic(rng, 0, 4, 4)
        lts = _dyadic(rng, 0, 4, 4)
        qte = qts + Fraction(2) ** int(rng.integers(-2, 3))
        lte = lts + Fraction(2) ** int(rng.integers(-2, 3))
        den = 2
        if rng.integers(0, 2):
            # aligned pairs with integer coordinates: exact ties with integer d
            lts, lte, den = qts, qte, 1
        qs = [_dyadic(rng, -4, 4, den) for _ in range(3)]
        qe = [_dyadic(rng, -4, 4, den) for _ in range(3)]
        ls = [_dyadic(rng, -4, 4, den) for _ in range(3)]
        le = [_dyadic(rng, -4, 4, den) for _ in range(3)]
        d = Fraction(int(rng.integers(0, 6)))
        ex = _exact_pair(qs, qe, qts, qte, ls, le, lts, lte, d)
        q = seg([float(x) for x in qs], [float(x) for x in qe], float(qts), float(qte))
        l = seg([float(x) for x in ls], [float(x) for x in le], float(lts), float(lte))
        got = oracle.pair(q, l, float(d))
        if ex is None:
            assert got is None
            continue
        assert (got is not None) == ex["member"], (qs, qe, qts, qte, ls, le, lts, lte, d, ex, got)
        n_member += ex["member"]
        fb = ex["c0"] + ex["c1"] * ex["T"] + ex["c2"] * ex["T"] ** 2
        n_tie += (ex["fmin"] == d * d) or (ex["c0"] == d * d) or (fb == d * d)
        if got is not None:
            _check_endpoints(ex, d, got)
    assert n_member > 200 and n_tie > 20


def test_tangent_cases_from_pythagorean_triples():
    """Closest approach exactly d at an interior time (B*B - A*C0 = 0 exactly):
    the query passes a stationary entry at distance d = hypotenuse."""
    rng = np.random.default_rng(99)
    for _ in range(300):
        p, q_, h = [(3, 4, 5), (5, 12, 13), (8, 15, 17), (7, 24, 25)][int(rng.integers(0, 4))]
        off = np.array([int(v) for v in rng.integers(-20, 21, 3)], dtype=float)
        k = float(rng.integers(1, 9))
        t0 = float(rng.integers(0, 50))
        axes = rng.permutation(3)
        s = np.zeros(3); e = np.zeros(3)
        s[axes[0]], e[axes[0]] = -k, k
        s[axes[1]] = e[axes[1]] = p
        s[axes[2]] = e[axes[2]] = q_
        q = seg(s + off, e + off, t0, t0 + 2.0)
        l = seg(off, off, t0 - 1.0, t0 + 3.0)
        assert oracle.pair(q, l, float(h)) == (t0 + 1.0, t0 + 1.0)
        assert oracle.pair(q, l, float(h) * (1 - 1e-12)) is None


def _check_endpoints(ex, d, got):
    """Exact endpoints: where f - d^2 changes sign, from 50-digit roots."""
    decimal.getcontext().prec = 50
    D = decimal.Decimal
    a, b, T = ex["a"], ex["b"], ex["T"]
    c0, c1, c2 = ex["c0"] - d * d, ex["c1"], ex["c2"]

    def dec(x):
        return D(x.numerator) / D(x.denominator)

    if c0 <= 0:
        lo = dec(a)
    else:
        disc = dec(c1) ** 2 - 4 * dec(c2) * dec(c0)
        lo = dec(a) + max(D(0), min(dec(T), (-dec(c1) - max(disc, D(0)).sqrt()) / (2 * dec(c2))))
    if c0 + c1 * T + c2 * T * T <= 0:
        hi = dec(b)
    else:
        disc = dec(c1) ** 2 - 4 * dec(c2) * dec(c0)
        hi = dec(a) + max(D(0), min(dec(T), (-dec(c1) + max(disc, D(0)).sqrt()) / (2 * dec(c2))))
    for g, e in ((got[0], lo), (got[1], hi)):
        assert abs(D(g) - e) <= D("1e-9") * max(D(1), abs(e)), (got, lo, hi)


# ------------------------------------------------------------ invariants

def test_swap_symmetry_bitwise():
    """Swapping the roles of query and entry gives the same pairs with bitwise
    identical intervals (the distance is symmetric)."""
    w = trajgen.tiny(scale=0.02)
    Dn = w.D.take(np.arange(0, len(w.D), 3))
    r1 = oracle.search(w.Q, Dn, 30.0, 0.0, 49.0)
    r2 = oracle.search(Dn, w.Q, 30.0, 0.0, 49.0)
    assert len(r1) > 50
    sw = r2.copy()
    sw["q_seg"], sw["e_seg"] = r2["e_seg"], r2["q_seg"]
    sw["q_traj"], sw["e_traj"] = r2["e_traj"], r2["q_traj"]
    sw = oracle.sort_results(sw)
    assert np.array_equal(r1, sw)


def _interp(S, i, t):
    f = (t - S.ts[i]) / (S.te[i] - S.ts[i])
    return np.stack([S.xs[i] + f * (S.xe[i] - S.xs[i]), S.ys[i] + f * (S.ye[i] - S.ys[i]),
                     S.zs[i] + f * (S.ze[i] - S.zs[i])], axis=-1)


def test_dense_time_sampling():
    """Sample each time-overlapping pair densely: samples clearly inside d lie in
    the reported interval, samples clearly outside lie outside it, and pairs
    with no record have no sample clearly inside."""
    w = trajgen.dense(scale=0.004, n_pts=12)
    Q, D = w.Q, w.D
    d = 15.0
    res = oracle.search(Q, D, d, 0.0, 11.0)
    got = {(int(r["q_seg"]), int(r["e_seg"])): (r["t_lo"], r["t_hi"]) for r in res}
    assert len(got) > 100
    checked = 0
    for k in range(len(Q)):
        for i in range(len(D)):
            a = max(Q.ts[k], D.ts[i], 0.0)
            b = min(Q.te[k], D.te[i], 11.0)
            if not a < b:
                assert (k, i) not in got
                continue
            t = np.linspace(a, b, 400)
            dist = np.linalg.norm(_interp(Q, k, t) - _interp(D, i, t), axis=1)
            inside = dist < d * (1 - 1e-9)
            outside = dist > d * (1 + 1e-9)
            if (k, i) in got:
                lo, hi = got[(k, i)]
                tol = 1e-9 * max(1.0, abs(b))
                assert np.all((t[inside] >= lo - tol) & (t[inside] <= hi + tol))
                assert not np.any((t[outside] > lo + tol) & (t[outside] < hi - tol))
            else:
                assert not inside.any()
            checked += 1
    assert checked > 1000


def test_records_carry_ids_and_no_duplicates():
    w = trajgen.tiny(scale=0.02)
    r = oracle.search(w.Q, w.D, 8.0, 0.0, 49.0)
    key = r["q_seg"].astype(np.uint64) << np.uint64(32) | r["e_seg"]
    assert np.unique(key).size == key.size
    assert np.array_equal(r["q_traj"], w.Q.traj[r["q_seg"]])
    assert np.array_equal(r["e_traj"], w.D.traj[r["e_seg"]])
    assert np.all(r["t_lo"] <= r["t_hi"])


# ------------------------------------------------------------ temporal bins

def _load_example():
    segs, bins_ = [], []
    with open(os.path.join(GOLDEN, "example_index.txt")) as f:
        for line in f:
            if line.startswith("segment"):
                _, i, a, b = line.split()
                segs.append((int(i), float(a), float(b)))
            elif line.startswith("bin"):
                _, j, bs, be, bf, bl = line.split()
                bins_.append((int(j), float(bs), float(be), int(bf), int(bl)))
    return segs, bins_


def test_temporal_bins_reproduce_paper_example():
    segs, printed = _load_example()
    ts = np.array([s[1] for s in segs])
    te = np.array([s[2] for s in segs])
    # shuffle the input so that the sort by t_start is exercised
    perm = np.random.default_rng(0).permutation(len(ts))
    tb = oracle.bins(ts[perm], te[perm], 4)
    # sorted order renumbers the entries as in the figure
    assert np.array_equal(perm[tb["order"]], np.arange(15))
    for j, bs, be, bf, bl in printed:
        assert tb["bstart"][j] == bs
        assert tb["bend"][j] == be
        assert tb["first"][j] == bf
        assert tb["last"][j] == bl


def test_schedule_paper_example_noncontiguous_overlap():
    """A query on [7, 7.2] overlaps bins B0 (end 7.5) and B2 but not B1 (end
    6.2); the candidate span E_k runs from B0^first = 0 to B2^last = 11 and
    covers every overlapping entry."""
    segs, _ = _load_example()
    ts = np.array([s[1] for s in segs])
    te = np.array([s[2] for s in segs])
    lo, hi = oracle.schedule(ts, te, 4, np.array([7.0]), np.array([7.2]))
    assert (lo[0], hi[0]) == (0, 12)
    # a query inside B1's extent only: [B0^first, B1^last] (B0 reaches 7.5)
    lo, hi = oracle.schedule(ts, te, 4, np.array([4.0]), np.array([4.5]))
    assert (lo[0], hi[0]) == (0, 9)
    # before every entry's end: nothing; after the last start: only B3
    lo, hi = oracle.schedule(ts, te, 4, np.array([11.95]), np.array([12.5]))
    assert (lo[0], hi[0]) == (12, 15)
    overl = [i for i in range(15) if max(ts[i], 7.0) < min(te[i], 7.2)]
    assert overl == [4, 9, 10]


def test_schedule_is_superset_of_time_overlap():
    rng = np.random.default_rng(7)
    for m in (1, 3, 17):
        n = 300
        ts = np.round(rng.uniform(0, 50, n), 1)
        te = ts + np.round(rng.uniform(0.1, 6, n), 1)
        qts = np.round(rng.uniform(-5, 55, 200), 2)
        qte = qts + rng.uniform(0.01, 5, 200)
        t0, t1 = 3.0, 47.5
        tb = oracle.bins(ts, te, m)
        lo, hi = oracle.schedule(ts, te, m, qts, qte, t0, t1, tables=tb)
        pos = np.empty(n, np.int64)
        pos[tb["order"]] = np.arange(n)
        for k in range(200):
            a, b = max(qts[k], t0), min(qte[k], t1)
            ov = np.flatnonzero(np.maximum(a, ts) < np.minimum(b, te))
            if not a < b:
                assert ov.size == 0 and lo[k] == hi[k] == 0
                continue
            assert np.all((pos[ov] >= lo[k]) & (pos[ov] < hi[k]))


def test_bin_end_is_at_least_the_nominal_bin_end():
    """B^end = max((j+1) b, max te): a bin whose entries all end early still
    extends to its nominal end (hand-computed: m = 2 over [0, 4], b = 2)."""
    ts = np.array([0.0, 2.5, 0.5])
    te = np.array([1.0, 4.0, 1.5])
    tb = oracle.bins(ts, te, 2)
    assert list(tb["bstart"]) == [0.0, 2.0]
    assert list(tb["bend"]) == [2.0, 4.0]
    assert list(tb["first"]) == [0, 2] and list(tb["last"]) == [1, 2]
    assert list(perm for perm in tb["order"]) == [0, 2, 1]


def test_schedule_is_exact_on_aligned_unit_steps():
    """Unit-step trajectories binned at the step width: a query segment [k, k+1]
    strictly overlaps exactly the entries with t_start = k, and the schedule is
    exactly that run (segments of bin k-1 end at k, which only touches)."""
    w = trajgen.tiny(scale=0.01)
    D = w.D
    m = 49
    tb = oracle.bins(D.ts, D.te, m)
    sorted_ts = D.ts[tb["order"]]
    qts = np.arange(0.0, 49.0)
    lo, hi = oracle.schedule(D.ts, D.te, m, qts, qts + 1.0, tables=tb)
    for k in range(49):
        run = np.flatnonzero(sorted_ts == k)
        assert (lo[k], hi[k]) == (run[0], run[-1] + 1)
    # a window ending inside a bin keeps that whole bin (bin granularity)
    lo, hi = oracle.schedule(D.ts, D.te, m, np.array([3.0]), np.array([4.0]), 0.0, 3.5, tables=tb)
    run = np.flatnonzero(sorted_ts == 3)
    assert (lo[0], hi[0]) == (run[0], run[-1] + 1)


# ---------------------------------------------------------------- trajectory level

def _recs(rows):
    """Records from (q_traj, e_traj, t_lo, t_hi) rows (segment ids = row index)."""
    a = np.zeros(len(rows), oracle.RESULT_DTYPE)
    for i, (qt, et, lo, hi) in enumerate(rows):
        a[i] = (i, 1000 + i, qt, et, lo, hi)
    return a


def test_merge_hand_example():
    """Touching and overlapping intervals of one trajectory pair merge, a gap
    separates, pairs stay apart, and the output is in (pair, t_lo) order."""
    rows = [(1, 2, 2.9, 4.0), (1, 2, 1.0, 2.0), (2, 1, 0.0, 1.0), (1, 2, 0.0, 1.0),
            (1, 2, 5.0, 5.0), (1, 2, 2.5, 3.0), (1, 3, 7.0, 8.0), (1, 2, 3.5, 3.75)]
    got = oracle.merge_trajectories(_recs(rows))
    want = [(1, 2, 0.0, 2.0), (1, 2, 2.5, 4.0), (1, 2, 5.0, 5.0), (1, 3, 7.0, 8.0),
            (2, 1, 0.0, 1.0)]
    assert [tuple(r) for r in got.tolist()] == want


def test_merge_preserves_the_union():
    """Random interval sets: the merged intervals are disjoint, separated by
    gaps, have endpoints taken from the input, and cover exactly the points
    the input intervals cover (checked at every endpoint and midpoint)."""
    rng = np.random.default_rng(5)
    rows = []
    for _ in range(400):
        qt, et = int(rng.integers(0, 4)), int(rng.integers(0, 4))
        lo = float(rng.integers(0, 60)) / 4.0
        rows.append((qt, et, lo, lo + float(rng.integers(0, 8)) / 4.0))
    recs = _recs(rows)
    got = oracle.merge_trajectories(recs)
    for (qt, et) in {(r[0], r[1]) for r in rows}:
        ins = [(lo, hi) for a, b, lo, hi in rows if (a, b) == (qt, et)]
        outs = [(r["t_lo"], r["t_hi"]) for r in got if (r["q_traj"], r["e_traj"]) == (qt, et)]
        assert all(outs[i][1] < outs[i + 1][0] for i in range(len(outs) - 1))
        ends = {x for iv in ins for x in iv}
        assert all(lo in ends and hi in ends for lo, hi in outs)
        probes = sorted(ends | {(a + b) / 2 for a, b in ins} | {x + 0.125 for x in ends})
        for t in probes:
            assert any(lo <= t <= hi for lo, hi in ins) == any(lo <= t <= hi for lo, hi in outs)


def test_self_join_is_the_symmetric_half_of_the_full_search():
    """Searching D against itself finds every cross-trajectory pair twice with
    bitwise identical intervals; the self-join keeps one of each."""
    w = trajgen.tiny(scale=0.05)
    full = oracle.search(w.D, w.D, 6.0, 3.0, 30.0)
    cross = full[full["q_traj"] != full["e_traj"]]
    fwd = {(int(r["q_seg"]), int(r["e_seg"])): (r["t_lo"], r["t_hi"]) for r in cross}
    for (a, b), iv in fwd.items():
        assert fwd[(b, a)] == iv
    sj = oracle.self_join(w.D, 6.0, 3.0, 30.0)
    assert sj.size * 2 == cross.size > 50
    assert np.all(sj["q_seg"] < sj["e_seg"]) and np.all(sj["q_traj"] != sj["e_traj"])
