"""Seeded synthetic trajectory workloads.

This module only draws inputs: it holds none of the search arithmetic, so the
oracle and the GPU library can both take their inputs from it without sharing
any code of the method itself.

A trajectory is a polyline of timestamped 3-D points; consecutive points form
the 4-D line segments of the problem definition (Sec. 3.1 of the paper: start
point, end point, segment id = array position, trajectory id).  The workloads
stand in for the paper's datasets (Sec. 5.1, Table "Characteristics of
Datasets"), which are not available:

* ``tiny``      - 3-D random walk, N(0,1) steps, start in [0,100]^3.
* ``uniform1m`` - random walk with per-step velocity U[-5,5]^3, start in
                  [0,1000]^3 (stand-in for Random-1M).
* ``dense``     - random walk in a [0,50]^3 box with reflecting walls
                  (stand-in for Random-dense).
* ``merger``    - test particles of two Plummer spheres on an approaching
                  hyperbolic orbit (stand-in for the Merger dataset).
* ``stream``    - Poisson request stream over the ``uniform1m`` database.

Random numbers come from a counter-based generator: the SplitMix64 output
function (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to ``key + counter * golden_gamma``; normals
by the Box-Muller transform.  Streams are therefore bit-stable across NumPy
versions.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
import os
from typing import Dict, List, Optional, Tuple

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (a bijective 64-bit finaliser)."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


class Rng:
    """Counter-based stream: draw i of stream ``seed`` is mix64(key + i*gamma)."""

    def __init__(self, seed: int):
        self.key = _mix64(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
        self.ctr = 0

    def u64(self, n: int) -> np.ndarray:
        idx = np.arange(self.ctr, self.ctr + n, dtype=np.uint64)
        self.ctr += n
        with np.errstate(over="ignore"):
            return _mix64(self.key + (idx + np.uint64(1)) * _GOLDEN)

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        """Uniform doubles in [lo, hi) with 53 random bits."""
        u = (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u

    def normal(self, n: int) -> np.ndarray:
        m = (n + 1) // 2
        u1 = 1.0 - self.uniform(m)          # (0, 1]
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log(u1))
        z = np.concatenate([r * np.cos(2.0 * np.pi * u2), r * np.sin(2.0 * np.pi * u2)])
        return z[:n]

    def integers(self, n: int, lo: int, hi_inclusive: int) -> np.ndarray:
        span = hi_inclusive - lo + 1
        return lo + np.minimum((self.uniform(n) * span).astype(np.int64), span - 1)


@dataclasses.dataclass
class Segments:
    """Structure-of-arrays 4-D segments; segment id = array position."""

    xs: np.ndarray
    ys: np.ndarray
    zs: np.ndarray
    ts: np.ndarray
    xe: np.ndarray
    ye: np.ndarray
    ze: np.ndarray
    te: np.ndarray
    traj: np.ndarray  # uint32

    def __len__(self) -> int:
        return int(self.xs.shape[0])

    def arrays(self) -> Dict[str, np.ndarray]:
        return {k: getattr(self, k) for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te", "traj")}

    def take(self, idx) -> "Segments":
        return Segments(**{k: np.ascontiguousarray(v[idx]) for k, v in self.arrays().items()})

    def digest(self) -> str:
        h = hashlib.sha256()
        for v in self.arrays().values():
            h.update(np.ascontiguousarray(v).tobytes())
        return h.hexdigest()[:16]


def concat(parts: List[Segments]) -> Segments:
    return Segments(**{k: np.concatenate([getattr(p, k) for p in parts])
                       for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te", "traj")})


def from_points(pos: np.ndarray, times: np.ndarray, traj_ids: Optional[np.ndarray] = None) -> Segments:
    """Polylines -> segments.  ``pos`` is (n_traj, n_pts, 3), ``times`` is (n_pts,)
    or (n_traj, n_pts).  Segments are trajectory-major, time-ordered."""
    n_traj, n_pts, _ = pos.shape
    t = np.broadcast_to(times, (n_traj, n_pts))
    if traj_ids is None:
        traj_ids = np.arange(n_traj, dtype=np.uint32)
    s = pos[:, :-1, :].reshape(-1, 3)
    e = pos[:, 1:, :].reshape(-1, 3)
    return Segments(
        xs=np.ascontiguousarray(s[:, 0]), ys=np.ascontiguousarray(s[:, 1]),
        zs=np.ascontiguousarray(s[:, 2]), ts=np.ascontiguousarray(t[:, :-1].reshape(-1)),
        xe=np.ascontiguousarray(e[:, 0]), ye=np.ascontiguousarray(e[:, 1]),
        ze=np.ascontiguousarray(e[:, 2]), te=np.ascontiguousarray(t[:, 1:].reshape(-1)),
        traj=np.repeat(np.asarray(traj_ids, dtype=np.uint32), n_pts - 1),
    )


# ---------------------------------------------------------------- random walks

def random_walk(n_traj: int, n_pts: int, seed: int, *, box: float, step: str,
                walls: bool = False, t0: float = 0.0, dt: float = 1.0) -> Segments:
    """Random-walk trajectories sampled at times t0 + k*dt, k = 0..n_pts-1.

    ``step`` is ``"normal"`` (N(0,1) per axis) or ``"uniform5"`` (U[-5,5] per
    axis).  Starts are U[0, box]^3.  With ``walls`` a coordinate that leaves
    [0, box] is mirrored about the wall it crossed until it is back inside.
    """
    rng = Rng(seed)
    p = rng.uniform(n_traj * 3, 0.0, box).reshape(n_traj, 3)
    pos = np.empty((n_traj, n_pts, 3), dtype=np.float64)
    pos[:, 0] = p
    for k in range(1, n_pts):
        if step == "normal":
            s = rng.normal(n_traj * 3).reshape(n_traj, 3)
        elif step == "uniform5":
            s = rng.uniform(n_traj * 3, -5.0, 5.0).reshape(n_traj, 3)
        else:
            raise ValueError(step)
        p = p + s
        if walls:
            while True:
                lo = p < 0.0
                hi = p > box
                if not (lo.any() or hi.any()):
                    break
                p = np.where(lo, -p, p)
                p = np.where(hi, 2.0 * box - p, p)
        pos[:, k] = p
    times = t0 + dt * np.arange(n_pts, dtype=np.float64)
    return from_points(pos, times)


# ---------------------------------------------------------------- galaxy merger

@dataclasses.dataclass(frozen=True)
class MergerParams:
    """Frozen physics of the merger-shaped workload (builder's choice).

    Units: G = 1, galaxy mass M = 1, length in kpc.  Each galaxy is a rigid
    Plummer sphere of scale ``a``; its test particles are drawn from the
    Plummer distribution function (Aarseth, Henon & Wielen 1974).  The two
    centres start ``sep0`` apart with impact parameter ``b_imp`` and relative
    speed ``v_fac`` times the parabolic speed, and move as a softened two-body
    orbit; particles feel both softened potentials.  Kick-drift-kick leapfrog
    with step ``dt``; ``n_snap`` snapshots every ``snap_dt``.
    """

    a: float = 1.0
    sep0: float = 6.0
    b_imp: float = 1.0
    v_fac: float = 1.5
    dt: float = 0.005
    snap_dt: float = 0.5
    n_snap: int = 20
    r_max: float = 10.0  # truncation radius of the sampled spheres (in units of a)


def _plummer_particles(rng: Rng, n: int, a: float, r_max: float):
    # radius from the inverted cumulative mass profile, truncated at r_max*a
    m_max = (r_max ** 3) / (1.0 + r_max ** 2) ** 1.5
    x1 = rng.uniform(n) * m_max
    x1 = np.maximum(x1, 1e-12)
    r = a / np.sqrt(x1 ** (-2.0 / 3.0) - 1.0)
    # isotropic direction
    cz = rng.uniform(n, -1.0, 1.0)
    ph = rng.uniform(n, 0.0, 2.0 * np.pi)
    sz = np.sqrt(1.0 - cz * cz)
    pos = r[:, None] * np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)
    # speed: q * v_esc with q drawn from g(q) = q^2 (1-q^2)^(7/2) by rejection
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(todo.size)
        y = rng.uniform(todo.size, 0.0, 0.1)
        ok = y < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (1.0 + (r / a) ** 2) ** (-0.25) / np.sqrt(a)
    v = q * vesc
    cz = rng.uniform(n, -1.0, 1.0)
    ph = rng.uniform(n, 0.0, 2.0 * np.pi)
    sz = np.sqrt(1.0 - cz * cz)
    vel = v[:, None] * np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)
    return pos, vel


def _centre_orbit(P: MergerParams):
    """Positions of the two galaxy centres at every force evaluation of the
    leapfrog (the initial one, then one after each drift): a softened
    two-body orbit, independent of the test particles."""
    v_par = math.sqrt(2.0 * 2.0 / P.sep0)
    v_rel = P.v_fac * v_par
    c = np.array([[-P.sep0 / 2, -P.b_imp / 2, 0.0], [P.sep0 / 2, P.b_imp / 2, 0.0]])
    cv = np.array([[v_rel / 2, 0.0, 0.0], [-v_rel / 2, 0.0, 0.0]])
    a2 = P.a * P.a

    def acc_centres(c):
        d = c[0] - c[1]
        r2 = float(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) + a2
        f = d / (r2 * math.sqrt(r2))
        return np.stack([-f, f])

    steps = int(round(P.snap_dt / P.dt)) * (P.n_snap - 1)
    out = np.empty((steps + 1, 2, 3))
    out[0] = c
    ac = acc_centres(c)
    for k in range(1, steps + 1):
        cv = cv + 0.5 * P.dt * ac
        c = c + P.dt * cv
        ac = acc_centres(c)
        cv = cv + 0.5 * P.dt * ac
        out[k] = c
    return out, cv


def _leapfrog_chunk(x, v, corbit, P: MergerParams):
    """Kick-drift-kick leapfrog of test particles (axis-major arrays x, v of
    shape (3, n), updated in place) in the two softened Plummer potentials
    centred on the precomputed centre orbit.  Only additions,
    multiplications, divisions and square roots, each correctly rounded and
    element by element, so every particle's path is the same whatever the
    chunking or the thread doing it.  Returns the (n, n_snap, 3) snapshots."""
    a2 = P.a * P.a
    hdt = 0.5 * P.dt
    per = int(round(P.snap_dt / P.dt))
    n = x.shape[1]
    snaps = np.empty((n, P.n_snap, 3))
    snaps[:, 0] = x.T

    def acc(c):
        g = np.zeros_like(x)
        for k in range(2):
            d = x - c[k][:, None]
            r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + a2
            g -= d * (1.0 / (r2 * np.sqrt(r2)))
        return g

    ax = acc(corbit[0])
    step = 0
    for s in range(1, P.n_snap):
        for _ in range(per):
            step += 1
            v += hdt * ax
            x += P.dt * v
            ax = acc(corbit[step])
            v += hdt * ax
        snaps[:, s] = x.T
    return snaps


def merger(n_per_galaxy: int, seed: int, params: MergerParams = MergerParams(),
           traj_offset: int = 0, threads: int = 0) -> Segments:
    """Particles of two approaching Plummer spheres; ``n_snap`` snapshots.
    The particles are integrated in chunks on ``threads`` threads (0: up to
    16); the result does not depend on either."""
    P = params
    rng = Rng(seed)
    corbit, _ = _centre_orbit(P)
    v_par = math.sqrt(2.0 * 2.0 / P.sep0)
    v_rel = P.v_fac * v_par
    cv0 = np.array([[v_rel / 2, 0.0, 0.0], [-v_rel / 2, 0.0, 0.0]])
    parts_p, parts_v = [], []
    for g in range(2):
        p, v = _plummer_particles(rng, n_per_galaxy, P.a, P.r_max)
        parts_p.append(p + corbit[0][g])
        parts_v.append(v + cv0[g])
    x = np.ascontiguousarray(np.concatenate(parts_p).T)
    v = np.ascontiguousarray(np.concatenate(parts_v).T)
    n = x.shape[1]
    chunk = 8192
    bounds = [(i, min(n, i + chunk)) for i in range(0, n, chunk)]
    snaps = np.empty((n, P.n_snap, 3))

    def run(b):
        xs = np.ascontiguousarray(x[:, b[0]:b[1]])
        vs = np.ascontiguousarray(v[:, b[0]:b[1]])
        snaps[b[0]:b[1]] = _leapfrog_chunk(xs, vs, corbit, P)

    nth = threads if threads > 0 else min(16, os.cpu_count() or 1)
    if nth > 1 and len(bounds) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=nth) as ex:
            list(ex.map(run, bounds))
    else:
        for b in bounds:
            run(b)
    times = P.snap_dt * np.arange(P.n_snap, dtype=np.float64)
    ids = np.arange(traj_offset, traj_offset + n, dtype=np.uint32)
    return from_points(snaps, times, ids)


# ---------------------------------------------------------------- grazing pairs

GRAZE_EPS = (0.0, 1e-15, -1e-15, 1e-12, -1e-12, 1e-9, -1e-9, 1e-7, -1e-7, 1e-5, -1e-5)


def grazing(n: int, seed: int, d: float, offset: float) -> Tuple[Segments, Segments]:
    """Pairs built to pass at distance d(1 + eps) of each other: entry k and
    query k, eps cycling through GRAZE_EPS, around a common offset (0 or a
    large coordinate magnitude, which stresses rounding margins).  Entry k
    spans [t0, t0 + 1] with a random velocity; query k has the entry's
    velocity plus w (every 7th w = 0: parallel motion) and at time tau is at
    the entry's position there plus n d (1 + eps), n a unit vector
    perpendicular to w, so that the closest approach is at tau (inside the
    entry's span for most pairs, past its end for every 5th, where the
    nearest point is an end point).  Query spans are shifted by up to half a
    unit against their entries.  Pairs are 50 units apart from each other
    (beyond reach at the d used), so only the built pairs are near."""
    rng = Rng(seed)
    k = np.arange(n)
    t0 = rng.integers(n, 0, 9).astype(np.float64)
    base = offset + 50.0 * np.stack([k % 37, (k // 37) % 37, k // 1369], 1).astype(np.float64)
    ve = rng.uniform(3 * n, -3.0, 3.0).reshape(n, 3)
    w = rng.uniform(3 * n, -2.0, 2.0).reshape(n, 3)
    w[k % 7 == 0] = 0.0
    r = rng.normal(3 * n).reshape(n, 3)
    # n perpendicular to w (any unit vector where w = 0)
    ww = np.einsum("ij,ij->i", w, w)
    coef = np.where(ww > 0, np.einsum("ij,ij->i", r, w) / np.where(ww > 0, ww, 1.0), 0.0)
    nv = r - coef[:, None] * w
    nv /= np.linalg.norm(nv, axis=1)[:, None]
    eps = np.array(GRAZE_EPS)[k % len(GRAZE_EPS)]
    tau = t0 + rng.uniform(n, 0.05, 0.95)
    tau = np.where(k % 5 == 4, t0 + 1.0 + rng.uniform(n, 0.0, 0.3), tau)
    sh = rng.uniform(n, -0.5, 0.5)
    qa, qb = t0 + sh, t0 + sh + 1.0
    pe0 = base
    pe1 = base + ve
    # query position at time t: entry position + n d (1 + eps) + w (t - tau)
    def entry_at(t):
        return pe0 + ve * (t - t0)[:, None]
    def query_at(t):
        return entry_at(t) + nv * (d * (1.0 + eps))[:, None] + w * (t - tau)[:, None]
    pq0, pq1 = query_at(qa), query_at(qb)
    traj = k.astype(np.uint32)

    def seg(p0, p1, a, b):
        return Segments(xs=p0[:, 0].copy(), ys=p0[:, 1].copy(), zs=p0[:, 2].copy(), ts=a.copy(),
                        xe=p1[:, 0].copy(), ye=p1[:, 1].copy(), ze=p1[:, 2].copy(), te=b.copy(),
                        traj=traj.copy())
    return seg(pe0, pe1, t0, t0 + 1.0), seg(pq0, pq1, qa, qb)


# ---------------------------------------------------------------- workloads

@dataclasses.dataclass
class Workload:
    name: str
    D: Segments
    Q: Segments
    ds: List[float]
    window: tuple
    q_traj_len: int  # segments per query trajectory (0 = ragged)

    def query_traj_slices(self):
        """(begin, end) segment ranges of each query trajectory in Q."""
        tr = self.Q.traj
        starts = np.flatnonzero(np.r_[True, tr[1:] != tr[:-1]])
        ends = np.r_[starts[1:], len(tr)]
        return list(zip(starts.tolist(), ends.tolist()))


def seeds(k: int):
    """Seeds of config k: database, queries, request stream."""
    return 1000 * k + 1, 1000 * k + 2, 1000 * k + 3


def tiny(scale: float = 1.0) -> Workload:
    """2,000 trajectories x 50 timesteps (98,000 segments), N(0,1) steps from
    U[0,100]^3; 100 query trajectories of the same process; d = 5 on [0,49]."""
    sd, sq, _ = seeds(1)
    nt = max(2, int(2000 * scale))
    nq = max(1, int(100 * scale))
    D = random_walk(nt, 50, sd, box=100.0, step="normal")
    Q = random_walk(nq, 50, sq, box=100.0, step="normal")
    return Workload("tiny", D, Q, [5.0], (0.0, 49.0), 49)


def uniform1m(scale: float = 1.0, n_pts: int = 401) -> Workload:
    """2,500 trajectories x 401 timesteps (1,000,000 segments), start U[0,1000]^3,
    per-step velocity U[-5,5]^3; 500 query trajectories over [0,400];
    d in {1, 5, 25}."""
    sd, sq, _ = seeds(2)
    nt = max(2, int(2500 * scale))
    nq = max(1, int(500 * scale))
    D = random_walk(nt, n_pts, sd, box=1000.0, step="uniform5")
    Q = random_walk(nq, n_pts, sq, box=1000.0, step="uniform5")
    return Workload("uniform1m", D, Q, [1.0, 5.0, 25.0], (0.0, float(n_pts - 1)), n_pts - 1)


def dense(scale: float = 1.0, n_pts: int = 101) -> Workload:
    """10,000 trajectories x 101 timesteps (1,000,000 segments) in [0,50]^3 with
    reflecting walls, N(0,1) steps; 1,000 query trajectories; d = 2."""
    sd, sq, _ = seeds(3)
    nt = max(2, int(10000 * scale))
    nq = max(1, int(1000 * scale))
    D = random_walk(nt, n_pts, sd, box=50.0, step="normal", walls=True)
    Q = random_walk(nq, n_pts, sq, box=50.0, step="normal", walls=True)
    return Workload("dense", D, Q, [2.0], (0.0, float(n_pts - 1)), n_pts - 1)


def galaxy(scale: float = 1.0, params: MergerParams = MergerParams()) -> Workload:
    """2 x 100,000 Plummer particles, 20 snapshots (3.8M segments); 2,000 query
    particles from the same process (separate draws); d = 0.5 kpc."""
    sd, sq, _ = seeds(4)
    npg = max(1, int(100000 * scale))
    nq = max(1, int(1000 * scale))
    D = merger(npg, sd, params)
    Q = merger(nq, sq, params)
    span = params.snap_dt * (params.n_snap - 1)
    return Workload("galaxy", D, Q, [0.5], (0.0, span), params.n_snap - 1)


@dataclasses.dataclass
class Request:
    arrival: float      # seconds since stream start
    Q: Segments         # one query trajectory (contiguous time steps)
    d: float
    t_start: float
    t_end: float


def request_stream(n_requests: int, rate: float = 5000.0, n_pts: int = 401,
                   seed: Optional[int] = None) -> List[Request]:
    """Poisson arrivals (exponential gaps at ``rate``/s) of one query trajectory
    each, drawn from the ``uniform1m`` process: L ~ U{5..400} segments starting
    at integer s ~ U{0..400-L}; window t_start ~ U[s, s+L), t_end ~ U(t_start,
    s+L]; d ~ U[1, 25]."""
    _, _, sr = seeds(5)
    rng = Rng(sr if seed is None else seed)
    max_l = n_pts - 1
    gaps = -np.log(1.0 - rng.uniform(n_requests)) / rate
    arrivals = np.cumsum(gaps)
    lens = rng.integers(n_requests, min(5, max_l), max_l)
    out = []
    for i in range(n_requests):
        L = int(lens[i])
        s = int(rng.integers(1, 0, max_l - L)[0])
        # one query trajectory of the uniform1m process, its own draws
        pts = np.empty((1, L + 1, 3))
        p = rng.uniform(3, 0.0, 1000.0)
        pts[0, 0] = p
        steps = rng.uniform(3 * L, -5.0, 5.0).reshape(L, 3)
        pts[0, 1:] = p + np.cumsum(steps, axis=0)
        times = float(s) + np.arange(L + 1, dtype=np.float64)
        Q = from_points(pts, times, np.array([i], dtype=np.uint32))
        t0 = float(rng.uniform(1, s, s + L)[0])
        u = float(rng.uniform(1)[0])
        t1 = (s + L) - u * ((s + L) - t0)   # in (t0, s+L]
        if not t1 > t0:
            t1 = float(s + L)
        d = float(rng.uniform(1, 1.0, 25.0)[0])
        out.append(Request(float(arrivals[i]), Q, d, t0, t1))
    return out


CONFIGS = {
    "tiny": tiny,
    "uniform1m": uniform1m,
    "dense": dense,
    "galaxy": galaxy,
}
