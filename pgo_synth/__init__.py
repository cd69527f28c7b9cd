"""Seeded synthetic pose graphs: the inputs that both the CPU oracle and the
HIP library are fed.

This module only builds inputs. It holds none of the solver's arithmetic:
no quaternion algebra, no cost, no update rule. Everything it produces is
plain rotation matrices and vectors in float64.

Measurement model (the paper's generative model, Model section, with the
isotropic so(3)-Gaussian rotation noise used in place of the von Mises-Fisher
draw, whose concentration parameter is garbled in the experiments section):

    R~_ij = R_i^T R_j Exp(eps),            eps ~ N(0, sigma_R^2 I_3)
    t~_ij = R_i^T (t_j - t_i) + eta,       eta ~ N(0, sigma_t^2 I_3)
    kappa_ij = 1/sigma_R^2,  tau_ij = 1/sigma_t^2

Draw order inside one graph: topology choices, then the (m,3) rotation
noise, then the (m,3) translation noise.  The first n-1 edges are always the
odometry chain (k -> k+1); the initial guess is the noisy odometry composed
from the ground-truth pose 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Graph", "Batch", "so3_exp", "heading_frames",
    "circle", "grid", "sphere", "tree", "random_small", "make_config",
    "batched", "boustrophedon", "grid_pairs", "cube_expected_edges",
    "CONFIGS",
]


@dataclass
class Graph:
    n: int
    ei: np.ndarray            # (m,) int32 tails
    ej: np.ndarray            # (m,) int32 heads
    Rm: np.ndarray            # (m,3,3) measured relative rotations
    tm: np.ndarray            # (m,3)   measured relative translations
    kappa: np.ndarray         # (m,)    rotation precisions
    tau: np.ndarray           # (m,)    translation precisions
    R0: np.ndarray            # (n,3,3) initial rotations
    t0: np.ndarray            # (n,3)   initial translations
    R_gt: np.ndarray          # (n,3,3) ground truth
    t_gt: np.ndarray          # (n,3)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.ei.shape[0])


@dataclass
class Batch:
    graphs: list

    @property
    def G(self) -> int:
        return len(self.graphs)

    def offsets(self):
        voff = np.zeros(self.G + 1, np.int64)
        eoff = np.zeros(self.G + 1, np.int64)
        for g, gr in enumerate(self.graphs):
            voff[g + 1] = voff[g] + gr.n
            eoff[g + 1] = eoff[g] + gr.m
        return voff, eoff

    def concat(self):
        """Graph-local indices, arrays concatenated in graph order."""
        cat = lambda name: np.concatenate([getattr(g, name) for g in self.graphs])
        return dict(ei=cat("ei"), ej=cat("ej"), Rm=cat("Rm"), tm=cat("tm"),
                    kappa=cat("kappa"), tau=cat("tau"), R0=cat("R0"), t0=cat("t0"),
                    R_gt=cat("R_gt"), t_gt=cat("t_gt"))


# ----------------------------------------------------------------------------
# rotations (input construction only)
# ----------------------------------------------------------------------------
def so3_exp(w: np.ndarray) -> np.ndarray:
    """Rodrigues' formula for a batch of axis-angle vectors (k,3) -> (k,3,3)."""
    w = np.asarray(w, np.float64).reshape(-1, 3)
    th = np.linalg.norm(w, axis=1)
    K = np.zeros((w.shape[0], 3, 3))
    K[:, 0, 1], K[:, 0, 2] = -w[:, 2], w[:, 1]
    K[:, 1, 0], K[:, 1, 2] = w[:, 2], -w[:, 0]
    K[:, 2, 0], K[:, 2, 1] = -w[:, 1], w[:, 0]
    small = th < 1e-8
    a = np.where(small, 1.0 - th**2 / 6.0, np.sin(th) / np.where(small, 1.0, th))
    b = np.where(small, 0.5 - th**2 / 24.0, (1.0 - np.cos(th)) / np.where(small, 1.0, th**2))
    return np.eye(3)[None] + a[:, None, None] * K + b[:, None, None] * (K @ K)


def heading_frames(pos: np.ndarray) -> np.ndarray:
    """Orientation rule for trajectories: the body x axis points along the
    step to the next pose (the last pose reuses the previous step); y is
    horizontal, z completes a right-handed frame."""
    pos = np.asarray(pos, np.float64)
    n = pos.shape[0]
    d = np.zeros_like(pos)
    if n > 1:
        d[:-1] = pos[1:] - pos[:-1]
        d[-1] = d[-2]
    else:
        d[:] = (1.0, 0.0, 0.0)
    x = d / np.linalg.norm(d, axis=1, keepdims=True)
    up = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    par = np.abs(x[:, 2]) > 0.9
    up[par] = (0.0, 1.0, 0.0)
    y = np.cross(up, x)
    y /= np.linalg.norm(y, axis=1, keepdims=True)
    z = np.cross(x, y)
    return np.stack([x, y, z], axis=2)  # columns


def _prefix_products(M: np.ndarray) -> np.ndarray:
    """P_k = M_0 M_1 ... M_k for a stack (k,3,3), by a log-depth scan."""
    P = M.copy()
    d = 1
    while d < P.shape[0]:
        P[d:] = P[:-d] @ P[d:]
        d *= 2
    return P


def odometry_init(R_first, t_first, Rm_odo, tm_odo):
    """Compose the odometry measurements (k -> k+1) from pose 0."""
    n = Rm_odo.shape[0] + 1
    R0 = np.empty((n, 3, 3))
    t0 = np.empty((n, 3))
    R0[0], t0[0] = R_first, t_first
    if n > 1:
        P = _prefix_products(Rm_odo)                # Rm_0 ... Rm_k
        R0[1:] = R_first[None] @ P
        step = np.einsum("kab,kb->ka", R0[:-1], tm_odo)
        t0[1:] = t_first[None] + np.cumsum(step, axis=0)
    return R0, t0


def _measure(R_gt, t_gt, ei, ej, sigma_R, sigma_t, rng, init="odometry", name="", meta=None):
    n, m = R_gt.shape[0], ei.shape[0]
    sigma_R = np.broadcast_to(np.asarray(sigma_R, np.float64), (m,))
    sigma_t = np.broadcast_to(np.asarray(sigma_t, np.float64), (m,))
    eps = rng.standard_normal((m, 3)) * sigma_R[:, None]
    eta = rng.standard_normal((m, 3)) * sigma_t[:, None]
    Ri, Rj = R_gt[ei], R_gt[ej]
    Rrel = np.transpose(Ri, (0, 2, 1)) @ Rj
    Rm = Rrel @ so3_exp(eps)
    tm = np.einsum("kba,kb->ka", Ri, t_gt[ej] - t_gt[ei]) + eta
    with np.errstate(divide="ignore"):
        kappa = np.where(sigma_R > 0, 1.0 / np.maximum(sigma_R, 1e-300) ** 2, 1e4)
        tau = np.where(sigma_t > 0, 1.0 / np.maximum(sigma_t, 1e-300) ** 2, 1e4)
    if init == "odometry":
        odo = (ei[: n - 1] == np.arange(n - 1)) & (ej[: n - 1] == np.arange(1, n))
        assert odo.all(), "the first n-1 edges must be the odometry chain"
        R0, t0 = odometry_init(R_gt[0], t_gt[0], Rm[: n - 1], tm[: n - 1])
    elif init == "gt":
        R0, t0 = R_gt.copy(), t_gt.copy()
    else:
        raise ValueError(init)
    return Graph(n=n, ei=ei.astype(np.int32), ej=ej.astype(np.int32), Rm=Rm, tm=tm,
                 kappa=kappa.astype(np.float64), tau=tau.astype(np.float64),
                 R0=R0, t0=t0, R_gt=R_gt, t_gt=t_gt, name=name, meta=meta or {})


# ----------------------------------------------------------------------------
# topologies
# ----------------------------------------------------------------------------
def boustrophedon(nx, ny, nz, n=None):
    """Snake order through an nx*ny*nz box; consecutive cells are neighbours.
    Returns integer coordinates (n,3); the last layer is truncated to n."""
    pts = []
    row = 0
    for z in range(nz):
        ys = range(ny) if z % 2 == 0 else range(ny - 1, -1, -1)
        for y in ys:
            xs = range(nx) if row % 2 == 0 else range(nx - 1, -1, -1)
            pts.extend((x, y, z) for x in xs)
            row += 1
    pts = np.asarray(pts, np.int64)
    return pts if n is None else pts[:n]


def _unique_pairs(lo, hi, n):
    """Distinct unordered pairs given as (lo, hi) arrays, sorted by (lo, hi)."""
    key = np.unique(lo.astype(np.int64) * n + hi.astype(np.int64))
    pairs = np.stack([key // n, key % n], 1)
    return pairs[pairs[:, 0] != pairs[:, 1]]


def grid_pairs(coords, offsets):
    """Unordered pairs (a<b in traversal order) of cells that differ by one of
    the given offsets."""
    coords = np.asarray(coords, np.int64)
    n = coords.shape[0]
    lo = coords.min(0) - 2
    span = coords.max(0) - lo + 3
    key = lambda c: ((c[:, 0] - lo[0]) * span[1] + (c[:, 1] - lo[1])) * span[2] + (c[:, 2] - lo[2])
    table = np.full(int(span.prod()), -1, np.int64)
    table[key(coords)] = np.arange(n)
    A, B = [], []
    for off in offsets:
        b = table[key(coords + np.asarray(off, np.int64))]
        a = np.nonzero(b >= 0)[0]
        A.append(a)
        B.append(b[a])
    a, b = np.concatenate(A), np.concatenate(B)
    return _unique_pairs(np.minimum(a, b), np.maximum(a, b), n)


_NB6 = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
_HOP2 = [(2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1),
         (0, 1, 1), (0, 1, -1)]


def _odometry(n):
    k = np.arange(n - 1)
    return k, k + 1


def _drop_odometry(pairs):
    return pairs[pairs[:, 1] - pairs[:, 0] != 1]


def circle(n=100, radius=10.0, n_closures=20, min_sep=10, sigma_R=0.01, sigma_t=0.01,
           seed=0, init="odometry", rng=None):
    """Poses on a horizontal circle, odometry chain plus closures between
    pairs whose cyclic index distance is at least min_sep."""
    rng = np.random.default_rng(seed) if rng is None else rng
    phi = 2 * np.pi * np.arange(n) / n
    t_gt = np.stack([radius * np.cos(phi), radius * np.sin(phi), np.zeros(n)], 1)
    c, s = np.cos(phi + np.pi / 2), np.sin(phi + np.pi / 2)
    R_gt = np.zeros((n, 3, 3))
    R_gt[:, 0, 0], R_gt[:, 0, 1], R_gt[:, 1, 0], R_gt[:, 1, 1], R_gt[:, 2, 2] = c, -s, s, c, 1
    a, b = np.triu_indices(n, 1)
    d = np.minimum(b - a, n - (b - a))
    pool = np.stack([a[d >= min_sep], b[d >= min_sep]], 1)
    k = min(n_closures, pool.shape[0])
    pick = pool[rng.choice(pool.shape[0], size=k, replace=False)] if k else np.zeros((0, 2), np.int64)
    oi, oj = _odometry(n)
    ei = np.concatenate([oi, pick[:, 0]])
    ej = np.concatenate([oj, pick[:, 1]])
    return _measure(R_gt, t_gt, ei, ej, sigma_R, sigma_t, rng, init, name=f"circle-{n}")


def grid(nx=10, ny=10, nz=10, p=0.3, all_pairs=False, spacing=1.0, sigma_R=0.05, sigma_t=0.1,
         seed=0, init="odometry", rng=None):
    """Boustrophedon trajectory through a box.  With all_pairs every
    6-neighbour pair is an edge (directed low -> high); otherwise each
    non-odometry neighbour pair gets an edge in each direction with
    probability p (the cube rule of the experiments section)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    cells = boustrophedon(nx, ny, nz)
    n = cells.shape[0]
    t_gt = cells.astype(np.float64) * spacing
    R_gt = heading_frames(t_gt)
    pairs = grid_pairs(cells, _NB6)
    oi, oj = _odometry(n)
    if all_pairs:
        clos = _drop_odometry(pairs)
        ei, ej = np.concatenate([oi, clos[:, 0]]), np.concatenate([oj, clos[:, 1]])
    else:
        clos = _drop_odometry(pairs)
        u = rng.random((clos.shape[0], 2)) < p
        fwd, bwd = clos[u[:, 0]], clos[u[:, 1]]
        ei = np.concatenate([oi, fwd[:, 0], bwd[:, 1]])
        ej = np.concatenate([oj, fwd[:, 1], bwd[:, 0]])
    return _measure(R_gt, t_gt, ei, ej, sigma_R, sigma_t, rng, init, name=f"grid-{nx}x{ny}x{nz}")


def cube_expected_edges(nhat, p):
    """Expected edge count of the cube generator (experiments section)."""
    return 2 * (2 * nhat**3 - 3 * nhat**2 + 1) * p + nhat**3 - 1


def _sphere_layout(rings, per_ring, radius, n=None):
    order = []
    for r in range(rings):
        ks = range(per_ring) if r % 2 == 0 else range(per_ring - 1, -1, -1)
        order.extend((r, k) for k in ks)
    order = np.asarray(order, np.int64)
    if n is not None:
        order = order[:n]
    th = np.pi * (order[:, 0] + 0.5) / rings
    ph = 2 * np.pi * order[:, 1] / per_ring
    pos = radius * np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], 1)
    return order, pos


def _sphere_pairs(order, rings, per_ring, dks):
    idx = np.full((rings, per_ring), -1, np.int64)
    idx[order[:, 0], order[:, 1]] = np.arange(order.shape[0])
    r, k = order[:, 0], order[:, 1]
    A, B = [], []
    for dk in dks:
        a = np.nonzero(r < rings - 1)[0]
        b = idx[r[a] + 1, (k[a] + dk) % per_ring]
        A.append(a[b >= 0])
        B.append(b[b >= 0])
    a, b = np.concatenate(A), np.concatenate(B)
    return _unique_pairs(np.minimum(a, b), np.maximum(a, b), order.shape[0])


def sphere(rings=50, per_ring=50, radius=50.0, sigma_R=0.05, sigma_t=0.1, seed=0,
           init="odometry", rng=None):
    """Snake trajectory over latitude rings of a sphere; closures from every
    pose to the three nearest poses of the next ring."""
    rng = np.random.default_rng(seed) if rng is None else rng
    order, pos = _sphere_layout(rings, per_ring, radius)
    n = pos.shape[0]
    R_gt = heading_frames(pos)
    clos = _drop_odometry(_sphere_pairs(order, rings, per_ring, (-1, 0, 1)))
    oi, oj = _odometry(n)
    ei, ej = np.concatenate([oi, clos[:, 0]]), np.concatenate([oj, clos[:, 1]])
    return _measure(R_gt, pos, ei, ej, sigma_R, sigma_t, rng, init, name=f"sphere-{n}")


def tree(n=6, seed=0, sigma_R=0.05, sigma_t=0.1, init="odometry", rng=None):
    """A random tree (m = n-1) whose first n-1 edges are a chain; used for the
    zero-optimal-cost property."""
    rng = np.random.default_rng(seed) if rng is None else rng
    R_gt = so3_exp(rng.standard_normal((n, 3)))
    t_gt = rng.standard_normal((n, 3)) * 2.0
    oi, oj = _odometry(n)
    return _measure(R_gt, t_gt, oi, oj, sigma_R, sigma_t, rng, init, name=f"tree-{n}")


def random_small(n=5, m_extra=4, seed=0, sigma_R=0.1, sigma_t=0.1, init="odometry", rng=None,
                 kappa_scale=1.0):
    """A tiny random graph: chain plus m_extra random non-chain edges, random
    ground-truth poses."""
    rng = np.random.default_rng(seed) if rng is None else rng
    R_gt = so3_exp(rng.standard_normal((n, 3)))
    t_gt = rng.standard_normal((n, 3)) * 2.0
    oi, oj = _odometry(n)
    a, b = np.nonzero(~np.eye(n, dtype=bool))
    pool = np.stack([a, b], 1)
    pool = pool[~((pool[:, 1] - pool[:, 0]) == 1)]
    pick = pool[rng.choice(pool.shape[0], size=min(m_extra, pool.shape[0]), replace=False)]
    ei, ej = np.concatenate([oi, pick[:, 0]]), np.concatenate([oj, pick[:, 1]])
    g = _measure(R_gt, t_gt, ei, ej, sigma_R, sigma_t, rng, init, name=f"small-{n}")
    g.kappa *= kappa_scale
    return g


# ----------------------------------------------------------------------------
# batched mix
# ----------------------------------------------------------------------------
def _sample_pool_tiers(tiers, k, rng):
    """k distinct pairs, drawn without replacement tier by tier."""
    got = []
    for pool in tiers:
        if k <= 0:
            break
        if pool.shape[0] <= k:
            got.append(pool)
            k -= pool.shape[0]
        else:
            got.append(pool[rng.choice(pool.shape[0], size=k, replace=False)])
            k = 0
    return np.concatenate(got) if got else np.zeros((0, 2), np.int64)


def _circle_pool_sample(n, k, min_sep, rng):
    """k distinct pairs a<b with cyclic distance >= min_sep, uniform over
    k-subsets of that pool."""
    pool_size = n * (n - 1) // 2 - n * (min_sep - 1)
    if pool_size < 4 * k or n <= 400:
        a, b = np.triu_indices(n, 1)
        d = np.minimum(b - a, n - (b - a))
        pool = np.stack([a[d >= min_sep], b[d >= min_sep]], 1)
        return _sample_pool_tiers([pool], k, rng)
    keys = np.zeros(0, np.int64)
    while keys.shape[0] < k:
        a = rng.integers(0, n, size=2 * k)
        b = rng.integers(0, n, size=2 * k)
        lo, hi = np.minimum(a, b), np.maximum(a, b)
        d = np.minimum(hi - lo, n - (hi - lo))
        ok = d >= min_sep
        keys = np.unique(np.concatenate([keys, lo[ok] * n + hi[ok]]))
    keys = keys[rng.permutation(keys.shape[0])[:k]]
    return np.stack([keys // n, keys % n], 1)


def batched_graph(g, seed_seq, n_range=(50, 5000), rho_range=(1.2, 4.0),
                  sR_range=(0.01, 0.1), st_range=(0.01, 0.2)):
    rng = np.random.default_rng(seed_seq)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    rho = float(rng.uniform(*rho_range))
    sR = float(rng.uniform(*sR_range))
    st = float(rng.uniform(*st_range))
    m = int(round(rho * n))
    kind = ("circle", "grid", "sphere")[g % 3]
    if kind == "circle":
        radius = n / (2 * np.pi)
        phi = 2 * np.pi * np.arange(n) / n
        pos = np.stack([radius * np.cos(phi), radius * np.sin(phi), np.zeros(n)], 1)
        clos = _circle_pool_sample(n, m - (n - 1), 10, rng)
    elif kind == "grid":
        side = max(2, int(round(n ** (1 / 3))))
        nz = -(-n // (side * side))
        cells = boustrophedon(side, side, nz, n)
        pos = cells.astype(np.float64)
        t1 = _drop_odometry(grid_pairs(cells, _NB6))
        t2 = grid_pairs(cells, _HOP2)
        clos = _sample_pool_tiers([t1, t2], m - (n - 1), rng)
    else:
        rings = max(2, int(round(math.sqrt(n))))
        per = -(-n // rings)
        order, pos = _sphere_layout(rings, per, per / (2 * np.pi), n)
        t1 = _drop_odometry(_sphere_pairs(order, rings, per, (-1, 0, 1)))
        t2 = _sphere_pairs(order, rings, per, (-2, 2))
        clos = _sample_pool_tiers([t1, t2], m - (n - 1), rng)
    R_gt = heading_frames(pos)
    oi, oj = _odometry(n)
    ei, ej = np.concatenate([oi, clos[:, 0]]), np.concatenate([oj, clos[:, 1]])
    return _measure(R_gt, pos, ei, ej, sR, st, rng, "odometry", name=f"b{g}-{kind}-{n}",
                    meta=dict(kind=kind, sigma_R=sR, sigma_t=st, rho=rho))


def _batched_chunk(args):
    seed, G, lo, hi, kw = args
    seqs = np.random.SeedSequence(seed).spawn(G)
    return [batched_graph(g, seqs[g], **kw) for g in range(lo, hi)]


def batched(G=4096, seed=0, first=0, count=None, workers=1, **kw):
    """Graphs first..first+count-1 of the G-graph mix; graph g is seeded by
    SeedSequence(seed).spawn(G)[g] so any subset is reproducible.  With
    workers > 1 the graphs are built in forked worker processes (call this
    before the process touches a GPU)."""
    count = G - first if count is None else count
    if workers <= 1 or count < 64:
        return Batch(_batched_chunk((seed, G, first, first + count, kw)))
    import multiprocessing as mp
    step = max(16, count // (workers * 4))
    jobs = [(seed, G, lo, min(lo + step, first + count), kw)
            for lo in range(first, first + count, step)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_batched_chunk, jobs)
    return Batch([g for part in parts for g in part])


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
CONFIGS = {
    "circle-100": dict(iters=200, beta_scale=0.005),
    "grid-1k": dict(iters=500, beta_scale=0.005),
    "sphere-2.5k": dict(iters=1000, beta_scale=0.005),
    "grid-100k": dict(iters=1000, beta_scale=0.005),
    "batched-4096": dict(iters=50, beta_scale=0.005),
    "diff-20k": dict(iters=50, beta_scale=0.005),
}


def make_config(name, seed=0, **kw):
    if name == "circle-100":
        return circle(100, 10.0, 20, 10, 0.01, 0.01, seed=seed, **kw)
    if name == "grid-1k":
        return grid(10, 10, 10, p=0.3, sigma_R=0.05, sigma_t=0.1, seed=seed, **kw)
    if name == "sphere-2.5k":
        return sphere(50, 50, 50.0, 0.05, 0.1, seed=seed, **kw)
    if name == "grid-100k":
        return grid(50, 50, 40, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=seed, **kw)
    if name == "diff-20k":
        return grid(20, 25, 40, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=seed, **kw)
    raise KeyError(name)


def random_info(m, tau, aniso, seed=0):
    """Per-edge 3x3 translation information matrices S_e = tau_e R diag(a) R^T
    with random orientation R and eigenvalue ratios up to `aniso` (for the
    general-Sigma workloads); shape (m, 3, 3), symmetric positive definite."""
    rng = np.random.default_rng(seed)
    R = so3_exp(rng.standard_normal((m, 3)))
    a = np.exp(rng.uniform(-0.5, 0.5, (m, 3)) * np.log(aniso))
    return np.asarray(tau, np.float64)[:, None, None] * (R * a[:, None, :]) @ np.transpose(R, (0, 2, 1))
