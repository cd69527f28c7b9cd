"""Brute-force local optimisation of model (1) for tiny graphs (test
infrastructure only).

Residuals of model (1) per edge, Sigma1 = tau I, Sigma2 = kappa I:
    sqrt(tau)   * Im(t~_j - t~_i - p_i t~_ij p_i^*)      (3 components; the real
                                                            part is 0 for unit p_i)
    sqrt(kappa) * (p_j^* p_i q~_ij - 1)                   (4 components)
with p_i = x_i / ||x_i|| for free x_i in R^4.  The minimiser is scipy's
Levenberg-Marquardt (a library routine), run from a given start or from many
random starts.
"""
import numpy as np
from scipy.optimize import least_squares


def _qmul(a, b):
    a0, a1, a2, a3 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    b0, b1, b2, b3 = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0], -1)


def _conj(a):
    return a * np.array([1.0, -1.0, -1.0, -1.0])


def _unpack(x, n):
    P = x[: 4 * n].reshape(n, 4)
    P = P / np.linalg.norm(P, axis=1, keepdims=True)
    return P, x[4 * n:].reshape(n, 3)


def residual(x, n, ei, ej, qm, tm, kappa, tau):
    p, t = _unpack(x, n)
    th = np.concatenate([np.zeros((len(ei), 1)), tm], 1)
    rot = _qmul(_qmul(p[ei], th), _conj(p[ei]))[:, 1:]
    rt = np.sqrt(tau)[:, None] * (t[ej] - t[ei] - rot)
    rq = np.sqrt(kappa)[:, None] * (_qmul(_qmul(_conj(p[ej]), p[ei]), qm) - np.array([1.0, 0, 0, 0]))
    return np.concatenate([rt.ravel(), rq.ravel()])


def model_cost(p, t, ei, ej, qm, tm, kappa, tau):
    x = np.concatenate([np.asarray(p).ravel(), np.asarray(t).ravel()])
    r = residual(x, len(p), ei, ej, qm, tm, kappa, tau)
    return float(r @ r)


def local_min(p0, t0, ei, ej, qm, tm, kappa, tau, tol=1e-15):
    """Levenberg-Marquardt on model (1) from (p0, t0); returns (cost, p, t)."""
    n = len(p0)
    x0 = np.concatenate([np.asarray(p0, float).ravel(), np.asarray(t0, float).ravel()])
    args = (n, np.asarray(ei), np.asarray(ej), np.asarray(qm, float), np.asarray(tm, float),
            np.asarray(kappa, float), np.asarray(tau, float))
    sol = least_squares(residual, x0, args=args, method="lm", xtol=tol, ftol=tol, gtol=tol,
                        max_nfev=20000)
    p, t = _unpack(sol.x, n)
    r = residual(sol.x, *args)
    return float(r @ r), p, t


def multistart_min(n, ei, ej, qm, tm, kappa, tau, starts=50, seed=0):
    """Smallest local-minimum cost over random starts (uniform rotations,
    Gaussian translations)."""
    rng = np.random.default_rng(seed)
    best = np.inf
    for _ in range(starts):
        p0 = rng.standard_normal((n, 4))
        t0 = rng.standard_normal((n, 3)) * 3.0
        c, _, _ = local_min(p0, t0, ei, ej, qm, tm, kappa, tau, tol=1e-12)
        best = min(best, c)
    return best


# ---------------------------------------------------------------------------
# Sparse damped Newton on model (1) for graphs of thousands of poses.  The
# same residuals as `residual` above; each pose is moved by a left increment
# (p_i <- Exp(d_i / 2) p_i as a unit quaternion, t_i <- t_i + u_i), so every
# pose has 6 unknowns.  First derivatives (the Jacobian J):
#   translation rows  sqrt(tau) (t_j - t_i - R(p_i) t~):
#       d/du_j = sqrt(tau) I,  d/du_i = -sqrt(tau) I,
#       d/dd_i = sqrt(tau) [R(p_i) t~]_x   (d R(p) t~ = d x R(p) t~)
#   rotation rows     sqrt(kappa) (p_j^* p_i q~ - 1):
#       d/dd_i = sqrt(kappa)/2 L(p_j^*) R(p_i q~) E,  d/dd_j = -d/dd_i
#       (L, R the left/right product matrices, E the pure part [0; I3]).
# Second derivatives, contracted with the residual (S = sum_k r_k Hess r_k):
#   translation rows: R(Exp d) v = v + d x v + (1/2) d x (d x v) + ..., so with
#       v = R(p_i) t~ and the edge's residual 3-vector r_t, block (d_i, d_i)
#       -sqrt(tau) ((v r_t^T + r_t v^T) / 2 - (v . r_t) I);
#   rotation rows: Exp(-d_j / 2) Exp(d_i / 2) = [1 - |d_i - d_j|^2 / 8,
#       (d_i - d_j) / 2 - (d_j x d_i) / 4] + ..., so with
#       rho = (sqrt(kappa) L(p_j^*) R(p_i q~))^T r_q and a = -rho_0 / 4,
#       blocks (d_i, d_i) = (d_j, d_j) = a I, (d_i, d_j) = -a I - [rho_v]_x / 4,
#       (d_j, d_i) its transpose.
# The Hessian of F = |r|^2 is 2 (J^T J + S).  Each step solves
# (J^T J + S + mu diag(J^T J)) x = -J^T r by a sparse LU factorisation, or
# by a dense Cholesky factorisation (LAPACK) when the graph has long-range
# loop closures (its reverse Cuthill-McKee bandwidth above a tenth of its
# poses) and at most 36000 unknowns: such graphs fill a sparse factorisation
# almost completely, and Krylov solvers do not converge on these systems.  A
# dense matrix that is not positive definite counts as a rejected step.  mu
# follows the gain-ratio rule on the quadratic model (a tenth after a step
# the model predicts well, doubled growth after a rejected one), so near the
# minimum the steps are Newton steps and converge quadratically.  (Gauss-
# Newton alone, without S, stalls on these graphs: along their soft modes the
# true curvature is a few percent of J^T J's.)  The first pose of every
# connected component is held fixed (the gauge).
# ---------------------------------------------------------------------------
def _qexp_half(d):
    th = np.linalg.norm(d, axis=1)
    s = np.where(th > 1e-12, np.sin(th / 2) / np.where(th > 0, th, 1.0), 0.5)
    return np.concatenate([np.cos(th / 2)[:, None], s[:, None] * d], 1)


def _lmat(a):   # L(a) b = a b
    w, x, y, z = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    return np.stack([np.stack([w, -x, -y, -z], -1), np.stack([x, w, -z, y], -1),
                     np.stack([y, z, w, -x], -1), np.stack([z, -y, x, w], -1)], -2)


def _rmat(a):   # R(a) b = b a
    w, x, y, z = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    return np.stack([np.stack([w, -x, -y, -z], -1), np.stack([x, w, z, -y], -1),
                     np.stack([y, -z, w, x], -1), np.stack([z, y, -x, w], -1)], -2)


def _skew(v):
    o = np.zeros(v.shape[:-1] + (3, 3))
    o[..., 0, 1], o[..., 0, 2] = -v[..., 2], v[..., 1]
    o[..., 1, 0], o[..., 1, 2] = v[..., 2], -v[..., 0]
    o[..., 2, 0], o[..., 2, 1] = -v[..., 1], v[..., 0]
    return o


def _blocks(shape, parts):
    """Sparse matrix from dense per-edge blocks: parts = [(r0, c0, B)] with
    B (m, a, b) placed at rows r0[e] + k, cols c0[e] + l."""
    import scipy.sparse as sp
    rows, cols, vals = [], [], []
    for r0, c0, B in parts:
        a, b = B.shape[1], B.shape[2]
        rows.append(((r0[:, None, None] + np.arange(a)[None, :, None])
                     + 0 * np.arange(b)[None, None, :]).ravel())
        cols.append(((c0[:, None, None] + np.arange(b)[None, None, :])
                     + 0 * np.arange(a)[None, :, None]).ravel())
        vals.append(B.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=shape)


def _rot_t(p, ei, tm):
    th = np.concatenate([np.zeros((len(ei), 1)), tm], 1)
    return _qmul(_qmul(p[ei], th), _conj(p[ei]))[:, 1:]


def _jacobian(p, t, ei, ej, qm, tm, kappa, tau):
    n, m = len(p), len(ei)
    st, sk = np.sqrt(tau), np.sqrt(kappa)
    e3 = 3 * np.arange(m)
    eq = 3 * m + 4 * np.arange(m)
    I3 = np.broadcast_to(np.eye(3), (m, 3, 3))
    E = np.zeros((4, 3))
    E[1:] = np.eye(3)
    D = 0.5 * sk[:, None, None] * (_lmat(_conj(p[ej])) @ _rmat(_qmul(p[ei], qm)) @ E)
    return _blocks((7 * m, 6 * n), [
        (e3, 6 * ej + 3, st[:, None, None] * I3),
        (e3, 6 * ei + 3, -st[:, None, None] * I3),
        (e3, 6 * ei, st[:, None, None] * _skew(_rot_t(p, ei, tm))),
        (eq, 6 * ei, D), (eq, 6 * ej, -D)])


def _second_order(p, t, r, ei, ej, qm, tm, kappa, tau):
    """S = sum_k r_k Hess(r_k) in the left-increment chart (6n x 6n; only
    rotation-rotation blocks are nonzero)."""
    n, m = len(p), len(ei)
    st, sk = np.sqrt(tau), np.sqrt(kappa)
    rt, rq = r[:3 * m].reshape(m, 3), r[3 * m:].reshape(m, 4)
    v = _rot_t(p, ei, tm)
    I3 = np.eye(3)
    Ht = -st[:, None, None] * (0.5 * (v[:, :, None] * rt[:, None, :] + rt[:, :, None] * v[:, None, :])
                               - (v * rt).sum(1)[:, None, None] * I3)
    M = sk[:, None, None] * (_lmat(_conj(p[ej])) @ _rmat(_qmul(p[ei], qm)))
    rho = np.einsum("mab,ma->mb", M, rq)
    a = (-rho[:, 0] / 4)[:, None, None] * I3
    X = -0.25 * _skew(rho[:, 1:])
    return _blocks((6 * n, 6 * n), [(6 * ei, 6 * ei, Ht + a), (6 * ej, 6 * ej, a),
                                    (6 * ei, 6 * ej, -a + X),
                                    (6 * ej, 6 * ei, -a + np.transpose(X, (0, 2, 1)))])


def _rcm_bandwidth(n, ei, ej):
    """Bandwidth of the pose graph's adjacency after reverse Cuthill-McKee."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    A = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(n, n)).tocsr()
    A = (A + A.T).tocsr()
    perm = reverse_cuthill_mckee(A, symmetric_mode=True)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    return int(np.abs(pos[ei] - pos[ej]).max()) if len(ei) else 0


def _damped_solve(H, dg, mu, g, dense):
    """x with (H + mu diag(dg)) x = -g, or None when the dense matrix is not
    positive definite."""
    import scipy.sparse as sp
    if dense:
        import scipy.linalg as la
        A = H.toarray()
        A[np.diag_indices_from(A)] += mu * dg
        try:
            c = la.cho_factor(A, overwrite_a=True, check_finite=False)
        except la.LinAlgError:
            return None
        return la.cho_solve(c, -g, check_finite=False)
    import scipy.sparse.linalg as spla
    return spla.splu((H + sp.diags(mu * dg)).tocsc()).solve(-g)


def sparse_local_min(p0, t0, ei, ej, qm, tm, kappa, tau, max_iter=200, ftol=1e-12,
                     dense_max=36000):
    """Damped Newton on model (1) from (p0, t0) with the exact sparse Hessian
    above; returns (cost, p, t, info).  Stops once an accepted step that the
    quadratic model predicted well (gain ratio above 1/2) lowers the cost by
    less than ftol * F -- in the quadratic regime the remaining gap is then
    far below that -- or once no damping gives a lower cost (rounding
    level).  info: iterations, the final max |J^T r| over the free unknowns,
    the last accepted relative decrease, and which rule stopped the run."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    p = np.asarray(p0, float) / np.linalg.norm(p0, axis=1, keepdims=True)
    t = np.asarray(t0, float).copy()
    n = len(p)
    ei, ej = np.asarray(ei), np.asarray(ej)
    args = (ei, ej, np.asarray(qm, float), np.asarray(tm, float), np.asarray(kappa, float),
            np.asarray(tau, float))
    _, lab = connected_components(sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(n, n)),
                                  directed=False)
    fixed = np.zeros(n, bool)
    fixed[[int(np.flatnonzero(lab == c)[0]) for c in range(lab.max() + 1)]] = True
    free = np.repeat(~fixed, 6)
    dense = 6 * n <= dense_max and _rcm_bandwidth(n, ei, ej) > 0.1 * n

    def res(p_, t_):
        return residual(np.concatenate([p_.ravel(), t_.ravel()]), n, *args)

    r = res(p, t)
    F = float(r @ r)
    mu, it, gmax, rel, stop = 1e-6, 0, np.inf, np.inf, "max_iter"
    for it in range(1, max_iter + 1):
        J = _jacobian(p, t, *args)[:, free]
        g = J.T @ r
        gmax = float(np.abs(g).max()) if g.size else 0.0
        if gmax == 0.0:
            stop = "zero gradient"
            break
        JJ = (J.T @ J).tocsc()
        H = (JJ + _second_order(p, t, r, *args)[free][:, free]).tocsc()
        dg = np.maximum(JJ.diagonal(), 1e-12)
        nu, rho = 2.0, -1.0
        while mu <= 1e12:
            x = _damped_solve(H, dg, mu, g, dense)
            if x is None:   # not positive definite: more damping
                mu *= nu
                nu *= 2.0
                continue
            pred = -(2 * g @ x + x @ (H @ x))
            step = np.zeros(6 * n)
            step[free] = x
            step = step.reshape(n, 6)
            p1 = _qmul(_qexp_half(step[:, :3]), p)
            p1 /= np.linalg.norm(p1, axis=1, keepdims=True)
            t1 = t + step[:, 3:]
            r1 = res(p1, t1)
            F1 = float(r1 @ r1)
            rho = (F - F1) / pred if pred > 0 else -1.0
            if rho > 0:
                break
            mu *= nu
            nu *= 2.0
        if rho <= 0:   # no damping lowers the cost: rounding level
            stop = "rounding"
            break
        rel = (F - F1) / F
        p, t, r, F = p1, t1, r1, F1
        mu = max(mu * (0.1 if rho > 0.75 else max(1.0 / 3.0, 1.0 - (2.0 * rho - 1.0) ** 3)), 1e-12)
        if rel < ftol and rho > 0.5:
            stop = "ftol"
            break
    return F, p, t, {"iterations": it, "grad_max": gmax, "last_rel_decrease": rel, "stop": stop}
