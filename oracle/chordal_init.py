"""Chordal initialisation -- oracle, FP64, test infrastructure only.

The experiments start every method from a chordal initial point (cited in
the experiments section, not described).  Reading taken here, the usual
three steps on a graph with measurements (R~_e, t~_e, kappa_e, tau_e):

  1. relaxed rotations: minimise sum_e kappa_e |R_i R~_e - R_j|_F^2 over
     unconstrained 3x3 blocks R_i, one anchor per connected component (the
     lowest-index vertex, held at its given rotation);
  2. projection of every R_i onto SO(3) (SVD, det fix);
  3. translations: minimise sum_e tau_e |t_j - t_i - R_i t~_e|^2 with the
     projected R_i, the same anchors held at their given translations.

Both least-squares problems are written as a stacked residual matrix
(one block row per edge) and solved through its normal equations with a
sparse direct factorisation -- not the operator form the library iterates.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

from .chordal import project_so3


def components(n, ei, ej):
    """Label of each vertex's connected component (undirected) and the
    anchor (lowest vertex index) of every component."""
    g = sp.coo_matrix((np.ones(len(ei)), (ei, ej)), shape=(n, n))
    _, lab = sp.csgraph.connected_components(g, directed=False)
    anchor = np.full(lab.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(anchor, lab, np.arange(n))
    is_anchor = np.zeros(n, bool)
    is_anchor[anchor] = True
    return lab, is_anchor


def _solve_rows(B, W, free, fixed_vals, ncols_per_vertex, n, extra_rhs=None):
    """min_x |W^(1/2) (B x - c)|^2 over the free unknowns, the fixed ones set
    to fixed_vals (n x ncols) -- c = extra_rhs (or 0).  Returns n x ncols."""
    k = ncols_per_vertex
    cols_free = (np.arange(n)[free][:, None] * k + np.arange(k)[None]).ravel()
    cols_fix = (np.arange(n)[~free][:, None] * k + np.arange(k)[None]).ravel()
    Bf = B[:, cols_free].tocsc()
    Bx = B[:, cols_fix]
    c = -(Bx @ fixed_vals[~free].ravel())
    if extra_rhs is not None:
        c = c + extra_rhs
    N = (Bf.T @ W @ Bf).tocsc()
    x = np.zeros((n, k))
    if cols_free.size:
        x[free] = spla.spsolve(N, Bf.T @ (W @ c)).reshape(-1, k)
    x[~free] = fixed_vals[~free]
    return x


def chordal_init(n, ei, ej, Rm, tm, kappa, tau, R_given, t_given, return_relaxed=False):
    """Chordal initial point (R (n,3,3), t (n,3)) as numpy arrays; measured
    and given rotations are projected onto SO(3) first (as the boundary
    does).  return_relaxed adds the unprojected least-squares blocks."""
    ei = np.asarray(ei, np.int64)
    ej = np.asarray(ej, np.int64)
    m = len(ei)
    Rm = project_so3(torch.as_tensor(np.asarray(Rm, np.float64).reshape(m, 3, 3))).numpy()
    _, is_anchor = components(n, ei, ej)
    free = ~is_anchor
    # rotations: the three rows of R_i decouple; for a row vector x_i of R_i
    # the residual of edge e is R~_e^T x_i^T - x_j^T (3 rows per edge)
    e3 = 3 * np.arange(m)
    a, b = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")   # entry (a, b)
    rows = np.concatenate([(e3[:, None, None] + a[None]).ravel(), (e3[:, None] + np.arange(3)).ravel()])
    cols = np.concatenate([(3 * ei[:, None, None] + b[None]).ravel(),
                           (3 * ej[:, None] + np.arange(3)).ravel()])
    vals = np.concatenate([np.transpose(Rm, (0, 2, 1)).ravel(), -np.ones(3 * m)])
    B = sp.csr_matrix((vals, (rows, cols)), shape=(3 * m, 3 * n))
    W = sp.diags(np.repeat(np.asarray(kappa, np.float64), 3))
    R_given = project_so3(torch.as_tensor(np.asarray(R_given, np.float64).reshape(n, 3, 3))).numpy()
    R = np.empty((n, 3, 3))
    for r in range(3):
        R[:, r, :] = _solve_rows(B, W, free, R_given[:, r, :], 3, n)
    Rp = project_so3(torch.as_tensor(R)).numpy()
    Rp[is_anchor] = R_given[is_anchor]
    # translations: residual of edge e is t_j - t_i - R_i t~_e
    rows = np.tile((e3[:, None] + np.arange(3)).ravel(), 2)
    cols = np.concatenate([(3 * ej[:, None] + np.arange(3)).ravel(),
                           (3 * ei[:, None] + np.arange(3)).ravel()])
    vals = np.concatenate([np.ones(3 * m), -np.ones(3 * m)])
    Bt = sp.csr_matrix((vals, (rows, cols)), shape=(3 * m, 3 * n))
    Wt = sp.diags(np.repeat(np.asarray(tau, np.float64), 3))
    c = np.einsum("kab,kb->ka", Rp[ei], np.asarray(tm, np.float64).reshape(m, 3)).ravel()
    t = _solve_rows(Bt, Wt, free, np.asarray(t_given, np.float64).reshape(n, 3), 3, n, extra_rhs=c)
    return (Rp, t, R) if return_relaxed else (Rp, t)


def chordal_init_graph(g, return_relaxed=False):
    return chordal_init(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, g.R0, g.t0, return_relaxed)


def relaxed_objective(n, ei, ej, Rm, kappa, R):
    """sum_e kappa_e |R_i R~_e - R_j|_F^2 for unconstrained blocks R."""
    r = R[ei] @ Rm - R[ej]
    return float((kappa * (r * r).sum((1, 2))).sum())
