"""Boundary preparation for the oracle (once per problem), torch float64.

Steps, in order:
 1. project every input rotation onto SO(3) (nearest rotation in Frobenius
    norm: U diag(1, 1, det(U V^T)) V^T from the SVD, a library primitive);
 2. convert each rotation to a unit quaternion with the rotation convention
    of App. A.2 ([0, R v] = q [0, v] q*), by the eigenvector of the symmetric
    4x4 matrix (4 qq^T - I)/3 that a rotation matrix determines (library
    symmetric eigensolver);
 3. fix the sign of each vertex quaternion: the first component, in
    (w, x, y, z) order, whose magnitude exceeds 1e-6 is made positive;
 4. fix the sign of each measurement quaternion so that the initial poses
    are consistent with it, <p_i^0 q~_e, p_j^0> >= 0.  The cost of model (1)
    depends on the sign of q~_ij (the term ||p_j^* p_i q~_ij - 1||), while a
    rotation matrix fixes it only up to sign; this reading is the boundary's
    choice (the paper draws quaternions directly).  Flipping one vertex sign
    flips the alignment of its edges, so any vertex sign rule gives the same
    problem up to the sign gauge p_i -> -p_i.
"""
import torch

from .quat import F64, qmul

SIGN_EPS = 1e-6


def project_so3(R):
    """Nearest rotation (det +1) to each 3x3 matrix."""
    R = torch.as_tensor(R, dtype=F64)
    U, _, Vh = torch.linalg.svd(R)
    d = torch.linalg.det(U @ Vh)
    S = torch.diag_embed(torch.stack([torch.ones_like(d), torch.ones_like(d), d], -1))
    return U @ S @ Vh


def rot_to_quat(R):
    """Unit quaternion [w,x,y,z] of a rotation matrix (sign arbitrary)."""
    R = torch.as_tensor(R, dtype=F64)
    r = lambda a, b: R[..., a, b]
    K = torch.stack([
        torch.stack([r(0, 0) - r(1, 1) - r(2, 2), r(0, 1) + r(1, 0), r(0, 2) + r(2, 0), r(2, 1) - r(1, 2)], -1),
        torch.stack([r(0, 1) + r(1, 0), r(1, 1) - r(0, 0) - r(2, 2), r(1, 2) + r(2, 1), r(0, 2) - r(2, 0)], -1),
        torch.stack([r(0, 2) + r(2, 0), r(1, 2) + r(2, 1), r(2, 2) - r(0, 0) - r(1, 1), r(1, 0) - r(0, 1)], -1),
        torch.stack([r(2, 1) - r(1, 2), r(0, 2) - r(2, 0), r(1, 0) - r(0, 1), r(0, 0) + r(1, 1) + r(2, 2)], -1),
    ], -2) / 3.0
    _, V = torch.linalg.eigh(K)
    xyzw = V[..., :, -1]
    q = torch.cat([xyzw[..., 3:], xyzw[..., :3]], -1)
    return q / q.norm(dim=-1, keepdim=True)


def canonical_sign(q):
    """Make the first component with |c| > 1e-6 positive."""
    big = q.abs() > SIGN_EPS
    first = torch.argmax(big.to(torch.int64), dim=-1, keepdim=True)
    lead = torch.gather(q, -1, first)
    return torch.where(lead < 0, -q, q)


def align_edges(p0, qm, ei, ej):
    """Flip q~_e where <p0_i q~_e, p0_j> < 0 (an exact 0 keeps the sign)."""
    s = (qmul(p0[ei], qm) * p0[ej]).sum(-1, keepdim=True)
    return torch.where(s < 0, -qm, qm)


def prepare(n, ei, ej, Rm, tm, kappa, tau, R0, t0):
    """Returns (problem dict, p0 (n,4), t0 (n,3)) in float64 tensors."""
    ei = torch.as_tensor(ei, dtype=torch.int64)
    ej = torch.as_tensor(ej, dtype=torch.int64)
    p0 = canonical_sign(rot_to_quat(project_so3(torch.as_tensor(R0, dtype=F64).reshape(n, 3, 3))))
    m = ei.shape[0]
    qm = rot_to_quat(project_so3(torch.as_tensor(Rm, dtype=F64).reshape(m, 3, 3)))
    qm = align_edges(p0, qm, ei, ej)
    prob = dict(n=n, m=m, ei=ei, ej=ej, qm=qm,
                tm=torch.as_tensor(tm, dtype=F64).reshape(m, 3).clone(),
                kappa=torch.as_tensor(kappa, dtype=F64).reshape(m).clone(),
                tau=torch.as_tensor(tau, dtype=F64).reshape(m).clone())
    return prob, p0, torch.as_tensor(t0, dtype=F64).reshape(n, 3).clone()


def prepare_graph(g):
    """Convenience wrapper for a pgo_synth.Graph."""
    return prepare(g.n, g.ei, g.ej, g.Rm, g.tm, g.kappa, g.tau, g.R0, g.t0)
