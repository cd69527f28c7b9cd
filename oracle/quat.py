"""Quaternion algebra, App. A.2 ("Quaternion and Pose"), in torch float64.

Quaternions are 4-vectors [q0, q1, q2, q3] = [w, x, y, z].  All functions
broadcast over leading dimensions.
"""
import torch

F64 = torch.float64


def qmul(a, b):
    """Hamilton product (App. A.2): [a0 b0 - a.b, a0 b + b0 a + a x b]."""
    a0, av = a[..., :1], a[..., 1:]
    b0, bv = b[..., :1], b[..., 1:]
    w = a0 * b0 - (av * bv).sum(-1, keepdim=True)
    v = a0 * bv + b0 * av + torch.cross(av, bv, dim=-1)
    return torch.cat([w, v], -1)


def qconj(a):
    """Conjugate q* = [q0, -q1, -q2, -q3] (App. A.2)."""
    return torch.cat([a[..., :1], -a[..., 1:]], -1)


def hat(v):
    """Pure quaternion [0, v] of a 3-vector (Model section, t~ = [0, t])."""
    return torch.cat([torch.zeros_like(v[..., :1]), v], -1)


def Mmat(a):
    """Left-multiplication matrix M(a) of App. A.2 (a b = M(a) b)."""
    a0, a1, a2, a3 = a.unbind(-1)
    rows = [torch.stack([a0, -a1, -a2, -a3], -1),
            torch.stack([a1, a0, -a3, a2], -1),
            torch.stack([a2, a3, a0, -a1], -1),
            torch.stack([a3, -a2, a1, a0], -1)]
    return torch.stack(rows, -2)


def Wmat(a):
    """Right-multiplication matrix W(a) of App. A.2 (b a = W(a) b)."""
    a0, a1, a2, a3 = a.unbind(-1)
    rows = [torch.stack([a0, -a1, -a2, -a3], -1),
            torch.stack([a1, a0, a3, -a2], -1),
            torch.stack([a2, -a3, a0, a1], -1),
            torch.stack([a3, a2, -a1, a0], -1)]
    return torch.stack(rows, -2)


D4 = torch.diag(torch.tensor([1.0, -1.0, -1.0, -1.0], dtype=F64))
ONE = torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=F64)


def mv(A, x):
    """Batched matrix-vector product."""
    return (A @ x.unsqueeze(-1)).squeeze(-1)


def rotmat(q):
    """Rotation matrix of a unit quaternion by its action [0, R v] = q [0, v] q*
    (App. A.2), column k being the image of the k-th basis vector."""
    cols = []
    for k in range(3):
        e = torch.zeros(q.shape[:-1] + (3,), dtype=q.dtype)
        e[..., k] = 1.0
        cols.append(qmul(qmul(q, hat(e)), qconj(q))[..., 1:])
    return torch.stack(cols, -1)
