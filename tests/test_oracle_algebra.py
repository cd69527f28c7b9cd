"""Pins of the oracle's quaternion algebra and boundary preparation against
what App. A.2 / A.4 fix independently: Hamilton's rules, Lemma MW, the
rotation formula, composition, the distance identities, and library polar
decomposition."""
import numpy as np
import pytest
import scipy.linalg
import torch

from oracle import prep
from oracle.quat import D4, Mmat, Wmat, qconj, qmul, rotmat
from tests import qref

F64 = torch.float64
rng = np.random.default_rng(1)


def rq(k):
    return torch.as_tensor(rng.standard_normal((k, 4)), dtype=F64)


def unit(k):
    q = rq(k)
    return q / q.norm(dim=1, keepdim=True)


def test_hamilton_rules():
    one, i, j, k = (torch.eye(4, dtype=F64)[a] for a in range(4))
    for u in (i, j, k):
        assert torch.equal(qmul(u, u), -one)
    assert torch.equal(qmul(qmul(i, j), k), -one)
    assert torch.equal(qmul(i, j), k) and torch.equal(qmul(j, k), i) and torch.equal(qmul(k, i), j)


def test_product_matches_test_local_product():
    a, b = rq(50), rq(50)
    assert np.allclose(qmul(a, b).numpy(), qref.qmul(a.numpy(), b.numpy()), atol=1e-15)


def test_product_properties():
    a, b, c = rq(20), rq(20), rq(20)
    assert torch.allclose(qmul(qmul(a, b), c), qmul(a, qmul(b, c)), atol=1e-13)
    assert torch.allclose(qconj(qmul(a, b)), qmul(qconj(b), qconj(a)), atol=1e-14)
    assert torch.allclose(qmul(a, b).norm(dim=1), a.norm(dim=1) * b.norm(dim=1), atol=1e-13)
    assert torch.allclose(qmul(a, qconj(a))[:, 1:], torch.zeros(20, 3, dtype=F64), atol=1e-15)


def test_lemma_MW():
    a, b = rq(30), rq(30)
    # (a) M(a*) = M(a)^T, W(a*) = W(a)^T
    assert torch.equal(Mmat(qconj(a)), Mmat(a).transpose(-1, -2))
    assert torch.equal(Wmat(qconj(a)), Wmat(a).transpose(-1, -2))
    # (b) ab = M(a) b = W(b) a
    ab = qmul(a, b)
    assert torch.allclose((Mmat(a) @ b[..., None])[..., 0], ab, atol=1e-14)
    assert torch.allclose((Wmat(b) @ a[..., None])[..., 0], ab, atol=1e-14)
    # (c) M^T M = W^T W = ||a||^2 I
    n2 = (a * a).sum(1)[:, None, None] * torch.eye(4, dtype=F64)
    assert torch.allclose(Mmat(a).transpose(-1, -2) @ Mmat(a), n2, atol=1e-13)
    assert torch.allclose(Wmat(a).transpose(-1, -2) @ Wmat(a), n2, atol=1e-13)
    # D x = x^*
    assert torch.equal((D4 @ a[..., None])[..., 0], qconj(a))


def test_rotation_matches_rodrigues():
    for _ in range(20):
        axis = rng.standard_normal(3)
        th = rng.uniform(0, np.pi)
        n = axis / np.linalg.norm(axis)
        q = torch.as_tensor(np.r_[np.cos(th / 2), np.sin(th / 2) * n], dtype=F64)
        assert np.allclose(rotmat(q).numpy(), qref.rodrigues(axis, th), atol=1e-14)


def test_composition():
    a, b = unit(10), unit(10)
    assert torch.allclose(rotmat(qmul(a, b)), rotmat(a) @ rotmat(b), atol=1e-14)


def test_distance_identities():
    """App. A.4: ||q1 - q2|| = 2 sin(theta/4) (signs aligned),
    ||R1 - R2||_F = 2 sqrt(2) sin(theta/2), theta = arccos((tr(R1^T R2)-1)/2)."""
    a, b = unit(40), unit(40)
    b = torch.where(((a * b).sum(1, keepdim=True)) < 0, -b, b)
    R1, R2 = rotmat(a), rotmat(b)
    tr = torch.diagonal(R1.transpose(-1, -2) @ R2, dim1=-2, dim2=-1).sum(-1)
    th = torch.arccos(torch.clamp((tr - 1) / 2, -1, 1))
    assert torch.allclose((a - b).norm(dim=1), 2 * torch.sin(th / 4), atol=1e-7)
    assert torch.allclose((R1 - R2).flatten(1).norm(dim=1), 2 * np.sqrt(2) * torch.sin(th / 2), atol=1e-7)


def test_project_so3_vs_library_polar():
    for _ in range(10):
        R = rotmat(unit(1))[0].numpy() + 1e-3 * rng.standard_normal((3, 3))
        U, _ = scipy.linalg.polar(R)
        assert np.allclose(prep.project_so3(torch.as_tensor(R)[None])[0].numpy(), U, atol=1e-13)
    # exact rotations are fixed; a reflection-free det fix
    Q = rotmat(unit(5))
    assert torch.allclose(prep.project_so3(Q), Q, atol=1e-14)
    P = prep.project_so3(torch.as_tensor(np.diag([1.0, 1.0, -0.2]))[None])
    assert abs(torch.linalg.det(P)[0].item() - 1) < 1e-14


def test_rot_to_quat_roundtrip_including_half_turns():
    qs = unit(200)
    half = torch.cat([torch.zeros(20, 1, dtype=F64), rq(20)[:, 1:]], 1)
    half = half / half.norm(dim=1, keepdim=True)
    qs = torch.cat([qs, half])
    R = rotmat(qs)
    q2 = prep.rot_to_quat(R)
    assert torch.allclose(rotmat(q2), R, atol=1e-13)
    assert torch.allclose((q2 * qs).sum(1).abs(), torch.ones(len(qs), dtype=F64), atol=1e-13)


def test_canonical_sign_rule():
    q = torch.tensor([[-0.5, 0.5, 0.5, 0.5], [1e-9, -1.0, 0, 0], [0, 0, -0.6, 0.8]], dtype=F64)
    c = prep.canonical_sign(q)
    assert torch.equal(c[0], -q[0]) and torch.equal(c[1], -q[1]) and torch.equal(c[2], -q[2])


def test_alignment_makes_noise_free_edges_exact():
    import pgo_synth as S
    g = S.grid(3, 3, 3, p=0.6, sigma_R=0.0, sigma_t=0.0, init="gt")
    P, p0, t0 = prep.prepare_graph(g)
    lhs = qmul(p0[P["ei"]], P["qm"])
    assert torch.allclose(lhs, p0[P["ej"]], atol=1e-14)
