"""Input generator checks: edge counts of the named workloads and the cube
edge-count law of the experiments section (Data Settings (b))."""
import json
import os

import numpy as np
import pytest

import pgo_synth as S

HERE = os.path.dirname(__file__)


@pytest.mark.parametrize("name,n,m", [
    ("circle-100", 100, 119),
    ("sphere-2.5k", 2500, 9800),
    ("grid-100k", 100_000, 293_500),
    ("diff-20k", 20_000, 57_700),
])
def test_named_sizes(name, n, m):
    g = S.make_config(name)
    assert (g.n, g.m) == (n, m)


def _closure_pairs(nhat):
    return 2 * nhat**3 - 3 * nhat**2 + 1


def test_cube_edge_law_mean():
    """Mean m over 200 seeds matches E(m) within 3 standard errors."""
    nhat, p = 4, 0.3
    ms = np.array([S.grid(nhat, nhat, nhat, p=p, seed=s).m for s in range(200)])
    N = 2 * _closure_pairs(nhat)
    se = np.sqrt(N * p * (1 - p) / len(ms))
    assert abs(ms.mean() - S.cube_expected_edges(nhat, p)) < 3 * se


def test_cube_edge_law_matches_paper_realisations():
    """Every m the paper reports for its cubes is a plausible draw (|z| < 3.5)
    of this generator's m = nhat^3 - 1 + Binomial(2(2nhat^3-3nhat^2+1), p)."""
    cases = json.load(open(os.path.join(HERE, "golden", "cube_edges.json")))["cases"]
    for c in cases:
        nhat, p, m = c["nhat"], c["p"], c["m"]
        N = 2 * _closure_pairs(nhat)
        mean = S.cube_expected_edges(nhat, p)
        sd = np.sqrt(N * p * (1 - p))
        assert abs(m - mean) <= 3.5 * sd, c


def test_boustrophedon_steps_are_unit():
    c = S.boustrophedon(5, 4, 3)
    assert len({tuple(x) for x in c}) == 60
    assert np.all(np.abs(np.diff(c, axis=0)).sum(1) == 1)


def test_noise_free_measurements_are_exact():
    g = S.grid(3, 3, 3, p=0.5, sigma_R=0.0, sigma_t=0.0, init="odometry")
    Ri, Rj = g.R_gt[g.ei], g.R_gt[g.ej]
    assert np.allclose(g.Rm, np.transpose(Ri, (0, 2, 1)) @ Rj, atol=1e-14)
    assert np.allclose(g.R0, g.R_gt, atol=1e-12) and np.allclose(g.t0, g.t_gt, atol=1e-12)


def test_rotation_noise_scale():
    """Angles of R_gt-relative noise have the chi(3) * sigma law: mean of
    theta^2 is 3 sigma^2."""
    g = S.grid(8, 8, 8, p=0.5, sigma_R=0.05, sigma_t=0.1, seed=3)
    Rrel = np.transpose(g.R_gt[g.ei] @ g.Rm, (0, 2, 1)) @ g.R_gt[g.ej]
    th = np.arccos(np.clip((np.trace(Rrel, axis1=1, axis2=2) - 1) / 2, -1, 1))
    assert abs((th**2).mean() / (3 * 0.05**2) - 1) < 0.1


def test_batched_subset_reproducible():
    a = S.batched(4096, first=7, count=2)
    b = S.batched(4096, first=8, count=1)
    assert np.array_equal(a.graphs[1].tm, b.graphs[0].tm)
    for gr in a.graphs:
        assert 50 <= gr.n <= 5000
        assert gr.ei.max() < gr.n and gr.ej.max() < gr.n and np.all(gr.ei != gr.ej)


def test_random_information_matrices():
    """random_info: symmetric positive definite, eigenvalues tau_e x [aniso^-1/2,
    aniso^1/2], seeded."""
    import pgo_synth as S
    tau = np.linspace(1.0, 100.0, 500)
    A = S.random_info(500, tau, 10.0, seed=3)
    assert A.shape == (500, 3, 3)
    assert np.abs(A - np.transpose(A, (0, 2, 1))).max() <= 1e-12 * np.abs(A).max()
    w = np.linalg.eigvalsh(A) / tau[:, None]
    assert w.min() >= 10.0 ** -0.5 * (1 - 1e-12) and w.max() <= 10.0 ** 0.5 * (1 + 1e-12)
    assert np.array_equal(A, S.random_info(500, tau, 10.0, seed=3))
    iso = S.random_info(20, np.full(20, 7.0), 1.0, seed=1)
    assert np.allclose(iso, 7.0 * np.eye(3), atol=1e-12)
