"""Pin of the oracle's reference adjoint (automatic differentiation through
K unrolled FP64 sweeps) against FP64 central finite differences taken
through the whole input pipeline (rotation perturbed as R~_e Exp(omega_e)
before projection, quaternion conversion and sign alignment)."""
import numpy as np
import torch

import pgo_synth as S
from oracle import prep
from oracle import pradmm as O

F64 = torch.float64


def _loss(g, K, beta, gamma):
    P, p0, t0 = prep.prepare_graph(g)
    return float(O.unrolled_loss(P, p0, t0, K, beta, gamma, torch.as_tensor(g.t_gt)))


def test_V11_adjoint_matches_central_differences():
    g = S.grid(4, 3, 3, all_pairs=True, sigma_R=0.05, sigma_t=0.1, seed=0)
    K, gamma = 10, 1.4
    P, p0, t0 = prep.prepare_graph(g)
    beta = 5.0e2
    L, grads = O.unrolled_grad(P, p0, t0, K, beta, gamma, torch.as_tensor(g.t_gt))
    assert abs(L - _loss(g, K, beta, gamma)) < 1e-12 * L
    rng = np.random.default_rng(0)
    edges = rng.choice(g.m, size=24, replace=False)
    h = 1e-6
    fd = {k: [] for k in ("log_kappa", "log_tau", "omega", "tm")}
    ad = {k: [] for k in fd}

    def perturbed(fn):
        gg = S.Graph(**{k: (v.copy() if isinstance(v, np.ndarray) else v)
                        for k, v in g.__dict__.items()})
        fn(gg)
        return _loss(gg, K, beta, gamma)

    for e in edges:
        def scale(name, f):
            def fn(gg):
                getattr(gg, name)[e] *= f
            return fn
        for name, key in (("kappa", "log_kappa"), ("tau", "log_tau")):
            d = (perturbed(scale(name, np.exp(h))) - perturbed(scale(name, np.exp(-h)))) / (2 * h)
            fd[key].append(d)
            ad[key].append(float(grads[name][e]) * float(getattr(g, name)[e]))
        for c in range(3):
            w = np.zeros(3)
            w[c] = h

            def rot(sign):
                def fn(gg):
                    gg.Rm[e] = gg.Rm[e] @ S.so3_exp(sign * w)[0]
                return fn

            def shift(sign):
                def fn(gg):
                    gg.tm[e, c] += sign * h
                return fn
            fd["omega"].append((perturbed(rot(1)) - perturbed(rot(-1))) / (2 * h))
            ad["omega"].append(float(grads["omega"][e, c]))
            fd["tm"].append((perturbed(shift(1)) - perturbed(shift(-1))) / (2 * h))
            ad["tm"].append(float(grads["tm"][e, c]))
    for k in fd:
        a, f = np.array(ad[k]), np.array(fd[k])
        assert np.linalg.norm(a - f) <= 1e-5 * np.linalg.norm(f), (k, np.linalg.norm(a - f) / np.linalg.norm(f))
