"""torch.autograd.Function over K unrolled PRADMM sweeps.

The forward pass runs the sweeps in the HIP library from the handle's
initial point with the given edge parameters; the backward pass is the
library's hand-written adjoint (pgo_adjoint).  Tensors are float64 on the
handle's device.  The library runs on a side stream of its own that first
waits for torch's current stream, and torch's current stream waits for it
before either call returns, so the calls are ordered with surrounding torch
work whichever stream (the legacy default one included) is current.

    state = unrolled_pradmm(graph, kappa, tau, tm, omega, K=50, beta=b, gamma=1.4, C=10)
    loss = ((state[:, 8:11] - t_gt) ** 2).sum()
    loss.backward()        # kappa.grad, tau.grad, tm.grad, omega.grad

state is n x 21: p(4) q(4) t(3) s(3) lambda(4) z(3) after K sweeps.
"""
import torch

from . import (pgo_adjoint, pgo_forward_record, pgo_get_state_dev, pgo_info, pgo_record_id,
               pgo_reset_state, pgo_set_edge_params, pgo_set_stream)


_SIDE = {}


def _enter(h, device):
    cur = torch.cuda.current_stream(device)
    side = _SIDE.get(device.index)
    if side is None:
        side = _SIDE[device.index] = torch.cuda.Stream(device=device)
    side.wait_stream(cur)
    pgo_set_stream(h, side.cuda_stream)
    return cur, side


class UnrolledPRADMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, tau, tm, omega, graph, K, beta, gamma, C):
        h = graph.h
        info = pgo_info(h)
        for name, x, shape in (("kappa", kappa, (info["m"],)), ("tau", tau, (info["m"],)),
                               ("tm", tm, (info["m"], 3)), ("omega", omega, (info["m"], 3))):
            if x.dtype != torch.float64 or not x.is_cuda or tuple(x.shape) != shape:
                raise ValueError(f"{name} must be a float64 CUDA tensor of shape {shape}")
        kappa, tau, tm, omega = (x.contiguous() for x in (kappa, tau, tm, omega))
        state = torch.empty((info["n"], 21), dtype=torch.float64, device=kappa.device)
        cur, side = _enter(h, kappa.device)
        pgo_set_edge_params(h, kappa.data_ptr(), tau.data_ptr(), tm.data_ptr(), omega.data_ptr())
        pgo_reset_state(h)
        pgo_forward_record(h, K, beta, gamma, C)
        pgo_get_state_dev(h, state.data_ptr())
        cur.wait_stream(side)
        ctx.graph = graph
        ctx.m = info["m"]
        ctx.record = pgo_record_id(h)
        return state

    @staticmethod
    def backward(ctx, grad_state):
        h = ctx.graph.h
        if pgo_record_id(h) != ctx.record:
            raise RuntimeError("the handle's recorded forward pass is no longer this one (a later "
                               "forward on the same handle replaced it): run backward before the "
                               "next forward, or use one handle per forward pass")
        dev = grad_state.device
        g = grad_state.contiguous().to(torch.float64)
        gk = torch.empty(ctx.m, dtype=torch.float64, device=dev)
        gt = torch.empty(ctx.m, dtype=torch.float64, device=dev)
        gtm = torch.empty((ctx.m, 3), dtype=torch.float64, device=dev)
        gom = torch.empty((ctx.m, 3), dtype=torch.float64, device=dev)
        cur, side = _enter(h, dev)
        pgo_adjoint(h, g.data_ptr(), gk.data_ptr(), gt.data_ptr(), gtm.data_ptr(), gom.data_ptr(), 0)
        cur.wait_stream(side)
        return gk, gt, gtm, gom, None, None, None, None, None


def unrolled_pradmm(graph, kappa, tau, tm, omega, K, beta, gamma, C=10):
    return UnrolledPRADMM.apply(kappa, tau, tm, omega, graph, K, beta, gamma, C)
