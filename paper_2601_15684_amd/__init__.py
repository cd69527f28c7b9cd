"""PRADMM sweep for SE(3) pose-graph optimisation on MI355X (gfx950).

Thin Python binding of the C ABI in include/pgo.h: every function here has
the C function's name and only marshals arguments (numpy float64/int32
arrays in, numpy arrays out).  All of the method runs in the HIP kernels of
libpgo.so.  The library is loaded on first use; if it has not been built,
that first use raises (build it with ``python -m paper_2601_15684_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "PgoError", "PgoOptions", "lib", "pgo_default_options", "pgo_create", "pgo_create_batched",
    "pgo_set_stream", "pgo_iterate", "pgo_iterate_graphs", "pgo_cost", "pgo_merit", "pgo_evaluate", "pgo_evaluate_noalloc", "pgo_iterate_until", "pgo_solve", "pgo_residuals", "pgo_get_poses",
    "pgo_get_state", "pgo_set_state", "pgo_get_prepared", "pgo_info", "pgo_autotune",
    "pgo_destroy", "pgo_last_error", "PoseGraph", "pgo_set_edge_params", "pgo_reset_state",
    "pgo_get_state_dev", "pgo_forward_record", "pgo_record_id", "pgo_adjoint", "pgo_chordal_init",
    "FP64", "FP32", "SCHED_AUTO", "SCHED_PHASE", "SCHED_GRAPH", "SCHED_COOP", "MODEL_QUAT", "MODEL_CHORDAL",
    "MODEL_QUAT_INFO", "pgo_create_info",
    "LIB_PATH", "split_state",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpgo.so")
FP64, FP32 = 0, 1
SCHED_AUTO, SCHED_PHASE, SCHED_GRAPH, SCHED_COOP = 0, 1, 2, 3
MODEL_QUAT, MODEL_CHORDAL, MODEL_QUAT_INFO = 0, 1, 2
STATE_WIDTH = {MODEL_QUAT: 21, MODEL_CHORDAL: 36, MODEL_QUAT_INFO: 21}
STATUS = {0: "PGO_OK", 1: "PGO_EINVAL", 2: "PGO_ENOMEM", 3: "PGO_EDEVICE", 4: "PGO_ENUMERIC",
          5: "PGO_ESTATE"}


class PgoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class PgoOptions(C.Structure):
    _fields_ = [("h1", C.c_double), ("h2", C.c_double), ("h3", C.c_double), ("h4", C.c_double),
                ("precision", C.c_int32), ("schedule", C.c_int32), ("block", C.c_int32),
                ("device", C.c_int32), ("model", C.c_int32)]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_lib = None

_SIGNATURES = {
    "pgo_default_options": (None, [C.POINTER(PgoOptions)]),
    "pgo_create": (C.c_int, [C.POINTER(_P), C.c_int32, _D, _D, C.c_int64, _I32, _I32, _D, _D, _D, _D,
                             C.POINTER(PgoOptions)]),
    "pgo_create_batched": (C.c_int, [C.POINTER(_P), C.c_int32, _I64, _I64, _D, _D, _I32, _I32, _D, _D,
                                     _D, _D, C.POINTER(PgoOptions)]),
    "pgo_create_info": (C.c_int, [C.POINTER(_P), C.c_int32, _I64, _I64, _D, _D, _I32, _I32, _D, _D,
                                  _D, _D, C.POINTER(PgoOptions)]),
    "pgo_set_stream": (C.c_int, [_P, _P]),
    "pgo_iterate": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double]),
    "pgo_iterate_graphs": (C.c_int, [_P, C.c_int32, _D, C.c_double]),
    "pgo_cost": (C.c_int, [_P, _D]),
    "pgo_merit": (C.c_int, [_P, _D]),
    "pgo_evaluate": (C.c_int, [_P, _D, _D, _D]),
    "pgo_evaluate_noalloc": (C.c_int, [_P, _P, C.c_double, _P]),
    "pgo_iterate_until": (C.c_int, [_P, C.c_int32, C.c_int32, _D, C.c_double, C.c_double, _I32]),
    "pgo_solve": (C.c_int, [_P, C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double, _D, _I32,
                            _I32]),
    "pgo_residuals": (C.c_int, [_P, _D]),
    "pgo_get_poses": (C.c_int, [_P, _D, _D]),
    "pgo_get_state": (C.c_int, [_P, _D]),
    "pgo_set_state": (C.c_int, [_P, _D]),
    "pgo_get_prepared": (C.c_int, [_P, _D, _D]),
    "pgo_info": (C.c_int, [_P, _I64, _I64, _I32, _I32, _I32, _I32, _I32, _I32]),
    "pgo_autotune": (C.c_int, [_P, C.c_double, C.c_double, C.c_int32]),
    "pgo_set_edge_params": (C.c_int, [_P, _P, _P, _P, _P]),
    "pgo_reset_state": (C.c_int, [_P]),
    "pgo_get_state_dev": (C.c_int, [_P, _P]),
    "pgo_forward_record": (C.c_int, [_P, C.c_int32, C.c_double, C.c_double, C.c_int32]),
    "pgo_record_id": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "pgo_adjoint": (C.c_int, [_P, _P, _P, _P, _P, _P, _P]),
    "pgo_chordal_init": (C.c_int, [_P, C.c_int32, C.c_double, _I32]),
    "pgo_destroy": (None, [_P]),
    "pgo_last_error": (C.c_char_p, []),
}


def lib():
    """The loaded libpgo.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2601_15684_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _chk(status):
    if status != 0:
        raise PgoError(status, pgo_last_error())


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(_I32) if a is not None else None


def pgo_last_error() -> str:
    return lib().pgo_last_error().decode()


def pgo_default_options(**kw) -> PgoOptions:
    o = PgoOptions()
    lib().pgo_default_options(C.byref(o))
    for k, v in kw.items():
        if k == "h":
            o.h1, o.h2, o.h3, o.h4 = v
        elif k == "precision" and isinstance(v, str):
            o.precision = {"fp64": FP64, "fp32": FP32}[v]
        elif k == "schedule" and isinstance(v, str):
            o.schedule = {"auto": SCHED_AUTO, "phase": SCHED_PHASE, "graph": SCHED_GRAPH,
                          "coop": SCHED_COOP}[v]
        elif k == "model" and isinstance(v, str):
            o.model = {"quat": MODEL_QUAT, "chordal": MODEL_CHORDAL, "info": MODEL_QUAT_INFO}[v]
        else:
            setattr(o, k, v)
    return o


def pgo_create(n, R0, t0, ei, ej, Rm, tm, kappa, tau, options=None):
    m = int(np.asarray(ei).shape[0])
    arrs = [_f64(R0), _f64(t0), _i32(ei), _i32(ej), _f64(Rm), _f64(tm), _f64(kappa), _f64(tau)]
    h = _P()
    _chk(lib().pgo_create(C.byref(h), int(n), _dp(arrs[0]), _dp(arrs[1]), m, _ip(arrs[2]),
                          _ip(arrs[3]), _dp(arrs[4]), _dp(arrs[5]), _dp(arrs[6]), _dp(arrs[7]),
                          C.byref(options) if options is not None else None))
    return h


def pgo_create_batched(voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, tau, options=None):
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    arrs = [_f64(R0), _f64(t0), _i32(ei), _i32(ej), _f64(Rm), _f64(tm), _f64(kappa), _f64(tau)]
    h = _P()
    _chk(lib().pgo_create_batched(C.byref(h), int(voff.shape[0] - 1), voff.ctypes.data_as(_I64),
                                  eoff.ctypes.data_as(_I64), _dp(arrs[0]), _dp(arrs[1]),
                                  _ip(arrs[2]), _ip(arrs[3]), _dp(arrs[4]), _dp(arrs[5]),
                                  _dp(arrs[6]), _dp(arrs[7]),
                                  C.byref(options) if options is not None else None))
    return h


def pgo_create_info(voff, eoff, R0, t0, ei, ej, Rm, tm, kappa, info, options=None):
    """The quaternion model with a 3x3 translation information matrix per edge
    (info: m x 3 x 3 or m x 9)."""
    voff = np.ascontiguousarray(voff, dtype=np.int64)
    eoff = np.ascontiguousarray(eoff, dtype=np.int64)
    arrs = [_f64(R0), _f64(t0), _i32(ei), _i32(ej), _f64(Rm), _f64(tm), _f64(kappa),
            _f64(info).reshape(-1, 9)]
    h = _P()
    _chk(lib().pgo_create_info(C.byref(h), int(voff.shape[0] - 1), voff.ctypes.data_as(_I64),
                               eoff.ctypes.data_as(_I64), _dp(arrs[0]), _dp(arrs[1]), _ip(arrs[2]),
                               _ip(arrs[3]), _dp(arrs[4]), _dp(arrs[5]), _dp(arrs[6]), _dp(arrs[7]),
                               C.byref(options) if options is not None else None))
    return h


def pgo_set_stream(h, stream):
    _chk(lib().pgo_set_stream(h, C.c_void_p(int(stream)) if stream else None))


def pgo_iterate(h, k, beta, gamma):
    _chk(lib().pgo_iterate(h, int(k), float(beta), float(gamma)))


def pgo_iterate_graphs(h, k, beta, gamma):
    b = _f64(beta)
    G = pgo_info(h)["G"]
    if b.shape != (G,):
        raise ValueError(f"beta must hold one value per graph ({G}), got shape {b.shape}")
    _chk(lib().pgo_iterate_graphs(h, int(k), _dp(b), float(gamma)))


def pgo_info(h):
    n, m = C.c_int64(), C.c_int64()
    G, prec, sched, block, model, lds = (C.c_int32() for _ in range(6))
    _chk(lib().pgo_info(h, C.byref(n), C.byref(m), C.byref(G), C.byref(prec), C.byref(sched),
                        C.byref(block), C.byref(model), C.byref(lds)))
    return dict(n=n.value, m=m.value, G=G.value, precision=prec.value, schedule=sched.value,
                block=block.value, model=model.value, width=STATE_WIDTH[model.value],
                lds=lds.value)


def pgo_cost(h):
    out = np.empty(pgo_info(h)["G"], np.float64)
    _chk(lib().pgo_cost(h, _dp(out)))
    return out


def pgo_merit(h):
    out = np.empty((pgo_info(h)["G"], 2), np.float64)
    _chk(lib().pgo_merit(h, _dp(out)))
    return out


def pgo_evaluate(h):
    """(cost G, residuals G x 6, merit G x 2) from one pass of the reductions."""
    G = pgo_info(h)["G"]
    F, res, mer = np.empty(G), np.empty((G, 6)), np.empty((G, 2))
    _chk(lib().pgo_evaluate(h, _dp(F), _dp(res), _dp(mer)))
    return F, res, mer


def pgo_evaluate_noalloc(h, beta_dev, gamma, out_dev):
    """The reductions of pgo_evaluate into a device buffer without allocating:
    beta_dev (G float64) and out_dev (G x 8 float64) are device pointers
    (e.g. a torch tensor's data_ptr()); enqueued on the handle's stream."""
    _chk(lib().pgo_evaluate_noalloc(h, C.c_void_p(int(beta_dev)), float(gamma),
                                    C.c_void_p(int(out_dev))))


def pgo_iterate_until(h, max_sweeps, check_every, beta, gamma, tol):
    """Sweeps per graph until the residual e < tol (checked every check_every
    sweeps) or max_sweeps; returns the sweeps each graph ran."""
    G = pgo_info(h)["G"]
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (G,)))
    done = np.zeros(G, np.int32)
    _chk(lib().pgo_iterate_until(h, int(max_sweeps), int(check_every), _dp(b), float(gamma),
                                 float(tol), done.ctypes.data_as(C.POINTER(C.c_int32))))
    return done


def pgo_solve(h, max_sweeps, check_every, gamma, tol, beta_growth, beta):
    """Returns (beta reached, accepted sweeps, converged flags), one per graph."""
    G = pgo_info(h)["G"]
    b = np.array(np.broadcast_to(np.asarray(beta, np.float64), (G,)))
    done = np.zeros(G, np.int32)
    conv = np.zeros(G, np.int32)
    _chk(lib().pgo_solve(h, int(max_sweeps), int(check_every), float(gamma), float(tol),
                         float(beta_growth), _dp(b), _ip(done), _ip(conv)))
    return b, done, conv.astype(bool)


def pgo_residuals(h):
    out = np.empty((pgo_info(h)["G"], 6), np.float64)
    _chk(lib().pgo_residuals(h, _dp(out)))
    return out


def pgo_get_poses(h):
    n = pgo_info(h)["n"]
    R = np.empty((n, 3, 3), np.float64)
    t = np.empty((n, 3), np.float64)
    _chk(lib().pgo_get_poses(h, _dp(R), _dp(t)))
    return R, t


def pgo_get_state(h):
    info = pgo_info(h)
    out = np.empty((info["n"], info["width"]), np.float64)
    _chk(lib().pgo_get_state(h, _dp(out)))
    return out


def pgo_set_state(h, state):
    info = pgo_info(h)
    s = _f64(state, (info["n"], info["width"]))
    _chk(lib().pgo_set_state(h, _dp(s)))


def pgo_get_prepared(h):
    """Quaternion model: (m x 4, n x 4) quaternions; chordal: (m x 3 x 3, n x 3 x 3)."""
    info = pgo_info(h)
    shape = (4,) if info["model"] == MODEL_QUAT else (3, 3)
    qe = np.empty((info["m"],) + shape, np.float64)
    p0 = np.empty((info["n"],) + shape, np.float64)
    _chk(lib().pgo_get_prepared(h, _dp(qe), _dp(p0)))
    return qe, p0


def pgo_autotune(h, beta, gamma, sweeps=10):
    _chk(lib().pgo_autotune(h, float(beta), float(gamma), int(sweeps)))
    return pgo_info(h)


def _vp(ptr):
    return C.c_void_p(int(ptr)) if ptr else None


def pgo_set_edge_params(h, kappa_dev=0, tau_dev=0, tm_dev=0, omega_dev=0):
    """Device pointers (ints, e.g. tensor.data_ptr()) of FP64 arrays; 0 keeps a value."""
    _chk(lib().pgo_set_edge_params(h, _vp(kappa_dev), _vp(tau_dev), _vp(tm_dev), _vp(omega_dev)))


def pgo_reset_state(h):
    _chk(lib().pgo_reset_state(h))


def pgo_get_state_dev(h, state_dev):
    _chk(lib().pgo_get_state_dev(h, _vp(state_dev)))


def pgo_forward_record(h, K, beta, gamma, C):
    _chk(lib().pgo_forward_record(h, int(K), float(beta), float(gamma), int(C)))


def pgo_record_id(h):
    """Count of pgo_forward_record calls on the handle, or -1 without a
    valid recording."""
    v = C.c_int64()
    _chk(lib().pgo_record_id(h, C.byref(v)))
    return int(v.value)


def pgo_adjoint(h, dL_dstate_dev, g_kappa=0, g_tau=0, g_tm=0, g_omega=0, dL_dstate0=0):
    _chk(lib().pgo_adjoint(h, _vp(dL_dstate_dev), _vp(g_kappa), _vp(g_tau), _vp(g_tm),
                           _vp(g_omega), _vp(dL_dstate0)))


def pgo_chordal_init(h, max_iters=2000, tol=1e-12):
    """Returns the (G, 2) iteration counts of the rotation and translation solves."""
    G = pgo_info(h)["G"]
    its = np.zeros((G, 2), np.int32)
    _chk(lib().pgo_chordal_init(h, int(max_iters), float(tol), _ip(its)))
    return its


def pgo_destroy(h):
    if h:
        lib().pgo_destroy(h)


def split_state(state):
    """(n,21) state -> dict p, q, t, s, lam, z; (n,36) chordal state ->
    dict P, Q (n,3,3), t, s, L (n,3,3), z."""
    s = np.asarray(state)
    if s.shape[1] == 36:
        n = s.shape[0]
        return dict(P=s[:, 0:9].reshape(n, 3, 3), Q=s[:, 9:18].reshape(n, 3, 3), t=s[:, 18:21],
                    s=s[:, 21:24], L=s[:, 24:33].reshape(n, 3, 3), z=s[:, 33:36])
    return dict(p=s[:, 0:4], q=s[:, 4:8], t=s[:, 8:11], s=s[:, 11:14], lam=s[:, 14:18], z=s[:, 18:21])


class PoseGraph:
    """Owning wrapper of one handle (single graph or batch)."""

    def __init__(self, handle):
        self.h = handle

    @classmethod
    def from_graph(cls, g, info=None, **opt):
        """info (m x 3 x 3): per-edge translation information (information model)."""
        if info is not None:
            return cls(pgo_create_info([0, g.n], [0, g.m], g.R0.reshape(-1, 9), g.t0, g.ei, g.ej,
                                       g.Rm.reshape(-1, 9), g.tm, g.kappa, info,
                                       pgo_default_options(**opt)))
        return cls(pgo_create(g.n, g.R0.reshape(-1, 9), g.t0, g.ei, g.ej, g.Rm.reshape(-1, 9), g.tm,
                              g.kappa, g.tau, pgo_default_options(**opt)))

    @classmethod
    def from_batch(cls, batch, info=None, **opt):
        voff, eoff = batch.offsets()
        c = batch.concat()
        if info is not None:
            return cls(pgo_create_info(voff, eoff, c["R0"].reshape(-1, 9), c["t0"], c["ei"], c["ej"],
                                       c["Rm"].reshape(-1, 9), c["tm"], c["kappa"], info,
                                       pgo_default_options(**opt)))
        return cls(pgo_create_batched(voff, eoff, c["R0"].reshape(-1, 9), c["t0"], c["ei"], c["ej"],
                                      c["Rm"].reshape(-1, 9), c["tm"], c["kappa"], c["tau"],
                                      pgo_default_options(**opt)))

    def iterate(self, k, beta, gamma):
        if np.ndim(beta):
            pgo_iterate_graphs(self.h, k, beta, gamma)
        else:
            pgo_iterate(self.h, k, beta, gamma)

    def cost(self):
        return pgo_cost(self.h)

    def residuals(self):
        return pgo_residuals(self.h)

    def merit(self):
        return pgo_merit(self.h)

    def evaluate(self):
        return pgo_evaluate(self.h)

    def iterate_until(self, max_sweeps, check_every, beta, gamma, tol):
        return pgo_iterate_until(self.h, max_sweeps, check_every, beta, gamma, tol)

    def solve(self, max_sweeps, check_every, gamma, beta, tol=0.0, beta_growth=2.0):
        return pgo_solve(self.h, max_sweeps, check_every, gamma, tol, beta_growth, beta)

    def poses(self):
        return pgo_get_poses(self.h)

    def state(self):
        return pgo_get_state(self.h)

    def set_state(self, s):
        pgo_set_state(self.h, s)

    def prepared(self):
        return pgo_get_prepared(self.h)

    def info(self):
        return pgo_info(self.h)

    def autotune(self, beta, gamma, sweeps=10):
        return pgo_autotune(self.h, beta, gamma, sweeps)

    def set_stream(self, stream):
        pgo_set_stream(self.h, stream)

    def chordal_init(self, max_iters=2000, tol=1e-12):
        return pgo_chordal_init(self.h, max_iters, tol)

    def close(self):
        if self.h:
            pgo_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
