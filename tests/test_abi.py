"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/pgo.h declares, and rejects invalid arguments before
touching a device."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pgo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pgo_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("pgo_create", "pgo_iterate", "pgo_cost", "pgo_residuals", "pgo_create_batched",
                 "pgo_get_state", "pgo_set_state", "pgo_destroy", "pgo_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol(pgo):
    L = pgo.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing


def test_default_options(pgo):
    o = pgo.pgo_default_options()
    assert (o.h1, o.h2, o.h3, o.h4) == (1.0, 1e-3, 1e-3, 1e-3)
    assert o.precision == pgo.FP64 and o.schedule == pgo.SCHED_AUTO and o.device == 0
    assert o.model == pgo.MODEL_QUAT


def _tiny():
    R = np.tile(np.eye(3).reshape(1, 9), (3, 1))
    t = np.zeros((3, 3))
    ei = np.array([0, 1], np.int32)
    ej = np.array([1, 2], np.int32)
    Rm = np.tile(np.eye(3).reshape(1, 9), (2, 1))
    tm = np.ones((2, 3))
    return dict(n=3, R0=R, t0=t, ei=ei, ej=ej, Rm=Rm, tm=tm, kappa=np.ones(2), tau=np.ones(2))


def _expect_einval(pgo, fn, match):
    with pytest.raises(pgo.PgoError) as ex:
        fn()
    assert ex.value.name == "PGO_EINVAL"
    assert match in str(ex.value)


@pytest.mark.parametrize("mutate,match", [
    (lambda a: a.update(n=0), "n must be"),
    (lambda a: a["ei"].__setitem__(0, 5), "out of range"),
    (lambda a: a["ej"].__setitem__(1, 1), "self-loop"),
    (lambda a: a["kappa"].__setitem__(0, 0.0), "kappa or tau"),
    (lambda a: a["tau"].__setitem__(1, np.nan), "kappa or tau"),
    (lambda a: a["R0"].__setitem__((0, 0), np.inf), "non-finite"),
    (lambda a: a["tm"].__setitem__((0, 0), np.nan), "non-finite"),
])
def test_create_rejects_invalid_input(pgo, mutate, match):
    a = _tiny()
    mutate(a)
    _expect_einval(pgo, lambda: pgo.pgo_create(a["n"], a["R0"], a["t0"], a["ei"], a["ej"], a["Rm"],
                                               a["tm"], a["kappa"], a["tau"]), match)


@pytest.mark.parametrize("kw,match", [
    (dict(h=(0.0, 1e-3, 1e-3, 1e-3)), "proximal"),
    (dict(precision=7), "precision"),
    (dict(block=100), "block"),
    (dict(schedule=9), "schedule"),
    (dict(model=5), "model"),
])
def test_create_rejects_invalid_options(pgo, kw, match):
    a = _tiny()
    o = pgo.pgo_default_options(**kw)
    _expect_einval(pgo, lambda: pgo.pgo_create(a["n"], a["R0"], a["t0"], a["ei"], a["ej"], a["Rm"],
                                               a["tm"], a["kappa"], a["tau"], o), match)


def test_batched_offsets_validated(pgo):
    a = _tiny()
    args = (a["R0"], a["t0"], a["ei"], a["ej"], a["Rm"], a["tm"], a["kappa"], a["tau"])
    _expect_einval(pgo, lambda: pgo.pgo_create_batched([1, 3], [0, 2], *args), "voff[0]")
    _expect_einval(pgo, lambda: pgo.pgo_create_batched([0, 0, 3], [0, 0, 2], *args), "no pose")
    _expect_einval(pgo, lambda: pgo.pgo_create_batched([0, 1, 3], [0, 2, 2], *args), "out of range")


def test_null_handle_calls(pgo):
    import ctypes as C
    lib = pgo.lib()
    buf = (C.c_double * 8)()
    for fn in (lambda: pgo.pgo_iterate(None, 1, 1.0, 1.0), lambda: pgo.pgo_set_stream(None, 0)):
        with pytest.raises(pgo.PgoError):
            fn()
    # every reduction entry point refuses a null handle before touching a device
    for call in (lambda: lib.pgo_cost(None, buf), lambda: lib.pgo_residuals(None, buf),
                 lambda: lib.pgo_merit(None, buf), lambda: lib.pgo_evaluate(None, buf, buf, buf),
                 lambda: lib.pgo_evaluate(None, None, None, None),
                 lambda: lib.pgo_iterate_until(None, 20, 10, buf, 1.4, 1e-3,
                                               (C.c_int32 * 8)())):
        assert call() == 1  # PGO_EINVAL
    pgo.pgo_destroy(None)


@pytest.mark.parametrize("mutate,match", [
    (lambda S: S.__setitem__((0, 1), S[0, 1] + 1.0), "not symmetric"),
    (lambda S: S.__setitem__((1, slice(None)), -S[1]), "not positive definite"),
    (lambda S: S.__setitem__((0, 4), np.nan), "not finite"),
])
def test_create_info_rejects_bad_information(pgo, mutate, match):
    a = _tiny()
    S = np.tile(np.eye(3).reshape(1, 9), (2, 1))
    mutate(S)
    _expect_einval(pgo, lambda: pgo.pgo_create_info([0, 3], [0, 2], a["R0"], a["t0"], a["ei"], a["ej"],
                                                    a["Rm"], a["tm"], a["kappa"], S), match)


def test_information_model_needs_its_own_constructor(pgo):
    a = _tiny()
    o = pgo.pgo_default_options(model="info")
    _expect_einval(pgo, lambda: pgo.pgo_create(a["n"], a["R0"], a["t0"], a["ei"], a["ej"], a["Rm"],
                                               a["tm"], a["kappa"], a["tau"], o), "pgo_create_info")
    o = pgo.pgo_default_options(block=512)
    S = np.tile(np.eye(3).reshape(1, 9), (2, 1))
    _expect_einval(pgo, lambda: pgo.pgo_create_info([0, 3], [0, 2], a["R0"], a["t0"], a["ei"], a["ej"],
                                                    a["Rm"], a["tm"], a["kappa"], S, o), "256")
