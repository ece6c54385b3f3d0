"""The C-ABI library loads, exports every declared symbol and validates its
arguments on the host (no GPU needed: validation precedes any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1911_10487_amd import flayer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flayer.h")

pytestmark = pytest.mark.skipif(not os.path.exists(flayer.LIB_PATH),
                                reason="libflayer.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fl_[a-z_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "fl_invert" in names and "fl_plan_create" in names
    L = ctypes.CDLL(flayer.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_defaults():
    o = flayer.default_opts()
    assert o.tau == 1.5 and o.eta == 1e-10 and o.precision == 0 and o.px == 0


def _create(nx=32, ny=32, nz=16, nd=16, h=0.125, planes=None, omegas=(2 * np.pi,), c0=1.0,
            **kw):
    L = flayer.lib()
    planes = np.asarray(planes if planes is not None else 2.25 + 0.125 * np.arange(nd), np.float64)
    om = np.asarray(omegas, np.float64)
    o = flayer.default_opts()
    for k, v in kw.items():
        setattr(o, k, v)
    out = ctypes.c_void_p()
    st = L.fl_plan_create(nx, ny, nz, nd, h,
                          planes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          om.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), c0, len(om),
                          ctypes.byref(o), ctypes.byref(out))
    return st, L.fl_last_error().decode(), out


@pytest.mark.parametrize("kw,status,needle", [
    (dict(nx=0), flayer.FL_EINVAL, "sizes"),
    (dict(h=-1.0), flayer.FL_EINVAL, "h must"),
    (dict(c0=0.0), flayer.FL_EINVAL, "c0"),
    (dict(omegas=(0.0,)), flayer.FL_EINVAL, "omegas"),
    (dict(omegas=(np.nan,)), flayer.FL_EINVAL, "omegas"),
    (dict(planes=1.0 + 0.125 * np.arange(16)), flayer.FL_EINVAL, "inside X"),
    (dict(px=40), flayer.FL_EINVAL, "too small"),
    (dict(px=77), flayer.FL_EUNSUPPORTED, "FFT sizes"),
    (dict(nz=160, nd=160, planes=21.0 + 0.125 * np.arange(160)), flayer.FL_EUNSUPPORTED,
     "at most 128"),
    (dict(precision=7), flayer.FL_EUNSUPPORTED, "precision"),
])
def test_invalid_arguments_are_rejected_on_the_host(kw, status, needle):
    st, msg, out = _create(**kw)
    assert st == status, msg
    assert needle in msg
    assert not out.value


def test_null_plan_is_rejected():
    L = flayer.lib()
    assert L.fl_invert(None, None, None, 0.0, None) == flayer.FL_EINVAL
    assert "NULL" in L.fl_last_error().decode()
    L.fl_plan_destroy(None)  # no-op


def test_tuning_calls_reject_null_arguments():
    L = flayer.lib()
    t = flayer.FlTuning()
    assert L.fl_tuning_variants(None) == 0
    assert L.fl_tuning_get(None, ctypes.byref(t)) == flayer.FL_EINVAL
    assert L.fl_tuning_set(None, ctypes.byref(t)) == flayer.FL_EINVAL
    i = ctypes.c_int()
    assert L.fl_tuning_describe(None, 0, ctypes.byref(i), ctypes.byref(i),
                                ctypes.byref(i)) == flayer.FL_EINVAL
    assert L.fl_plan_tune(None, None, None, 0.0, 1, None, None) == flayer.FL_EINVAL


def test_closed_form_kernel_needs_damping_on_the_k0_circle():
    # 32x32x16 on the 64^2 torus, h = 0.125, omega = 2 pi: k0 / (2 pi / (64 h))
    # = 8, so the wavenumber (8, 0) lies on |k| = k0 and gamma = 0 there
    st, msg, out = _create(kernel_mode=1, damping=0.0)
    assert st == flayer.FL_ENUMERIC, msg
    assert "gamma = 0" in msg and not out.value
    st, msg, out = _create(kernel_mode=2)
    assert st == flayer.FL_EINVAL and "kernel_mode" in msg
    st, msg, out = _create(kernel_mode=1, damping=-1.0)
    assert st == flayer.FL_EINVAL and "damping" in msg


def test_alpha_rule_is_validated():
    st, msg, out = _create(alpha_rule=3)
    assert st == flayer.FL_EINVAL and "alpha_rule" in msg and not out.value
    # one alpha per wavenumber over the frequencies: shared factorizations,
    # Tikhonov, at most 8 frequencies
    for kw in (dict(factor_per_system=1), dict(prefactor=1), dict(regularizer=1),
               dict(omegas=np.linspace(1.0, 9.0, 9))):
        st, msg, out = _create(alpha_rule=2, **kw)
        assert st == flayer.FL_EUNSUPPORTED and "alpha_rule 2" in msg and not out.value, kw


def test_forward_method_is_validated():
    st, msg, out = _create(forward_method=2)
    assert st == flayer.FL_EINVAL and "forward_method" in msg and not out.value


def test_prefactor_is_validated():
    st, msg, out = _create(prefactor=2)
    assert st == flayer.FL_EINVAL and "prefactor" in msg and not out.value
    st, msg, out = _create(prefactor=1, factor_per_system=1)
    assert st == flayer.FL_EUNSUPPORTED and "prefactor" in msg and not out.value
    st, msg, out = _create(prefactor=1, alpha_rule=1)
    assert st == flayer.FL_EUNSUPPORTED and not out.value


def test_thin_layer_validation():
    # two planes 0.01 apart (off the lattice) form a thin layer: the host
    # checks refuse what it does not support before any device work
    thin = 3.0 + 0.01 * np.arange(2)
    st, msg, out = _create(nd=2, planes=thin, alpha_rule=1)
    assert st == flayer.FL_EUNSUPPORTED and "thin" in msg and not out.value
    st, msg, out = _create(nd=2, planes=thin, prefactor=1)
    assert st == flayer.FL_EUNSUPPORTED and not out.value
    st, msg, out = _create(nd=2, planes=np.array([-1.0, 3.0]))
    assert st == flayer.FL_EINVAL and "straddle" in msg
    # a general plane set (off the lattice, or nd != nz) is padded to a solver
    # size of at most 128
    st, msg, out = _create(nd=130, planes=3.0 + 0.01 * np.arange(130))
    assert st == flayer.FL_EUNSUPPORTED and "at most 128" in msg and not out.value


def test_tsvd_validation():
    # square systems (any supported nz): TSVD runs on the per-call orbit
    # factorizations only
    for kw in (dict(factor_per_system=1), dict(alpha_rule=1), dict(prefactor=1)):
        st, msg, out = _create(regularizer=1, **kw)
        assert st == flayer.FL_EUNSUPPORTED and "TSVD" in msg and not out.value, kw
    st, msg, out = _create(regularizer=3)
    assert st == flayer.FL_EINVAL and "regularizer" in msg


def test_binding_refuses_host_and_misshaped_tensors():
    # the argument checks run before any library call (no GPU needed)
    import torch
    t = torch.zeros((2, 3), dtype=torch.complex128)
    with pytest.raises(ValueError, match="GPU"):
        flayer._need("W", t, (2, 3), (torch.complex128,))
    with pytest.raises(TypeError):
        flayer._need("W", np.zeros((2, 3)), (2, 3), (torch.complex128,))


def test_vertical_cell_size_is_validated():
    for hz in (-0.1, float("nan"), float("inf")):
        st, msg, out = _create(hz=hz)
        assert st == flayer.FL_EINVAL and "hz" in msg and not out.value
    # planes inside X = [0, nz hz] are refused with the vertical size
    st, msg, out = _create(hz=0.2, planes=2.25 + 0.125 * np.arange(16))
    assert st == flayer.FL_EINVAL and "inside X" in msg
