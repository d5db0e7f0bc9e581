"""C-ABI checks that need no GPU: the library loads, exports every symbol the header
declares, validates arguments before touching the device, and its host-side window
transform (its own double-exponential quadrature) agrees with the oracle's
Gauss-Legendre rule."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blnfft.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2502_07155_amd as bl
    return bl.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    import paper_2502_07155_amd as bl
    assert sorted(bl.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    for s in range(7):
        assert lib.bl_status_string(s).startswith(b"BL_")
    assert b"gfx950" in lib.bl_version()


@pytest.mark.parametrize("M,L,m", [(256, 512, 6), (512, 1024, 5), (128, 256, 4), (40, 80, 5),
                                   (64, 100, 3), (1000, 2000, 8)])
@pytest.mark.parametrize("method", ["shannon", "nfft"])
def test_host_window_transform_matches_oracle_quadrature(M, L, m, method):
    from paper_2502_07155_amd import window_transform
    k = np.arange(M) - M // 2
    beta = O.default_beta(M, L, m, method)
    got = window_transform(k, M, L, m, 0.0, "sinh", method)
    ref = O.psihat1(k, L, m, beta) if method == "shannon" else O.phihat1(k, L, m, beta)
    assert np.max(np.abs(got - ref)) <= 2e-14 * np.max(np.abs(ref))
    got_ckb = window_transform(k, M, L, m, beta, "ckb", method)
    ref_ckb = O.psihat1(k, L, m, beta, "ckb") if method == "shannon" else O.phihat1(k, L, m, beta, "ckb")
    assert np.max(np.abs(got_ckb - ref_ckb)) <= 2e-14 * np.max(np.abs(ref_ckb))


def _create(lib, d=2, M=64, L=128, m=5, win=0, beta=0.0, method=0, prec=2):
    h = ctypes.c_void_p()
    st = lib.bl_plan_create(ctypes.byref(h), d, M, L, m, win, beta, method, prec, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(d=0), 1), (dict(d=4), 1), (dict(M=63), 1), (dict(M=0), 1), (dict(L=127), 1),
    (dict(L=32, M=64), 1), (dict(m=0), 1), (dict(m=64), 1), (dict(win=7), 1),
    (dict(method=3), 1), (dict(prec=9), 1), (dict(beta=float("nan")), 1),
    (dict(m=9, L=256), 6), (dict(L=16384), 6), (dict(d=3, L=2048, M=64), 6),
])
def test_plan_create_rejects_before_device_use(lib, kw, status):
    st, h = _create(lib, **kw)
    assert st == status
    assert h.value is None
    assert len(lib.bl_last_error()) > 0


def _batch_create(lib, spec, prec=1):
    n = len(spec)
    i64 = ctypes.c_int64 * max(n, 1)
    i32 = ctypes.c_int * max(n, 1)
    h = ctypes.c_void_p()
    st = lib.bl_batch_create(ctypes.byref(h), n, i64(*[s[0] for s in spec]), i64(*[s[1] for s in spec]),
                             i32(*[s[2] for s in spec]), i64(*[s[3] for s in spec]), prec, None)
    return st, h


@pytest.mark.parametrize("spec,prec,status", [
    ([], 1, 1),                                            # no instance
    ([(64, 128, 4, 10)], 0, 6),                            # FP64 batches unsupported
    ([(64, 128, 4, 10)], 9, 1),                            # unknown precision
    ([(64, 128, 4, 10), (63, 128, 4, 10)], 1, 1),          # odd M
    ([(64, 64, 4, 10)], 1, 1),                             # L = M: default beta is zero
    ([(64, 130, 4, 10), (64, 127, 4, 10)], 2, 1),          # odd L
    ([(8, 16, 8, 10)], 1, 1),                              # 2m >= L
    ([(64, 128, 4, -1)], 1, 1),                            # negative N
    ([(64, 128, 9, 10)], 1, 6),                            # m above the kernels' range
    ([(64, 128, 1, 10)], 1, 6),                            # m below it
    ([(10000, 24000, 4, 10)], 1, 6),                       # L + M - 1 above 32768
])
def test_batch_create_rejects_before_device_use(lib, spec, prec, status):
    st, h = _batch_create(lib, spec, prec)
    assert st == status
    assert h.value is None
    assert len(lib.bl_last_error()) > 0


def test_batch_calls_with_null_handle(lib):
    assert lib.bl_batch_set_nodes(None, None) == 1
    assert lib.bl_batch_forward(None, None, None) == 1
    assert lib.bl_batch_destroy(None) == 0


def test_calls_with_null_plan(lib):
    assert lib.bl_set_nodes(None, 10, None) == 1
    assert lib.bl_forward(None, None, None) == 1
    assert lib.bl_adjoint(None, None, None) == 1
    assert lib.bl_grad_x(None, None, None) == 1
    assert lib.bl_interpolate(None, None, None) == 1
    assert lib.bl_precompute_weights(None, 1) == 1
    assert lib.bl_plan_destroy(None) == 0


def test_window_transform_argument_checks(lib):
    P = ctypes.POINTER(ctypes.c_double)
    v = (ctypes.c_double * 2)(0.0, 1.0)
    out = (ctypes.c_double * 2)()
    assert lib.bl_window_transform(0, 0, 64, 128, 5, 0.0, 2, v, out) == 0
    assert lib.bl_window_transform(0, 0, 64, 128, 0, 0.0, 2, v, out) == 1
    assert lib.bl_window_transform(0, 0, 64, 128, 5, 0.0, 2, None, out) == 1
    assert lib.bl_window_transform(5, 0, 64, 128, 5, 0.0, 2, v, out) == 1
