"""The C ABI library: it loads, exports every symbol the header declares, and
rejects invalid arguments on the host (no device work needed)."""
import ctypes as ct
import os
import re

import pytest

from paper_2603_08883_amd import iqcc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iqcc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(iqcc_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(iqcc.LIB_PATH):
        from paper_2603_08883_amd import build
        build.build()
    return iqcc.lib()


def test_header_symbols_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(iqcc.exported_symbols()) | {"iqcc_version"}


def test_version(lib):
    assert iqcc.iqcc_version().startswith("iqcc-gfx950")


def test_null_context_is_rejected(lib):
    P = ct.c_void_p
    assert lib.iqcc_set_param(None, b"anti_cap", 64) == iqcc.IQCC_ERR_INVALID_ARG
    v = ct.c_int64()
    assert lib.iqcc_get_param(None, b"anti_cap", ct.byref(v)) == iqcc.IQCC_ERR_INVALID_ARG
    h = P()
    assert lib.iqcc_store_create(None, 8, 100, ct.byref(h)) == iqcc.IQCC_ERR_INVALID_ARG
    n = ct.c_int64()
    assert lib.iqcc_store_count(None, None, ct.byref(n), None) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_dress(None, None, None, None, 0.1, 0.0, None, None, None, None, None) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_qmf_energy(None, None, None, None, None, None) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_dis_gradients(None, None, None, None, None, None, 0, 0, 0, None, None) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_ctx_create(None, 0) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_ctx_destroy(None) == iqcc.IQCC_OK
    assert lib.iqcc_last_error(None) == b"null context"


def test_no_device_fails_loudly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_ctx_create(0)


def test_bucket_hash_is_linear():
    """The bucket hash the library uses must satisfy h(K ^ P) = h(K) ^ h(P).

    Re-implemented here from its definition (rotations, xors, three xorshift
    rounds) and checked for linearity on random keys."""
    import numpy as np
    rng = np.random.default_rng(0)
    U = np.uint64

    def rotl(v, r):
        return v if r == 0 else ((v << U(r)) | (v >> U(64 - r)))

    def xs(f):
        f ^= f << U(13); f ^= f >> U(7); f ^= f << U(17); return f

    def h(x, z):
        f = np.zeros(x.shape[0], U)
        for w in range(x.shape[1]):
            f ^= rotl(x[:, w], (11 * w) % 64) ^ rotl(z[:, w], (37 + 19 * w) % 64)
        return xs(xs(xs(f))) >> U(32)

    a = rng.integers(0, 2**63, size=(1000, 2), dtype=np.uint64)
    b = rng.integers(0, 2**63, size=(1000, 2), dtype=np.uint64)
    c = rng.integers(0, 2**63, size=(1000, 2), dtype=np.uint64)
    d = rng.integers(0, 2**63, size=(1000, 2), dtype=np.uint64)
    assert np.array_equal(h(a ^ c, b ^ d), h(a, b) ^ h(c, d))


def test_new_entry_points_reject_null_context(lib):
    P = ct.c_void_p
    h = P()
    n = ct.c_int64()
    bad = iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_store_create_ex(None, 8, 100, 0, ct.byref(h)) == bad
    assert lib.iqcc_store_wrap(None, 8, 100, 0, None, 0, ct.byref(h), None) == bad
    assert lib.iqcc_dress_count(None, None, None, None, ct.byref(n), None) == bad
    assert lib.iqcc_dress_inplace(None, None, None, None, 0.1, 0.0, None, None, None, None, None) == bad
    assert lib.iqcc_store_copy(None, None, None, None) == bad
    assert lib.iqcc_store_inplace_stats(None, None, None, None, None, None, None) == bad
    assert lib.iqcc_pauli_products(None, 8, None, None, None, None, 0, 0, None, None, None, None) == bad
    assert lib.iqcc_chain_forward(None, None, 0, None, None, None, 0.0, None, None, None, None) == bad
    assert lib.iqcc_chain_backward(None, None, 0, None, None, None, None, None, None, None,
                                   None, None, None, None, None) == bad


def test_store_bytes_host_only(lib):
    """Sizing is a host computation: it needs no device and checks its arguments."""
    b = iqcc.iqcc_store_bytes
    small, big = b(124, 1000), b(124, 100000)
    assert 0 < small < big
    # the arena dominates: 2 * max_terms rows of (16 W + 8) bytes for W = 2
    assert big >= 2 * 100000 * 40
    # an in-place store: 3.5 * max_terms rows (regions + pool), below 2^31 rows
    assert b(124, 100000, iqcc.IQCC_STORE_INPLACE) >= 1.7 * big
    with pytest.raises(iqcc.IqccError) as e:
        b(124, 1 << 30, iqcc.IQCC_STORE_INPLACE)
    assert e.value.code == iqcc.IQCC_ERR_INVALID_ARG
    assert b(64, 1000) < b(65, 1000)               # one more word per key
    for args in ((0, 100), (8, 0), (8, -5), (8, 1 << 40), (8, 100, 2)):
        with pytest.raises(iqcc.IqccError) as e:
            b(*args)
        assert e.value.code == iqcc.IQCC_ERR_INVALID_ARG
    with pytest.raises(iqcc.IqccError) as e:
        b(257, 100)
    assert e.value.code == iqcc.IQCC_ERR_UNSUPPORTED
    v = ct.c_int64()
    assert lib.iqcc_store_bytes(8, 100, 0, None) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_store_bytes(8, 100, 0, ct.byref(v)) == iqcc.IQCC_OK and v.value % 256 == 0


def test_trig_poly_host_checks(lib):
    import math

    import numpy as np
    coef = np.zeros(3, np.float64)
    tau = np.zeros(1, np.float64)
    e = ct.c_double()
    P = lambda a: a.ctypes.data_as(ct.c_void_p)
    assert lib.iqcc_trig_poly_minimize(0, P(coef), P(tau), 5, ct.byref(e)) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_trig_poly_minimize(9, P(coef), P(tau), 5, ct.byref(e)) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_trig_poly_minimize(1, None, P(tau), 5, ct.byref(e)) == iqcc.IQCC_ERR_INVALID_ARG
    assert lib.iqcc_trig_poly_minimize(1, P(coef), P(tau), -1, ct.byref(e)) == iqcc.IQCC_ERR_INVALID_ARG
    assert math.isnan(lib.iqcc_trig_poly_eval(0, P(coef), P(tau)))
    assert math.isnan(lib.iqcc_trig_poly_eval(1, None, P(tau)))
    # a + b cos + c sin with (a, b, c) = (1, 3, 4): minimum 1 - 5
    coef[:] = (1.0, 3.0, 4.0)
    assert lib.iqcc_trig_poly_minimize(1, P(coef), P(tau), 10, ct.byref(e)) == iqcc.IQCC_OK
    assert abs(e.value - (1.0 - 5.0)) < 1e-14


def test_binding_rejects_bad_arguments_before_any_call(lib):
    """Argument checks of the Python binding run on the host and raise before
    anything reaches the library (so no kernel can see a bad pointer)."""
    import numpy as np
    import torch
    bad = iqcc.IQCC_ERR_INVALID_ARG
    cases = [
        lambda: iqcc._f64(torch.zeros(4, dtype=torch.float32), "theta", 4),   # wrong dtype
        lambda: iqcc._f64(torch.zeros(4, dtype=torch.float64), "theta", 4),   # host memory
        lambda: iqcc._f64(None, "theta", 4),                                 # required
        lambda: iqcc._f64([0.0] * 4, "theta", 4),                            # not a tensor
        lambda: iqcc._dev(torch.zeros(4, dtype=torch.int32), "tape", torch.int64),
        lambda: iqcc._planes(torch.zeros((2, 5), dtype=torch.int32), "x", 2),
        lambda: iqcc._planes(torch.zeros((2, 5), dtype=torch.int64), "x", 2),  # host memory
        lambda: iqcc._words(np.zeros(3, np.uint64), 2),                       # wrong word count
        lambda: iqcc._words(np.zeros(1, np.uint64), 2),
    ]
    for f in cases:
        with pytest.raises(iqcc.IqccError) as e:
            f()
        assert e.value.code == bad
    assert iqcc._f64(None, "dE", 1, optional=True) is None
    w, _ = iqcc._words(np.array([5, 7], np.uint64), 2)
    assert w.tolist() == [5, 7]
