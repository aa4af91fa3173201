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
