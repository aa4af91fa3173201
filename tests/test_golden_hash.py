"""The device form of the multiset digest equals its numpy definition, and the
digest is order-independent and sensitive to keys and coefficient bits."""
import numpy as np
import torch

from tests.golden.multiset_hash import multiset_hash, multiset_hash_torch


def _rows(n, W, seed):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2**63, size=(n, W), dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=(n, W), dtype=np.uint64)
    z = rng.integers(0, 2**63, size=(n, W), dtype=np.uint64)
    c = rng.normal(size=n)
    return x, z, c


def test_torch_digest_equals_numpy_definition():
    for W in (1, 2, 3):
        x, z, c = _rows(5000, W, W)
        c[:7] = 0.0
        c[7:9] = -0.0
        h = multiset_hash(x, z, c)
        tx = torch.from_numpy(x.T.copy().view(np.int64))
        tz = torch.from_numpy(z.T.copy().view(np.int64))
        assert multiset_hash_torch(tx, tz, torch.from_numpy(c), chunk=777) == h


def test_digest_is_order_independent_and_sensitive():
    x, z, c = _rows(2000, 2, 11)
    h = multiset_hash(x, z, c)
    p = np.random.default_rng(3).permutation(len(c))
    assert multiset_hash(x[p], z[p], c[p]) == h
    c2 = c.copy(); c2[5] = np.nextafter(c2[5], np.inf)
    assert multiset_hash(x, z, c2) != h
    x2 = x.copy(); x2[9, 1] ^= np.uint64(1 << 40)
    assert multiset_hash(x2, z, c) != h
    c3 = c.copy(); c3[[1, 2]] = c3[[2, 1]]          # coefficients swapped between keys
    assert multiset_hash(x, z, c3) != h
    c4 = c.copy(); c4[0] = 0.0
    c5 = c.copy(); c5[0] = -0.0
    assert multiset_hash(x, z, c4) == multiset_hash(x, z, c5)
    assert multiset_hash(x[:0], z[:0], c[:0]) == 0
