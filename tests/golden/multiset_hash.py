"""Order-independent 64-bit digest of a set of terms (test infrastructure).

digest(term) folds the words x[0..W-1], z[0..W-1] and the IEEE bits of the
coefficient (with -0.0 read as +0.0, since coefficients compare by value)
through the splitmix64 finaliser; the digest of a term set is the sum of the
term digests modulo 2^64, so it does not depend on row order.  Two sets with
the same digest are, for test purposes, the same set of (key, coefficient)
pairs.  The numpy form is the definition; the torch form computes the same
value on a device (signed int64 with wrap-around) and is checked against it.
"""
from __future__ import annotations

import numpy as np

_SEED = 0x9E3779B97F4A7C15
_C1 = 0xBF58476D1CE4E5B9
_C2 = 0x94D049BB133111EB
_M64 = (1 << 64) - 1


def _coef_bits_np(c):
    c = np.ascontiguousarray(c, np.float64)
    bits = c.view(np.uint64).copy()
    bits[c == 0.0] = 0
    return bits


def _mix_np(v):
    v = v ^ (v >> np.uint64(30))
    v = v * np.uint64(_C1)
    v = v ^ (v >> np.uint64(27))
    v = v * np.uint64(_C2)
    return v ^ (v >> np.uint64(31))


def multiset_hash(x, z, c) -> int:
    """x, z: (N, W) uint64 rows; c: (N,) float64.  Returns an int in [0, 2^64)."""
    x = np.ascontiguousarray(x, np.uint64)
    z = np.ascontiguousarray(z, np.uint64)
    if x.ndim == 1:
        x = x[:, None]; z = z[:, None]
    n, W = x.shape
    if n == 0:
        return 0
    with np.errstate(over="ignore"):
        acc = np.full(n, _SEED, np.uint64)
        for w in range(W):
            acc = _mix_np(acc ^ x[:, w])
        for w in range(W):
            acc = _mix_np(acc ^ z[:, w])
        acc = _mix_np(acc ^ _coef_bits_np(c))
        return int(np.add.reduce(acc, dtype=np.uint64))


def _s64(v):
    return v - (1 << 64) if v >= (1 << 63) else v


def _mix_t(v):
    import torch
    def shr(a, k):   # logical shift right of int64 bit patterns
        return torch.bitwise_and(torch.bitwise_right_shift(a, k), (1 << (64 - k)) - 1)
    v = torch.bitwise_xor(v, shr(v, 30))
    v = v * _s64(_C1)
    v = torch.bitwise_xor(v, shr(v, 27))
    v = v * _s64(_C2)
    return torch.bitwise_xor(v, shr(v, 31))


def multiset_hash_torch(x, z, c, chunk: int = 1 << 24) -> int:
    """Same digest for torch tensors: x, z as (W, N) int64 word planes, c (N,)
    float64, on any device."""
    import torch
    W, n = x.shape
    total = 0
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        cb = c[s:e].contiguous().view(torch.int64)
        cb = torch.where(c[s:e] == 0.0, torch.zeros_like(cb), cb)
        acc = torch.full((e - s,), _s64(_SEED), dtype=torch.int64, device=x.device)
        for w in range(W):
            acc = _mix_t(torch.bitwise_xor(acc, x[w, s:e]))
        for w in range(W):
            acc = _mix_t(torch.bitwise_xor(acc, z[w, s:e]))
        acc = _mix_t(torch.bitwise_xor(acc, cb))
        total = (total + int(acc.sum().item())) & _M64
    return total
