"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use this module.  It loads ``liboracle.so`` built from ``iqcc_oracle.cpp`` in
this directory (``build()`` compiles it with g++) and shares no code with the
HIP library.

Every function takes row-major numpy arrays x, z of shape (N, W) (uint64) and
c of shape (N,) (float64); see ``iqcc_oracle.cpp`` for the conventions and the
passages of the paper each function follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "iqcc_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle (g++ -O2, no FP contraction, no fast-math)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ct.CDLL(LIB)
        P = ct.c_void_p
        i64 = ct.c_int64
        L.oracle_pauli_product.restype = ct.c_int
        L.oracle_pauli_product.argtypes = [ct.c_int, ct.c_int, P, P, P, P, P, P]
        L.oracle_dress_raw.restype = i64
        L.oracle_dress_raw.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, ct.c_double, P, P, P]
        L.oracle_dress_raw_tangent.restype = i64
        L.oracle_dress_raw_tangent.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, P,
                                               ct.c_double, ct.c_int, P, P, P, P]
        L.oracle_merge_truncate.restype = i64
        L.oracle_merge_truncate.argtypes = [ct.c_int, i64, P, P, P, P, ct.c_double, P, P, P, P]
        L.oracle_qmf_energy.restype = ct.c_double
        L.oracle_qmf_energy.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P]
        L.oracle_expectations.restype = None
        L.oracle_expectations.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P]
        L.oracle_dis_gradients.restype = None
        L.oracle_dis_gradients.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, i64, P, P, P]
        L.oracle_chain_point.restype = None
        L.oracle_chain_point.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, ct.c_int, P, P, P,
                                         ct.c_double, i64, P, P, P, P]
        L.oracle_dress_step_par.restype = i64
        L.oracle_dress_step_par.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, ct.c_double,
                                            ct.c_double, ct.c_int, P, P, P]
        L.oracle_qmf_energy_par.restype = ct.c_double
        L.oracle_qmf_energy_par.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, ct.c_int]
        L.oracle_qmf_grad_angles.restype = None
        L.oracle_qmf_grad_angles.argtypes = [ct.c_int, ct.c_int, i64, P, P, P, P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def _rows(x, z, c=None):
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    if x.ndim == 1:
        x = x[None, :]
        z = z[None, :]
    if c is not None:
        c = np.ascontiguousarray(c, dtype=np.float64)
    return x, z, c


def pauli_product(nq, x1, z1, x2, z2):
    """P1 P2 = i^e P3 -> (x3, z3, e) for single words (W,)."""
    x1 = np.ascontiguousarray(x1, np.uint64); z1 = np.ascontiguousarray(z1, np.uint64)
    x2 = np.ascontiguousarray(x2, np.uint64); z2 = np.ascontiguousarray(z2, np.uint64)
    W = x1.shape[-1]
    x3 = np.zeros(W, np.uint64); z3 = np.zeros(W, np.uint64)
    e = lib().oracle_pauli_product(nq, W, _p(x1), _p(z1), _p(x2), _p(z2), _p(x3), _p(z3))
    return x3, z3, e


def dress_raw(nq, x, z, c, px, pz, tau):
    """Raw multiset of the dressed terms (no merge)."""
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    px = np.ascontiguousarray(px, np.uint64); pz = np.ascontiguousarray(pz, np.uint64)
    ox = np.zeros((2 * n, W), np.uint64); oz = np.zeros((2 * n, W), np.uint64)
    oc = np.zeros(2 * n, np.float64)
    m = lib().oracle_dress_raw(nq, W, n, _p(x), _p(z), _p(c), _p(px), _p(pz), float(tau),
                               _p(ox), _p(oz), _p(oc))
    return ox[:m], oz[:m], oc[:m]


def merge_truncate(x, z, c, eps=0.0, dc=None):
    """Unique canonical-ordered terms with |c| >= eps (and merged tangent if given)."""
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    ox = np.zeros((n, W), np.uint64); oz = np.zeros((n, W), np.uint64)
    oc = np.zeros(n, np.float64)
    odc = np.zeros(n, np.float64) if dc is not None else None
    if dc is not None:
        dc = np.ascontiguousarray(dc, np.float64)
    m = lib().oracle_merge_truncate(W, n, _p(x), _p(z), _p(c), _p(dc), float(eps),
                                    _p(ox), _p(oz), _p(oc), _p(odc))
    if dc is not None:
        return ox[:m], oz[:m], oc[:m], odc[:m]
    return ox[:m], oz[:m], oc[:m]


def dress(nq, x, z, c, px, pz, tau, eps=0.0):
    """One dressing step: raw dressing, merge, compression."""
    return merge_truncate(*dress_raw(nq, x, z, c, px, pz, tau), eps=eps)


def dress_par(nq, x, z, c, px, pz, tau, eps=0.0, nthreads=1):
    """dress() on `nthreads` host threads: the same terms and coefficients
    (rows grouped by a key-hash partition, canonical inside each)."""
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    px = np.ascontiguousarray(px, np.uint64); pz = np.ascontiguousarray(pz, np.uint64)
    ox = np.empty((max(2 * n, 1), W), np.uint64); oz = np.empty((max(2 * n, 1), W), np.uint64)
    oc = np.empty(max(2 * n, 1), np.float64)
    m = lib().oracle_dress_step_par(nq, W, n, _p(x), _p(z), _p(c), _p(px), _p(pz), float(tau),
                                    float(eps), int(nthreads), _p(ox), _p(oz), _p(oc))
    return ox[:m], oz[:m], oc[:m]


def qmf_energy_par(nq, x, z, c, theta, phi, nthreads=1):
    """qmf_energy() with the per-term products on `nthreads` threads (same value)."""
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    th = np.ascontiguousarray(theta, np.float64); ph = np.ascontiguousarray(phi, np.float64)
    return lib().oracle_qmf_energy_par(nq, W, n, _p(x), _p(z), _p(c), _p(th), _p(ph), int(nthreads))


def chain(nq, x, z, c, ents, taus, eps=0.0, callback=None):
    """Iterated dressing H <- trunc(merge(dress(H, P_j, tau_j)))."""
    for j, ((px, pz), t) in enumerate(zip(ents, taus)):
        x, z, c = dress(nq, x, z, c, px, pz, t, eps)
        if callback is not None:
            callback(j, x, z, c)
    return x, z, c


def qmf_energy(nq, x, z, c, theta, phi):
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    th = np.ascontiguousarray(theta, np.float64); ph = np.ascontiguousarray(phi, np.float64)
    return lib().oracle_qmf_energy(nq, W, n, _p(x), _p(z), _p(c), _p(th), _p(ph))


def expectations(nq, x, z, theta, phi):
    x, z, _ = _rows(x, z)
    n, W = x.shape
    th = np.ascontiguousarray(theta, np.float64); ph = np.ascontiguousarray(phi, np.float64)
    out = np.zeros(n, np.float64)
    lib().oracle_expectations(nq, W, n, _p(x), _p(z), _p(th), _p(ph), _p(out))
    return out


def dis_gradients(nq, x, z, c, theta, phi, cx, cz):
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    cx = np.ascontiguousarray(cx, np.uint64).reshape(-1, W)
    cz = np.ascontiguousarray(cz, np.uint64).reshape(-1, W)
    th = np.ascontiguousarray(theta, np.float64); ph = np.ascontiguousarray(phi, np.float64)
    g = np.zeros(cx.shape[0], np.float64)
    lib().oracle_dis_gradients(nq, W, n, _p(x), _p(z), _p(c), _p(th), _p(ph), cx.shape[0],
                               _p(cx), _p(cz), _p(g))
    return g


def qmf_grad_angles(nq, x, z, c, theta, phi):
    x, z, c = _rows(x, z, c)
    n, W = x.shape
    th = np.ascontiguousarray(theta, np.float64); ph = np.ascontiguousarray(phi, np.float64)
    dt = np.zeros(nq, np.float64); dp = np.zeros(nq, np.float64)
    lib().oracle_qmf_grad_angles(nq, W, n, _p(x), _p(z), _p(c), _p(th), _p(ph), _p(dt), _p(dp))
    return dt, dp


def chain_tau_gradient(nq, x, z, c, ents, taus, eps, theta, phi, k):
    """dE/dtau_k of the iterated dressing with frozen compression masks.

    Forward-mode: a tangent channel dc travels with every coefficient; step k
    contributes the derivative of its cos/sin, later steps rotate dc like c, and
    compression drops a row's tangent together with the row.
    """
    x, z, c = _rows(x, z, c)
    dc = np.zeros_like(c)
    L = lib()
    for j, ((px, pz), t) in enumerate(zip(ents, taus)):
        n, W = x.shape
        px = np.ascontiguousarray(px, np.uint64); pz = np.ascontiguousarray(pz, np.uint64)
        ox = np.zeros((2 * n, W), np.uint64); oz = np.zeros((2 * n, W), np.uint64)
        oc = np.zeros(2 * n); odc = np.zeros(2 * n)
        m = L.oracle_dress_raw_tangent(nq, W, n, _p(x), _p(z), _p(c), _p(dc), _p(px), _p(pz),
                                       float(t), int(j == k), _p(ox), _p(oz), _p(oc), _p(odc))
        x, z, c, dc = merge_truncate(ox[:m], oz[:m], oc[:m], eps=eps, dc=odc[:m])
    ev = expectations(nq, x, z, theta, phi)
    # Neumaier-free: tangent energies are compared at 1e-10 relative
    return float(np.sum(dc * ev)), (x, z, c)


def canonical(x, z, c):
    """Rows in canonical order (x[W-1..0], z[W-1..0] unsigned)."""
    x, z, c = _rows(x, z, c)
    W = x.shape[1]
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)]
    o = np.lexsort(keys)
    return x[o], z[o], c[o]


def truncate_top(x, z, c, max_terms):
    """The max_terms terms of largest |c|; at equal |c| the smaller canonical key
    (x words, then z words, most significant first) comes first.  Rows are
    returned in canonical order."""
    x, z, c = _rows(x, z, c)
    W = x.shape[1]
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)] + [-np.abs(c)]
    o = np.lexsort(keys)[:max(0, int(max_terms))]
    return canonical(x[o], z[o], c[o])


def chain_point(nq, x0, z0, c0, ents, taus, eps, qx, qz):
    """Coefficient of each query key after the whole chain, one key at a time.

    Returns (found: bool array, value: float array).  H0 need not be sorted.
    """
    x0, z0, c0 = canonical(x0, z0, c0)
    W = x0.shape[1]
    K = len(ents)
    px = np.ascontiguousarray(np.array([np.asarray(p, np.uint64).reshape(W) for p, _ in ents]), np.uint64)
    pz = np.ascontiguousarray(np.array([np.asarray(q, np.uint64).reshape(W) for _, q in ents]), np.uint64)
    tt = np.ascontiguousarray(taus, np.float64)
    qx = np.ascontiguousarray(qx, np.uint64).reshape(-1, W)
    qz = np.ascontiguousarray(qz, np.uint64).reshape(-1, W)
    found = np.zeros(qx.shape[0], np.int8)
    val = np.zeros(qx.shape[0], np.float64)
    lib().oracle_chain_point(nq, W, x0.shape[0], _p(x0), _p(z0), _p(c0), K, _p(px), _p(pz), _p(tt),
                             float(eps), qx.shape[0], _p(qx), _p(qz), _p(found), _p(val))
    return found.astype(bool), val
