"""Python binding of libiqcc (argument marshalling only).

Each function carries the name of the C entry point it wraps (include/iqcc.h)
and forwards torch tensors as raw device pointers; every step of the
computation runs in the HIP library.  There is no fallback: if libiqcc.so is
missing or no GPU is present the calls raise.

Tensor conventions: Pauli words are int64 tensors of shape (W, n) on the GPU
(the bits of uint64 words, word-major planes, leading dimension n); real
coefficients, angles and gradients are float64 tensors.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IQCC_LIB points the binding at another build of the library (developer override)
LIB_PATH = os.environ.get("IQCC_LIB", os.path.join(HERE, "libiqcc.so"))

IQCC_OK = 0
IQCC_ERR_INVALID_ARG = -1
IQCC_ERR_CAPACITY = -2
IQCC_ERR_HIP = -3
IQCC_ERR_UNSUPPORTED = -4
IQCC_DIS_BATCHED = 0
IQCC_DIS_PLAIN = 1
IQCC_STORE_INPLACE = 1
NOALLOC_MAX_PARTIALS = 8192   # workgroup partials the allocation-free energy holds

_lib = None


class IqccError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"iqcc error {code}: {msg}")
        self.code = code


def lib():
    """Load libiqcc.so (built in-tree by paper_2603_08883_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2603_08883_amd.build`")
    # PyTorch brings its own HIP runtime; load it first so that libiqcc binds to
    # the same runtime instance (a second runtime loaded earlier under the same
    # soname would be picked up by torch instead and hide the devices from it).
    import torch  # noqa: F401
    L = ct.CDLL(LIB_PATH)
    P, i64, i32, d = ct.c_void_p, ct.c_int64, ct.c_int, ct.c_double
    sig = {
        "iqcc_version": (ct.c_char_p, []),
        "iqcc_last_error": (ct.c_char_p, [P]),
        "iqcc_ctx_create": (i32, [ct.POINTER(P), i32]),
        "iqcc_ctx_destroy": (i32, [P]),
        "iqcc_set_param": (i32, [P, ct.c_char_p, i64]),
        "iqcc_get_param": (i32, [P, ct.c_char_p, ct.POINTER(i64)]),
        "iqcc_store_create": (i32, [P, i32, i64, ct.POINTER(P)]),
        "iqcc_store_create_ex": (i32, [P, i32, i64, ct.c_uint32, ct.POINTER(P)]),
        "iqcc_store_bytes": (i32, [i32, i64, ct.c_uint32, ct.POINTER(i64)]),
        "iqcc_store_wrap": (i32, [P, i32, i64, ct.c_uint32, P, i64, ct.POINTER(P), P]),
        "iqcc_dress_count": (i32, [P, P, P, P, ct.POINTER(i64), P]),
        "iqcc_pauli_products": (i32, [P, i32, P, P, P, P, i64, i64, P, P, P, P]),
        "iqcc_chain_forward": (i32, [P, P, i32, P, P, P, d, P, P, P, P]),
        "iqcc_chain_backward": (i32, [P, P, i32, P, P, P, P, P, P, P, P, P, P, P, P]),
        "iqcc_store_destroy": (i32, [P, P]),
        "iqcc_store_shape": (i32, [P, ct.POINTER(i32), ct.POINTER(i32)]),
        "iqcc_store_load": (i32, [P, P, P, P, P, i64, i64, P]),
        "iqcc_store_count": (i32, [P, P, ct.POINTER(i64), P]),
        "iqcc_store_export": (i32, [P, P, P, P, P, i64, i64, ct.POINTER(i64), P]),
        "iqcc_store_stats": (i32, [P, P, ct.POINTER(i64), ct.POINTER(i64), P]),
        "iqcc_store_sum_squares": (i32, [P, P, P, P]),
        "iqcc_store_lookup": (i32, [P, P, P, P, i64, i64, P, P, P]),
        "iqcc_dress": (i32, [P, P, P, P, d, d, P, P, P, P, P]),
        "iqcc_dress_energy_update": (i32, [P, P, P, P, d, d, P, P, P, P, P, P]),
        "iqcc_dress_inplace": (i32, [P, P, P, P, d, d, P, P, P, P, P]),
        "iqcc_store_copy": (i32, [P, P, P, P]),
        "iqcc_store_inplace_stats": (i32, [P, P, ct.POINTER(i64), ct.POINTER(i64), ct.POINTER(i64),
                                           ct.POINTER(i64), P]),
        "iqcc_dress_raw": (i32, [P, i32, P, P, P, i64, i64, P, P, d, P, P, P, P, i64, P]),
        "iqcc_merge_truncate": (i32, [P, P, P, P, i64, i64, d, P, P]),
        "iqcc_qmf_energy": (i32, [P, P, P, P, P, P]),
        "iqcc_qmf_energy_noalloc": (i32, [P, P, P, P, P, P]),
        "iqcc_qmf_energy_backward": (i32, [P, P, P, P, P, P, P, P, P]),
        "iqcc_dis_gradients": (i32, [P, P, P, P, P, P, i64, i64, i32, P, P]),
        "iqcc_store_rows": (i32, [P, ct.POINTER(i64)]),
        "iqcc_dress_taped": (i32, [P, P, P, P, d, d, P, P, P, P]),
        "iqcc_dress_backward": (i32, [P, P, P, P, d, P, P, P, P, P, P]),
        "iqcc_expectations": (i32, [P, P, P, P, P, P, P]),
        "iqcc_dress_batched": (i32, [P, i32, P, P, P, P, P, d, P]),
        "iqcc_batch_create": (i32, [P, i32, P, P, P, P, P, d, ct.POINTER(P)]),
        "iqcc_batch_launch": (i32, [P, P, P]),
        "iqcc_batch_destroy": (i32, [P, P]),
        "iqcc_qmf_energy_anti": (i32, [P, P, P, P, P, P, P, P]),
        "iqcc_truncate_top": (i32, [P, P, i64, P, P]),
        "iqcc_energy_trig_poly": (i32, [P, P, i32, P, P, P, P, P, P]),
        "iqcc_trig_poly_eval": (d, [i32, P, P]),
        "iqcc_trig_poly_minimize": (i32, [i32, P, P, i32, ct.POINTER(d)]),
        "iqcc_sortless_dress": (i32, [P, i32, P, P, P, i64, i64, P, P, d, d, P, P, P, i64, i64,
                                      ct.POINTER(i64), P]),
        "iqcc_flip_sets": (i32, [P, P, i32, P, i64, ct.POINTER(i64)]),
        "iqcc_qcc_iteration": (i32, [P, ct.POINTER(P), ct.POINTER(P), P, P, i32, i32, d, P, P, P, P, P,
                                     ct.POINTER(i64), ct.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    return [
        "iqcc_version", "iqcc_last_error", "iqcc_ctx_create", "iqcc_ctx_destroy",
        "iqcc_set_param", "iqcc_get_param", "iqcc_store_create", "iqcc_store_destroy",
        "iqcc_store_create_ex", "iqcc_store_bytes", "iqcc_store_wrap", "iqcc_dress_count",
        "iqcc_pauli_products", "iqcc_chain_forward", "iqcc_chain_backward",
        "iqcc_store_shape", "iqcc_store_load", "iqcc_store_count", "iqcc_store_export",
        "iqcc_store_stats", "iqcc_store_sum_squares", "iqcc_store_lookup",
        "iqcc_dress", "iqcc_dress_energy_update", "iqcc_dress_inplace", "iqcc_store_copy",
        "iqcc_store_inplace_stats", "iqcc_dress_raw", "iqcc_merge_truncate", "iqcc_qmf_energy",
        "iqcc_qmf_energy_noalloc", "iqcc_qmf_energy_backward", "iqcc_dis_gradients", "iqcc_store_rows",
        "iqcc_dress_taped", "iqcc_dress_backward", "iqcc_expectations",
        "iqcc_dress_batched", "iqcc_batch_create", "iqcc_batch_launch", "iqcc_batch_destroy",
        "iqcc_qmf_energy_anti", "iqcc_flip_sets", "iqcc_qcc_iteration", "iqcc_truncate_top",
        "iqcc_sortless_dress", "iqcc_energy_trig_poly", "iqcc_trig_poly_eval",
        "iqcc_trig_poly_minimize",
    ]


def _check(rc, ctx):
    if rc != IQCC_OK:
        msg = lib().iqcc_last_error(ctx).decode() if ctx else ""
        raise IqccError(rc, msg)


def _stream(stream):
    if stream is None:
        import torch
        return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ct.c_void_p(int(stream))


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _bad(msg):
    raise IqccError(IQCC_ERR_INVALID_ARG, msg)


def _dev(t, name, dtype, min_numel=1, optional=False):
    """Device pointer of a contiguous CUDA tensor of `dtype` with at least
    min_numel elements (None passes through when optional)."""
    import torch
    if t is None:
        if optional:
            return None
        _bad(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        _bad(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        _bad(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        _bad(f"{name} must be on the GPU")
    if not t.is_contiguous():
        _bad(f"{name} must be contiguous")
    if t.numel() < min_numel:
        _bad(f"{name} needs at least {min_numel} elements, has {t.numel()}")
    return ct.c_void_p(t.data_ptr())


def _f64(t, name, min_numel=1, optional=False):
    import torch
    return _dev(t, name, torch.float64, min_numel, optional)


def _planes(t, name, W):
    """(W, n) int64 word planes on the GPU, each plane contiguous: (pointer, n, ld)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int64 or not t.is_cuda:
        _bad(f"{name} must be an int64 GPU tensor of shape (W, n)")
    if t.dim() != 2 or t.shape[0] != W:
        _bad(f"{name} must have shape ({W}, n), got {tuple(t.shape)}")
    if t.shape[1] > 0 and (t.stride(1) != 1 or t.stride(0) < t.shape[1]):
        _bad(f"{name} planes must be contiguous rows")
    ld = int(t.stride(0)) if t.shape[1] > 0 else 1
    return ct.c_void_p(t.data_ptr()), int(t.shape[1]), ld


def _words(a, W=None):
    """uint64 numpy words of a host Pauli key (exactly W words) for the entangler argument."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64).reshape(-1))
    if W is not None and a.size != W:
        _bad(f"a Pauli key of this store has {W} words, got {a.size}")
    return a, a.ctypes.data_as(ct.c_void_p)


def _nq(store):
    return iqcc_store_shape(store)


def _angles(store, theta, phi, optional=False):
    nq, _ = _nq(store)
    return (_f64(theta, "theta", nq, optional), _f64(phi, "phi", nq, optional))


# ---------------------------------------------------------------------------
# one wrapper per C entry point
# ---------------------------------------------------------------------------

def iqcc_version():
    return lib().iqcc_version().decode()


def iqcc_ctx_create(device: int = 0):
    h = ct.c_void_p()
    rc = lib().iqcc_ctx_create(ct.byref(h), int(device))
    if rc != IQCC_OK:
        raise IqccError(rc, "iqcc_ctx_create failed (no usable HIP device?)")
    return h


def iqcc_ctx_destroy(ctx):
    _check(lib().iqcc_ctx_destroy(ctx), None)


def iqcc_set_param(ctx, name: str, value: int):
    _check(lib().iqcc_set_param(ctx, name.encode(), int(value)), ctx)


def iqcc_get_param(ctx, name: str) -> int:
    v = ct.c_int64()
    _check(lib().iqcc_get_param(ctx, name.encode(), ct.byref(v)), ctx)
    return v.value


def iqcc_store_create(ctx, n_qubits: int, max_terms: int, flags: int = 0):
    h = ct.c_void_p()
    _check(lib().iqcc_store_create_ex(ctx, int(n_qubits), int(max_terms), int(flags), ct.byref(h)), ctx)
    return h


def iqcc_store_bytes(n_qubits: int, max_terms: int, flags: int = 0) -> int:
    b = ct.c_int64()
    rc = lib().iqcc_store_bytes(int(n_qubits), int(max_terms), int(flags), ct.byref(b))
    if rc != IQCC_OK:
        raise IqccError(rc, "invalid store parameters")
    return b.value


def iqcc_store_wrap(ctx, n_qubits: int, max_terms: int, flags: int, mem, stream=None):
    """Store inside caller-owned device memory `mem` (a uint8 CUDA tensor)."""
    import torch
    p = _dev(mem, "mem", torch.uint8, 1)
    h = ct.c_void_p()
    _check(lib().iqcc_store_wrap(ctx, int(n_qubits), int(max_terms), int(flags), p, int(mem.numel()),
                                 ct.byref(h), _stream(stream)), ctx)
    return h


def iqcc_store_destroy(ctx, store):
    _check(lib().iqcc_store_destroy(ctx, store), ctx)


def iqcc_store_shape(store):
    nq, W = ct.c_int(), ct.c_int()
    _check(lib().iqcc_store_shape(store, ct.byref(nq), ct.byref(W)), None)
    return nq.value, W.value


def iqcc_store_load(ctx, store, x, z, c, stream=None):
    """x, z: int64 (W, n) device tensors; c: float64 (n,) device tensor."""
    _, W = _nq(store)
    px, n, ld = _planes(x, "x", W)
    pz, nz, ldz = _planes(z, "z", W)
    if nz != n or ldz != ld:
        _bad("x and z must have the same shape and layout")
    pc = _f64(c, "c", n, optional=(n == 0))
    if c is not None and c.numel() != n:
        _bad("c must have one coefficient per row")
    _check(lib().iqcc_store_load(ctx, store, px, pz, pc, n, ld, _stream(stream)), ctx)


def iqcc_store_count(ctx, store, stream=None) -> int:
    n = ct.c_int64()
    _check(lib().iqcc_store_count(ctx, store, ct.byref(n), _stream(stream)), ctx)
    return n.value


def iqcc_store_sum_squares(ctx, store, out=None, stream=None):
    """Sum of c^2 over the live terms (float64 device scalar; `out` optional)."""
    import torch
    if out is None:
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
    _check(lib().iqcc_store_sum_squares(ctx, store, _f64(out, "out", 1), _stream(stream)), ctx)
    return out


def iqcc_store_stats(ctx, store, stream=None):
    """(anticommuting input terms, new output terms) of the step that produced store."""
    a, b = ct.c_int64(), ct.c_int64()
    _check(lib().iqcc_store_stats(ctx, store, ct.byref(a), ct.byref(b), _stream(stream)), ctx)
    return a.value, b.value


def iqcc_store_lookup(ctx, store, qx, qz, stream=None):
    """qx, qz: int64 (W, n) device tensors -> (found bool, value float64) device tensors."""
    import torch
    _, W = _nq(store)
    px, n, ld = _planes(qx, "qx", W)
    pz, nz, ldz = _planes(qz, "qz", W)
    if nz != n or ldz != ld:
        _bad("qx and qz must have the same shape and layout")
    found = torch.empty((max(n, 1),), dtype=torch.int8, device="cuda")
    val = torch.empty((max(n, 1),), dtype=torch.float64, device="cuda")
    _check(lib().iqcc_store_lookup(ctx, store, px, pz, n, ld, _ptr(found), _ptr(val),
                                   _stream(stream)), ctx)
    return found[:n].bool(), val[:n]


def iqcc_store_export(ctx, store, stream=None):
    """Returns (x, z, c) device tensors with the live terms (grouped by bucket)."""
    import torch
    n = iqcc_store_count(ctx, store, stream)
    _, W = iqcc_store_shape(store)
    cap = max(n, 1)
    x = torch.empty((W, cap), dtype=torch.int64, device="cuda")
    z = torch.empty((W, cap), dtype=torch.int64, device="cuda")
    c = torch.empty((cap,), dtype=torch.float64, device="cuda")
    got = ct.c_int64()
    _check(lib().iqcc_store_export(ctx, store, _ptr(x), _ptr(z), _ptr(c), cap, cap, ct.byref(got),
                                   _stream(stream)), ctx)
    return x[:, :got.value], z[:, :got.value], c[:got.value]


def iqcc_dress(ctx, store_in, px, pz, tau: float, eps: float, store_out, theta=None, phi=None,
               energy=None, stream=None):
    """One fused dressing step (store_in -> store_out); px, pz host uint64 words."""
    _, W = _nq(store_in)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    opt = theta is None and phi is None and energy is None
    th, ph = _angles(store_in, theta, phi, optional=opt)
    pe = _f64(energy, "energy", 1, optional=opt)
    _check(lib().iqcc_dress(ctx, store_in, pxp, pzp, float(tau), float(eps), th, ph, pe, store_out,
                            _stream(stream)), ctx)


def iqcc_dress_energy_update(ctx, store_in, px, pz, tau: float, eps: float, store_out, theta, phi,
                             energy_in, energy_out, stream=None):
    """Dressing step with the energy carried forward: energy_out = <out> given energy_in = <in>."""
    _, W = _nq(store_in)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    th, ph = _angles(store_in, theta, phi)
    _check(lib().iqcc_dress_energy_update(ctx, store_in, pxp, pzp, float(tau), float(eps), th, ph,
                                          _f64(energy_in, "energy_in"),
                                          _f64(energy_out, "energy_out"), store_out,
                                          _stream(stream)), ctx)


def iqcc_dress_inplace(ctx, store, px, pz, tau: float, eps: float, theta=None, phi=None,
                       energy_in=None, energy_out=None, stream=None):
    """In-place dressing step of an IQCC_STORE_INPLACE store; px, pz host uint64
    words.  energy_out (with theta, phi) receives the energy after the step;
    energy_in, if given, is the energy before it (only the change is evaluated)."""
    _, W = _nq(store)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    opt = theta is None and phi is None and energy_out is None
    if opt and energy_in is not None:
        _bad("energy_in needs theta, phi and energy_out")
    th, ph = _angles(store, theta, phi, optional=opt)
    _check(lib().iqcc_dress_inplace(ctx, store, pxp, pzp, float(tau), float(eps), th, ph,
                                    _f64(energy_in, "energy_in", 1, optional=True),
                                    _f64(energy_out, "energy_out", 1, optional=opt),
                                    _stream(stream)), ctx)


def iqcc_store_copy(ctx, src, dst, stream=None):
    """Copy the terms of src into the IQCC_STORE_INPLACE store dst (bucket regions)."""
    _check(lib().iqcc_store_copy(ctx, src, dst, _stream(stream)), ctx)


def iqcc_store_inplace_stats(ctx, store, stream=None):
    """Synchronising: {relocated, freed, region_rows, pool_used} of the last in-place step."""
    v = [ct.c_int64() for _ in range(4)]
    _check(lib().iqcc_store_inplace_stats(ctx, store, *[ct.byref(a) for a in v], _stream(stream)), ctx)
    return dict(zip(("relocated", "freed", "region_rows", "pool_used"), (a.value for a in v)))


def iqcc_dress_count(ctx, store_in, px, pz, stream=None) -> int:
    """Synchronising: number of terms of store_in that anticommute with P."""
    _, W = _nq(store_in)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    n = ct.c_int64()
    _check(lib().iqcc_dress_count(ctx, store_in, pxp, pzp, ct.byref(n), _stream(stream)), ctx)
    return n.value


def iqcc_pauli_products(ctx, n_qubits, x1, z1, x2, z2, stream=None):
    """(x3, z3, e) device tensors with P1 P2 = i^e P3 row by row."""
    import torch
    W = (int(n_qubits) + 63) // 64
    a, n, ld = _planes(x1, "x1", W)
    args = [a]
    for t, nm in ((z1, "z1"), (x2, "x2"), (z2, "z2")):
        p_, n_, ld_ = _planes(t, nm, W)
        if n_ != n or ld_ != ld:
            _bad("all operand planes must have the same shape and layout")
        args.append(p_)
    x3 = torch.empty((W, max(ld, 1)), dtype=torch.int64, device="cuda")
    z3 = torch.empty_like(x3)
    e = torch.empty((max(n, 1),), dtype=torch.int8, device="cuda")
    _check(lib().iqcc_pauli_products(ctx, int(n_qubits), *args, n, ld, _ptr(x3), _ptr(z3), _ptr(e),
                                     _stream(stream)), ctx)
    return x3[:, :n], z3[:, :n], e[:n]


def iqcc_dress_raw(ctx, n_qubits, x, z, c, px, pz, tau, stream=None):
    """Raw dressing of flat rows; returns (ox, oz, oc, flag) device tensors."""
    import torch
    W = (int(n_qubits) + 63) // 64
    _, n, ld = _planes(x, "x", W)
    _, nz, ldz = _planes(z, "z", W)
    if nz != n or ldz != ld or ld != max(n, 1) or c.numel() != n:
        _bad("x, z must be (W, n) contiguous planes and c (n,)")
    _f64(c, "c", n, optional=(n == 0))
    px, _ = _words(px, W)
    pz, _ = _words(pz, W)
    ox = torch.empty((W, max(2 * n, 1)), dtype=torch.int64, device="cuda")
    oz = torch.empty_like(ox)
    oc = torch.empty((max(2 * n, 1),), dtype=torch.float64, device="cuda")
    flag = torch.empty((max(n, 1),), dtype=torch.int8, device="cuda")
    ax, pxp = _words(px)
    az, pzp = _words(pz)
    _check(lib().iqcc_dress_raw(ctx, int(n_qubits), _ptr(x), _ptr(z), _ptr(c), n, max(n, 1), pxp, pzp,
                                float(tau), _ptr(ox), _ptr(oz), _ptr(oc), _ptr(flag), max(2 * n, 1),
                                _stream(stream)), ctx)
    return ox[:, :2 * n], oz[:, :2 * n], oc[:2 * n], flag[:n]


def iqcc_merge_truncate(ctx, x, z, c, eps, store_out, stream=None):
    _, W = _nq(store_out)
    px, n, ld = _planes(x, "x", W)
    pz, nz, ldz = _planes(z, "z", W)
    if nz != n or ldz != ld or c.numel() != n:
        _bad("x, z must be (W, n) planes with one coefficient per row")
    _check(lib().iqcc_merge_truncate(ctx, px, pz, _f64(c, "c", n, optional=(n == 0)), n, ld,
                                     float(eps), store_out, _stream(stream)), ctx)


def iqcc_qmf_energy_noalloc(ctx, store, theta, phi, energy=None, stream=None):
    """iqcc_qmf_energy without any device allocation by the library (its scratch
    is a fixed device array); `energy` must be given when the caller cannot
    allocate either."""
    import torch
    if energy is None:
        energy = torch.empty((), dtype=torch.float64, device="cuda")
    th, ph = _angles(store, theta, phi)
    _check(lib().iqcc_qmf_energy_noalloc(ctx, store, th, ph, _f64(energy, "energy"), _stream(stream)), ctx)
    return energy


def iqcc_qmf_energy(ctx, store, theta, phi, energy=None, stream=None):
    import torch
    if energy is None:
        energy = torch.empty((), dtype=torch.float64, device="cuda")
    th, ph = _angles(store, theta, phi)
    _check(lib().iqcc_qmf_energy(ctx, store, th, ph, _f64(energy, "energy"), _stream(stream)), ctx)
    return energy


def iqcc_qmf_energy_backward(ctx, store, theta, phi, dE=None, lam=None, stream=None):
    """dE/dtheta, dE/dphi (scaled by dE); `lam`, if given, receives dE * <P_r> per row."""
    import torch
    th, ph = _angles(store, theta, phi)
    pdE = _f64(dE, "dE", 1, optional=True)
    plam = _f64(lam, "lambda", iqcc_store_rows(store), optional=True)
    dtheta = torch.empty_like(theta)
    dphi = torch.empty_like(phi)
    _check(lib().iqcc_qmf_energy_backward(ctx, store, th, ph, pdE, _ptr(dtheta), _ptr(dphi), plam,
                                          _stream(stream)), ctx)
    return dtheta, dphi


def iqcc_dis_gradients(ctx, store, theta, phi, cx, cz, mode=IQCC_DIS_BATCHED, stream=None):
    """cx, cz: int64 (W, n_cand) device tensors; returns g (n_cand,) float64."""
    import torch
    _, W = _nq(store)
    pcx, n_cand, ld = _planes(cx, "cx", W)
    pcz, nz, ldz = _planes(cz, "cz", W)
    if nz != n_cand or ldz != ld:
        _bad("cx and cz must have the same shape and layout")
    th, ph = _angles(store, theta, phi)
    g = torch.empty((max(n_cand, 1),), dtype=torch.float64, device="cuda")
    _check(lib().iqcc_dis_gradients(ctx, store, th, ph, pcx, pcz, n_cand, ld, int(mode), _ptr(g),
                                    _stream(stream)), ctx)
    return g[:n_cand]


def iqcc_store_rows(store) -> int:
    r = ct.c_int64()
    _check(lib().iqcc_store_rows(store, ct.byref(r)), None)
    return r.value


def _check_tape(store_in, *tapes):
    """Tapes are int32 device arrays with one entry per arena row of the input."""
    import torch
    rows = iqcc_store_rows(store_in)
    for t in tapes:
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous() or t.numel() < rows:
            raise IqccError(IQCC_ERR_INVALID_ARG,
                            f"tape must be a contiguous int32 device array of >= {rows} entries")


def iqcc_dress_taped(ctx, store_in, px, pz, tau, eps, store_out, tape_self, tape_partner,
                     stream=None):
    _check_tape(store_in, tape_self, tape_partner)
    _, W = _nq(store_in)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    _check(lib().iqcc_dress_taped(ctx, store_in, pxp, pzp, float(tau), float(eps), store_out,
                                  _ptr(tape_self), _ptr(tape_partner), _stream(stream)), ctx)


def iqcc_dress_backward(ctx, store_in, px, pz, tau, tape_self, tape_partner, lambda_out,
                        lambda_in, dtau, stream=None, store_out=None):
    """One reverse step; lambda_out has one entry per arena row of the step's
    output store (checked when store_out is given), lambda_in one per row of
    store_in."""
    _check_tape(store_in, tape_self, tape_partner)
    _, W = _nq(store_in)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    rows_out = iqcc_store_rows(store_out) if store_out is not None else 1
    _check(lib().iqcc_dress_backward(ctx, store_in, pxp, pzp, float(tau), _ptr(tape_self),
                                     _ptr(tape_partner), _f64(lambda_out, "lambda_out", rows_out),
                                     _f64(lambda_in, "lambda_in", iqcc_store_rows(store_in)),
                                     _f64(dtau, "dtau"), _stream(stream)), ctx)


def iqcc_chain_forward(ctx, h0, pxs, pzs, taus, eps, outs, tapes_self, tapes_partner, stream=None):
    """Taped chain in one call: outs[j] (store handles) = step j; tapes per step."""
    n = len(outs)
    _, W = _nq(h0)
    px = np.ascontiguousarray(np.asarray(pxs, np.uint64).reshape(n, -1))
    pz = np.ascontiguousarray(np.asarray(pzs, np.uint64).reshape(n, -1))
    if n and (px.shape[1] != W or pz.shape[1] != W):
        _bad(f"entanglers must have {W} words")
    tt = np.ascontiguousarray(np.asarray(taus, np.float64).reshape(-1))
    if tt.size != n or len(tapes_self) != n or len(tapes_partner) != n:
        _bad("one tau and one pair of tapes per step")
    src = h0
    for j in range(n):
        _check_tape(src, tapes_self[j], tapes_partner[j])
        src = outs[j]
    a_out = (ct.c_void_p * max(n, 1))(*[o.value if hasattr(o, "value") else o for o in outs])
    a_ts = (ct.c_void_p * max(n, 1))(*[t.data_ptr() for t in tapes_self])
    a_tp = (ct.c_void_p * max(n, 1))(*[t.data_ptr() for t in tapes_partner])
    _check(lib().iqcc_chain_forward(ctx, h0, n, px.ctypes.data_as(ct.c_void_p),
                                    pz.ctypes.data_as(ct.c_void_p), tt.ctypes.data_as(ct.c_void_p),
                                    float(eps), a_out, a_ts, a_tp, _stream(stream)), ctx)


def iqcc_chain_backward(ctx, h0, pxs, pzs, taus, outs, tapes_self, tapes_partner, lambda_final,
                        lambda_h0=None, stream=None):
    """Reverse sweep of iqcc_chain_forward; returns dE/dtau (device, n_steps)."""
    import torch
    n = len(outs)
    _, W = _nq(h0)
    px = np.ascontiguousarray(np.asarray(pxs, np.uint64).reshape(n, -1))
    pz = np.ascontiguousarray(np.asarray(pzs, np.uint64).reshape(n, -1))
    tt = np.ascontiguousarray(np.asarray(taus, np.float64).reshape(-1))
    if tt.size != n or len(tapes_self) != n or len(tapes_partner) != n:
        _bad("one tau and one pair of tapes per step")
    rows = max([iqcc_store_rows(h0)] + [iqcc_store_rows(o) for o in outs])
    src = h0
    for j in range(n):
        _check_tape(src, tapes_self[j], tapes_partner[j])
        src = outs[j]
    plf = _f64(lambda_final, "lambda_final", iqcc_store_rows(outs[-1]) if n else 1)
    ph0 = _f64(lambda_h0, "lambda_h0", iqcc_store_rows(h0), optional=True)
    w0 = torch.empty(rows, dtype=torch.float64, device="cuda")
    w1 = torch.empty(rows, dtype=torch.float64, device="cuda")
    dtau = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
    a_out = (ct.c_void_p * max(n, 1))(*[o.value if hasattr(o, "value") else o for o in outs])
    a_ts = (ct.c_void_p * max(n, 1))(*[t.data_ptr() for t in tapes_self])
    a_tp = (ct.c_void_p * max(n, 1))(*[t.data_ptr() for t in tapes_partner])
    _check(lib().iqcc_chain_backward(ctx, h0, n, px.ctypes.data_as(ct.c_void_p),
                                     pz.ctypes.data_as(ct.c_void_p), tt.ctypes.data_as(ct.c_void_p),
                                     a_out, a_ts, a_tp, plf, _ptr(w0), _ptr(w1), ph0, _ptr(dtau),
                                     _stream(stream)), ctx)
    return dtau[:n]


def iqcc_expectations(ctx, store, theta, phi, out, scale=None, stream=None):
    th, ph = _angles(store, theta, phi)
    _check(lib().iqcc_expectations(ctx, store, th, ph, _f64(scale, "scale", 1, optional=True),
                                   _f64(out, "out", iqcc_store_rows(store)), _stream(stream)), ctx)
    return out


def _batch_args(ins, outs, pxs, pzs, taus):
    n = len(ins)
    if n < 1 or len(outs) != n:
        _bad("a batch needs one output store per input store")
    W = _nq(ins[0])[1]
    a_in = (ct.c_void_p * n)(*[s.value if hasattr(s, "value") else s for s in ins])
    a_out = (ct.c_void_p * n)(*[s.value if hasattr(s, "value") else s for s in outs])
    px = np.ascontiguousarray(np.asarray(pxs, dtype=np.uint64).reshape(n, -1))
    pz = np.ascontiguousarray(np.asarray(pzs, dtype=np.uint64).reshape(n, -1))
    if px.shape[1] != W or pz.shape[1] != W:
        _bad(f"batch entanglers must have {W} words each")
    tt = np.ascontiguousarray(np.asarray(taus, dtype=np.float64).reshape(-1))
    if tt.size != n:
        _bad("one tau per Hamiltonian")
    return n, a_in, a_out, px, pz, tt


def iqcc_dress_batched(ctx, ins, outs, pxs, pzs, taus, eps, stream=None):
    """ins/outs: lists of store handles; pxs, pzs: (n, W) uint64; taus: (n,)."""
    n, a_in, a_out, px, pz, tt = _batch_args(ins, outs, pxs, pzs, taus)
    _check(lib().iqcc_dress_batched(ctx, n, a_in, a_out, px.ctypes.data_as(ct.c_void_p),
                                    pz.ctypes.data_as(ct.c_void_p), tt.ctypes.data_as(ct.c_void_p),
                                    float(eps), _stream(stream)), ctx)


def iqcc_batch_create(ctx, ins, outs, pxs, pzs, taus, eps):
    n, a_in, a_out, px, pz, tt = _batch_args(ins, outs, pxs, pzs, taus)
    h = ct.c_void_p()
    _check(lib().iqcc_batch_create(ctx, n, a_in, a_out, px.ctypes.data_as(ct.c_void_p),
                                   pz.ctypes.data_as(ct.c_void_p), tt.ctypes.data_as(ct.c_void_p),
                                   float(eps), ct.byref(h)), ctx)
    return h


def iqcc_batch_launch(ctx, batch, stream=None):
    _check(lib().iqcc_batch_launch(ctx, batch, _stream(stream)), ctx)


def iqcc_batch_destroy(ctx, batch):
    _check(lib().iqcc_batch_destroy(ctx, batch), ctx)


# ---------------------------------------------------------------------------
# conversions between row-major numpy keys (N, W) and device word planes
# ---------------------------------------------------------------------------

def to_device_words(a: np.ndarray):
    """(N, W) uint64 numpy -> (W, N) int64 cuda tensor."""
    import torch
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint64).T).view(np.int64)
    return torch.from_numpy(a.copy()).cuda()


def from_device_words(t) -> np.ndarray:
    """(W, N) int64 cuda tensor -> (N, W) uint64 numpy."""
    a = t.detach().cpu().numpy().view(np.uint64)
    return np.ascontiguousarray(a.T)


class Context:
    """Owning wrapper of an iqcc context."""

    def __init__(self, device: int = 0):
        self.handle = iqcc_ctx_create(device)

    def close(self):
        if self.handle is not None:
            iqcc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def iqcc_qmf_energy_anti(ctx, store, px, pz, theta, phi, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty((), dtype=torch.float64, device="cuda")
    _, W = _nq(store)
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    th, ph = _angles(store, theta, phi)
    _check(lib().iqcc_qmf_energy_anti(ctx, store, pxp, pzp, th, ph, _f64(out, "out"),
                                      _stream(stream)), ctx)
    return out


def iqcc_sortless_dress(ctx, n_qubits, x, z, c, px, pz, tau, eps, cap=None, stream=None):
    """Sortless dressing of a canonically sorted flat Hamiltonian (device planes
    x, z of shape (W, n) int64, c (n,) float64); returns (ox, oz, oc) trimmed."""
    import torch
    W = (int(n_qubits) + 63) // 64
    _, n, ld = _planes(x, "x", W)
    _, nz, ldz = _planes(z, "z", W)
    if nz != n or ldz != ld or c.numel() != n:
        _bad("x, z must be (W, n) planes with one coefficient per row")
    _f64(c, "c", n, optional=(n == 0))
    cap = int(cap if cap is not None else max(2 * n, 1))
    ox = torch.empty((W, cap), dtype=torch.int64, device="cuda")
    oz = torch.empty((W, cap), dtype=torch.int64, device="cuda")
    oc = torch.empty((cap,), dtype=torch.float64, device="cuda")
    ax, pxp = _words(px, W)
    az, pzp = _words(pz, W)
    nout = ct.c_int64()
    _check(lib().iqcc_sortless_dress(ctx, int(n_qubits), _ptr(x), _ptr(z), _ptr(c), n, ld if n else 0,
                                     pxp, pzp, float(tau), float(eps), _ptr(ox), _ptr(oz), _ptr(oc), cap, cap,
                                     ct.byref(nout), _stream(stream)), ctx)
    k = nout.value
    return ox[:, :k], oz[:, :k], oc[:k]


def iqcc_energy_trig_poly(ctx, store, pxs, pzs, theta, phi, work):
    """3^n coefficients of E(tau_1..tau_n); pxs, pzs (n, W) host words, work: n Stores."""
    _, W = _nq(store)
    pxs = np.ascontiguousarray(np.asarray(pxs, np.uint64).reshape(len(work), -1))
    pzs = np.ascontiguousarray(np.asarray(pzs, np.uint64).reshape(len(work), -1))
    if pxs.shape[1] != W or pzs.shape[1] != W:
        _bad(f"generators must have {W} words")
    _angles(store, theta, phi)
    n = pxs.shape[0]
    coef = np.zeros(3 ** n)
    arr = (ct.c_void_p * n)(*[w.handle for w in work])
    _check(lib().iqcc_energy_trig_poly(ctx, store, n, pxs.ctypes.data_as(ct.c_void_p),
                                       pzs.ctypes.data_as(ct.c_void_p), _ptr(theta), _ptr(phi), arr,
                                       coef.ctypes.data_as(ct.c_void_p)), ctx)
    return coef


def iqcc_trig_poly_eval(coef, tau):
    coef = np.ascontiguousarray(coef, np.float64); tau = np.ascontiguousarray(tau, np.float64)
    return lib().iqcc_trig_poly_eval(len(tau), coef.ctypes.data_as(ct.c_void_p), tau.ctypes.data_as(ct.c_void_p))


def iqcc_trig_poly_minimize(coef, tau0, sweeps=100):
    coef = np.ascontiguousarray(coef, np.float64)
    tau = np.array(tau0, dtype=np.float64)
    e = ct.c_double()
    rc = lib().iqcc_trig_poly_minimize(len(tau), coef.ctypes.data_as(ct.c_void_p),
                                       tau.ctypes.data_as(ct.c_void_p), int(sweeps), ct.byref(e))
    if rc:
        raise IqccError(rc, "invalid polynomial arguments")
    return tau, e.value


def iqcc_truncate_top(ctx, store_in, max_terms: int, store_out, stream=None):
    """Keep the max_terms terms of largest |c| (ties: smaller canonical key)."""
    _check(lib().iqcc_truncate_top(ctx, store_in, int(max_terms), store_out, _stream(stream)), ctx)


def iqcc_flip_sets(ctx, store, w_max: int):
    """Distinct flip sets (1 <= |F| <= w_max) as a (n, W) uint64 host array."""
    nq, W = iqcc_store_shape(store)
    n = ct.c_int64()
    rc = lib().iqcc_flip_sets(ctx, store, int(w_max), None, 0, ct.byref(n))
    if rc not in (IQCC_OK, IQCC_ERR_CAPACITY):
        _check(rc, ctx)
    out = np.zeros((max(n.value, 1), W), dtype=np.uint64)
    _check(lib().iqcc_flip_sets(ctx, store, int(w_max), out.ctypes.data_as(ct.c_void_p), n.value,
                                ct.byref(n)), ctx)
    return out[:n.value]


def iqcc_qcc_iteration(ctx, h: "Store", spare: "Store", theta, phi, w_max: int, n_select: int,
                       eps: float):
    """One iQCC iteration; swaps the handles of h and spare as the steps ping-pong.

    Returns dict(sel_x, sel_z (n_applied, W), sel_g, sel_tau, energy (n_applied + 1),
    n_candidates)."""
    W = iqcc_store_shape(h.handle)[1]
    _angles(h.handle, theta, phi)
    k = max(int(n_select), 1)
    sx = np.zeros((k, W), np.uint64); sz = np.zeros((k, W), np.uint64)
    sg = np.zeros(k); st = np.zeros(k); en = np.zeros(k + 1)
    nc = ct.c_int64(); na = ct.c_int32()
    hh, hs = h.handle, spare.handle          # c_void_p handles, swapped in place by the call
    rc = lib().iqcc_qcc_iteration(ctx, ct.byref(hh), ct.byref(hs), _ptr(theta), _ptr(phi), int(w_max),
                                  int(n_select), float(eps), sx.ctypes.data_as(ct.c_void_p),
                                  sz.ctypes.data_as(ct.c_void_p), sg.ctypes.data_as(ct.c_void_p),
                                  st.ctypes.data_as(ct.c_void_p), en.ctypes.data_as(ct.c_void_p),
                                  ct.byref(nc), ct.byref(na))
    h.handle, spare.handle = hh, hs
    _check(rc, ctx)
    a = na.value
    return {"sel_x": sx[:a], "sel_z": sz[:a], "sel_g": sg[:a], "sel_tau": st[:a],
            "energy": en[:a + 1], "n_candidates": nc.value}


class Store:
    """A device term store whose memory is a torch tensor (iqcc_store_wrap)."""

    def __init__(self, ctx: Context, n_qubits: int, max_terms: int, flags: int = 0):
        import torch
        self.ctx = ctx
        self.n_qubits = n_qubits
        self.handle = None
        nbytes = iqcc_store_bytes(n_qubits, max_terms, flags)
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.handle = iqcc_store_wrap(ctx.handle, n_qubits, max_terms, flags, self.mem)

    def load_numpy(self, x, z, c):
        import torch
        self._keep = (to_device_words(x), to_device_words(z),
                      torch.from_numpy(np.ascontiguousarray(c, dtype=np.float64)).cuda())
        iqcc_store_load(self.ctx.handle, self.handle, *self._keep)
        return self

    def count(self):
        return iqcc_store_count(self.ctx.handle, self.handle)

    def to_numpy(self):
        x, z, c = iqcc_store_export(self.ctx.handle, self.handle)
        return from_device_words(x), from_device_words(z), c.cpu().numpy()

    def close(self):
        if self.handle is not None and self.ctx.handle is not None:
            iqcc_store_destroy(self.ctx.handle, self.handle)
        self.handle = None
        self.mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
