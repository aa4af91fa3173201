"""Seeded synthetic inputs for the iQCC hot path.

This module only *creates* inputs: one- and two-electron integrals, their
Jordan-Wigner image as a Pauli sum H = sum_k C_k P_k (Eq. 2 of the paper),
QMF Bloch angles (Eq. 3), entangler amplitudes and DIS-admissible candidate
generators (App. A, "Direct Interaction Space").  It holds none of the
arithmetic of the method itself (no dressing, merging, expectation values or
gradients); both the HIP library and the CPU oracle read the arrays it
returns.

Layout of a Pauli sum (shared by every consumer):
  x, z : uint64 arrays of shape (N, W); qubit j is bit (j % 64) of word j // 64
         (W = ceil(n_qubits / 64)); the local operator on qubit j is
         I (x=0,z=0), X (1,0), Z (0,1), Y (1,1) -- Hermitian Y, no stored phase.
  c    : float64 array of shape (N,), real coefficients.

Fermion modes are spin orbitals interleaved as qubit 2i = orbital i alpha,
qubit 2i+1 = orbital i beta.  The electronic Hamiltonian is taken in chemists'
notation, H = sum h_pq a+_p a_q + 1/2 sum (pq|rs) a+_p a+_r a_s a_q with
spin-conserving pairs (p,q) and (r,s); the paper prints two index orders for
the two-electron operator (Eq. 1 versus the appendix restatement) and this
reading is the one used here.

The Jordan-Wigner expansion is done with explicit 2x2 operator products per
qubit (a+ = |1><0|, a = |0><1|, string of Z on lower qubits), followed by a
Pauli decomposition of each local 2x2 matrix; it does not use a symplectic
product formula.

Seeds: numpy PCG64 ``default_rng(260308883 + k)`` with
k = 100 * config_index + purpose (PURPOSE_* below).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 260308883
PURPOSE_INTEGRALS = 1
PURPOSE_ANGLES = 2
PURPOSE_ENTANGLERS = 3
PURPOSE_CANDIDATES = 4
PURPOSE_SUBSET = 5
PURPOSE_TAUS = 6


def rng_for(config: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 100 * config + purpose)


def n_words(n_qubits: int) -> int:
    return max(1, (n_qubits + 63) // 64)


# ----------------------------------------------------------------------------
# integrals
# ----------------------------------------------------------------------------

def _pair_index(p, q):
    hi = np.maximum(p, q)
    lo = np.minimum(p, q)
    return hi * (hi + 1) // 2 + lo


def integrals(n_spatial: int, rng: np.random.Generator, band: int | None = None,
              decay: float | None = None, sigma_h: float = 1.0, sigma_g: float = 0.1):
    """Random real integrals with the 8-fold permutational symmetry.

    h_pq ~ N(0, sigma_h) symmetric; (pq|rs) ~ N(0, sigma_g) drawn once per
    symmetry class and mirrored.  With ``band`` set, two-electron integrals
    survive only for |p-q| <= band and |r-s| <= band and are scaled by
    exp(-(|p-q|+|r-s|)/decay); h is banded and scaled the same way
    (|p-q| <= band, exp(-|p-q|/decay)).
    """
    n = n_spatial
    npair = n * (n + 1) // 2
    hv = rng.normal(0.0, sigma_h, size=npair)
    ncanon = npair * (npair + 1) // 2
    gv = rng.normal(0.0, sigma_g, size=ncanon)
    p, q = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    h = hv[_pair_index(p, q)]
    pq = _pair_index(p, q)                      # (n, n)
    PQ = pq[:, :, None, None]
    RS = pq[None, None, :, :]
    g = gv[_pair_index(PQ, RS)]                 # (n, n, n, n)
    if band is not None:
        d1 = np.abs(p - q)
        hmask = d1 <= band
        h = np.where(hmask, h * np.exp(-d1 / decay), 0.0)
        D1 = d1[:, :, None, None]
        D2 = d1[None, None, :, :]
        gmask = (D1 <= band) & (D2 <= band)
        g = np.where(gmask, g * np.exp(-(D1 + D2) / decay), 0.0)
    return h, g


# ----------------------------------------------------------------------------
# Jordan-Wigner expansion with explicit per-qubit 2x2 algebra
# ----------------------------------------------------------------------------

_ZM = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_CRE = np.array([[0, 0], [1, 0]], dtype=np.complex128)    # a+ = |1><0|
_ANN = np.array([[0, 1], [0, 0]], dtype=np.complex128)    # a  = |0><1|
_ID = np.eye(2, dtype=np.complex128)


def _set_bit(words, q, on):
    """words: (N, W) uint64; set bit q (per row) where on is True."""
    W = words.shape[1]
    for w in range(W):
        sel = on & (q // 64 == w)
        if np.any(sel):
            words[sel, w] |= np.left_shift(np.uint64(1), (q[sel] % 64).astype(np.uint64))


def _toggle_lt(words, m):
    """Toggle bits 0..m-1 of each row (m: (N,) int)."""
    W = words.shape[1]
    for w in range(W):
        lo = w * 64
        k = np.clip(m - lo, 0, 64).astype(np.int64)
        full = k == 64
        mask = np.where(full, np.uint64(0xFFFFFFFFFFFFFFFF),
                        (np.left_shift(np.uint64(1), np.minimum(k, 63).astype(np.uint64)) - np.uint64(1)))
        words[:, w] ^= mask


def _get_bit(words, q):
    N = words.shape[0]
    out = np.zeros(N, dtype=bool)
    W = words.shape[1]
    for w in range(W):
        sel = q // 64 == w
        if np.any(sel):
            out[sel] = ((words[sel, w] >> (q[sel] % 64).astype(np.uint64)) & np.uint64(1)).astype(bool)
    return out


def _right_mul(M, op):
    """M @ op for a stack of 2x2 matrices held as (m00, m01, m10, m11) arrays.

    op is one of "Z" = diag(1, -1), "c" = a+ = |1><0|, "a" = a = |0><1|.
    """
    m00, m01, m10, m11 = M
    if op == "Z":
        return (m00, -m01, m10, -m11)
    if op == "c":            # [[m00,m01],[m10,m11]] @ [[0,0],[1,0]] = [[m01,0],[m11,0]]
        return (m01, np.zeros_like(m01), m11, np.zeros_like(m11))
    # a: [[m00,m01],[m10,m11]] @ [[0,1],[0,0]] = [[0,m00],[0,m10]]
    return (np.zeros_like(m00), m00, np.zeros_like(m10), m10)


def jw_expand(modes: np.ndarray, creates: np.ndarray, coef: np.ndarray, n_qubits: int):
    """Expand products of ladder operators into (unsummed) Pauli strings.

    modes   : (N, k) int   spin-orbital index of each operator, left to right
    creates : (k,) bool    True for a+ at that position
    coef    : (N,) complex
    Returns x, z (M, W) uint64 and complex coefficients (M,).

    Each operator is Z on every lower qubit times a+ or a on its own qubit.  The
    product is kept as a Z mask on the ordinary qubits plus one explicit 2x2
    matrix per distinct mode ("slot"), multiplied left to right.
    """
    N, k = modes.shape
    W = n_words(n_qubits)
    zmask = np.zeros((N, W), dtype=np.uint64)
    slot_q = np.full((N, k), -1, dtype=np.int64)
    one = np.ones(N, dtype=np.complex128)
    zero = np.zeros(N, dtype=np.complex128)
    slots = [[zero, zero, zero, zero] for _ in range(k)]
    for i in range(k):
        m = modes[:, i].astype(np.int64)
        op = "c" if creates[i] else "a"
        merged = np.zeros(N, dtype=bool)
        for j in range(i):
            qj = slot_q[:, j]
            valid = qj >= 0
            lt = valid & (qj < m)
            eq = valid & (qj == m)
            Mz = _right_mul(slots[j], "Z")
            Ms = _right_mul(slots[j], op)
            slots[j] = [np.where(lt, Mz[t], np.where(eq, Ms[t], slots[j][t])) for t in range(4)]
            merged |= eq
        new = ~merged
        zb = _get_bit(zmask, m)
        # initial matrix of a new slot: Z if the mask already holds a Z there, else I
        init = (one, zero, zero, np.where(zb, -one, one))
        Mi = _right_mul(init, op)
        slots[i] = [np.where(new, Mi[t], zero) for t in range(4)]
        slot_q[:, i] = np.where(new, m, -1)
        clr = new & zb
        for w in range(W):
            sel = clr & (m // 64 == w)
            if np.any(sel):
                zmask[sel, w] ^= np.left_shift(np.uint64(1), (m[sel] % 64).astype(np.uint64))
        # Z string on every qubit below m, except qubits that are slots (done above)
        _toggle_lt(zmask, m)
        for j in range(i + 1):
            qj = slot_q[:, j]
            back = (qj >= 0) & (qj < m)
            if np.any(back):
                for w in range(W):
                    sel = back & (qj // 64 == w)
                    if np.any(sel):
                        zmask[sel, w] ^= np.left_shift(np.uint64(1), (qj[sel] % 64).astype(np.uint64))
    # expand each slot into Pauli components (Hermitian basis)
    xs = [np.zeros((N, W), dtype=np.uint64)]
    zs = [zmask.copy()]
    cs = [coef.astype(np.complex128)]
    rows = [np.arange(N)]
    for j in range(k):
        q = slot_q[:, j]
        m00, m01, m10, m11 = slots[j]
        comps = {
            "I": (m00 + m11) / 2,
            "X": (m01 + m10) / 2,
            "Y": 1j * (m01 - m10) / 2,
            "Z": (m00 - m11) / 2,
        }
        nx, nz, nc, nr = [], [], [], []
        for X, Z, C, R in zip(xs, zs, cs, rows):
            qr = q[R]
            valid = qr >= 0
            for lab, (bx, bz) in (("I", (0, 0)), ("X", (1, 0)), ("Y", (1, 1)), ("Z", (0, 1))):
                a = comps[lab][R]
                if lab == "I":
                    a = np.where(valid, a, 1.0)
                else:
                    a = np.where(valid, a, 0.0)
                keep = a != 0
                if not np.any(keep):
                    continue
                X2 = X[keep]
                Z2 = Z[keep]
                qk = qr[keep]
                if bx:
                    _set_bit(X2, qk, np.ones(len(qk), dtype=bool))
                if bz:
                    _set_bit(Z2, qk, np.ones(len(qk), dtype=bool))
                nx.append(X2)
                nz.append(Z2)
                nc.append(C[keep] * a[keep])
                nr.append(R[keep])
        xs, zs, cs, rows = nx, nz, nc, nr
    return np.concatenate(xs), np.concatenate(zs), np.concatenate(cs)


def combine(x: np.ndarray, z: np.ndarray, c: np.ndarray, drop_abs: float = 1e-12):
    """Sum coefficients of equal strings; keep real parts; drop |c| <= drop_abs.

    The imaginary parts of a Hermitian operator's expansion cancel; this is
    asserted.  Output rows are in canonical order (lexicographic on
    x[W-1..0], z[W-1..0] as unsigned words).
    """
    W = x.shape[1]
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)]
    order = np.lexsort(keys)            # last key is primary: x[W-1] ... z[0]
    x = x[order]
    z = z[order]
    c = c[order]
    if len(c) == 0:
        return x, z, c.real.copy()
    diff = np.zeros(len(c), dtype=bool)
    diff[0] = True
    for w in range(W):
        diff[1:] |= x[1:, w] != x[:-1, w]
        diff[1:] |= z[1:, w] != z[:-1, w]
    starts = np.flatnonzero(diff)
    csum = np.add.reduceat(c, starts)
    scale = max(1.0, float(np.max(np.abs(csum)))) if len(csum) else 1.0
    assert np.max(np.abs(csum.imag)) <= 1e-9 * scale, "non-Hermitian expansion"
    cr = csum.real
    keep = np.abs(cr) > drop_abs
    return x[starts][keep], z[starts][keep], np.ascontiguousarray(cr[keep])


def jw_hamiltonian(h: np.ndarray, g: np.ndarray, chunk: int = 400_000):
    """Jordan-Wigner Pauli sum of the electronic Hamiltonian (chemists' notation)."""
    n = h.shape[0]
    nq = 2 * n
    W = n_words(nq)
    parts_x, parts_z, parts_c = [], [], []
    # one-body: h_pq a+_{p s} a_{q s}
    p, q = np.nonzero(h)
    for s in (0, 1):
        modes = np.stack([2 * p + s, 2 * q + s], axis=1)
        X, Z, C = jw_expand(modes, np.array([True, False]), h[p, q].astype(np.complex128), nq)
        parts_x.append(X); parts_z.append(Z); parts_c.append(C)
    # two-body: 1/2 (pq|rs) a+_{p s} a+_{r t} a_{s t} a_{q s}
    P, Q, R, S = np.nonzero(g)
    vals = g[P, Q, R, S]
    for s in (0, 1):
        for t in (0, 1):
            mp = 2 * P + s
            mq = 2 * Q + s
            mr = 2 * R + t
            ms = 2 * S + t
            ok = (mp != mr) & (ms != mq)
            idx = np.flatnonzero(ok)
            for c0 in range(0, len(idx), chunk):
                sl = idx[c0:c0 + chunk]
                modes = np.stack([mp[sl], mr[sl], ms[sl], mq[sl]], axis=1)
                X, Z, C = jw_expand(modes, np.array([True, True, False, False]),
                                    0.5 * vals[sl].astype(np.complex128), nq)
                # partial combine keeps peak memory bounded
                X, Z, Cr = _combine_complex(X, Z, C)
                parts_x.append(X); parts_z.append(Z); parts_c.append(Cr)
    X = np.concatenate(parts_x) if parts_x else np.zeros((0, W), np.uint64)
    Z = np.concatenate(parts_z) if parts_z else np.zeros((0, W), np.uint64)
    C = np.concatenate(parts_c) if parts_c else np.zeros(0, np.complex128)
    return combine(X, Z, C)


def _combine_complex(x, z, c):
    W = x.shape[1]
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)]
    order = np.lexsort(keys)
    x = x[order]; z = z[order]; c = c[order]
    if len(c) == 0:
        return x, z, c
    diff = np.zeros(len(c), dtype=bool)
    diff[0] = True
    for w in range(W):
        diff[1:] |= x[1:, w] != x[:-1, w]
        diff[1:] |= z[1:, w] != z[:-1, w]
    starts = np.flatnonzero(diff)
    return x[starts], z[starts], np.add.reduceat(c, starts)


# ----------------------------------------------------------------------------
# angles, amplitudes, entanglers and DIS candidates
# ----------------------------------------------------------------------------

def qmf_angles(n_qubits: int, rng: np.random.Generator):
    """theta ~ U(0, pi), phi ~ U(0, 2 pi), one pair per qubit."""
    theta = rng.uniform(0.0, np.pi, size=n_qubits)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=n_qubits)
    return theta, phi


def taus(n: int, rng: np.random.Generator, lo: float = -0.2, hi: float = 0.2):
    return rng.uniform(lo, hi, size=n)


def _popcount_rows(words):
    return np.bitwise_count(words).sum(axis=1).astype(np.int64)


def dis_candidates(x: np.ndarray, n_qubits: int, count: int, w_max: int,
                   rng: np.random.Generator, w_min: int = 2, max_tries: int | None = None):
    """Seeded DIS-admissible Pauli generators (App. A conditions).

    Each candidate takes the flip set F of a randomly chosen term of H with
    1 <= |F| <= w_max, puts exactly one Y at a random position of F and X
    elsewhere in F, then adds Z's on random qubits outside F up to a target
    weight w ~ U{max(w_min, |F|) .. w_max}.  Hence every candidate has an odd
    number of Y's and a flip set that matches a term of H.  Duplicates are
    rejected.  Returns cx, cz of shape (count, W).
    """
    W = x.shape[1]
    fw = _popcount_rows(x)
    pool = np.flatnonzero((fw >= 1) & (fw <= w_max))
    if len(pool) == 0:
        raise ValueError("no term of H has a flip set of admissible weight")
    seen = set()
    out_x = np.zeros((count, W), dtype=np.uint64)
    out_z = np.zeros((count, W), dtype=np.uint64)
    got = 0
    tries = 0
    max_tries = max_tries or 100 * count + 1000
    while got < count:
        tries += 1
        if tries > max_tries:
            raise ValueError("could not draw enough distinct candidates")
        k = pool[rng.integers(len(pool))]
        F = []
        for w in range(W):
            v = int(x[k, w])
            while v:
                b = v & -v
                F.append(w * 64 + b.bit_length() - 1)
                v ^= b
        nF = len(F)
        wt = int(rng.integers(max(w_min, nF), w_max + 1)) if max(w_min, nF) <= w_max else nF
        ypos = F[int(rng.integers(nF))]
        cx = [0] * W
        cz = [0] * W
        for q in F:
            cx[q // 64] |= 1 << (q % 64)
        cz[ypos // 64] |= 1 << (ypos % 64)
        outside = np.setdiff1d(np.arange(n_qubits), np.array(F))
        nz_extra = wt - nF
        if nz_extra > 0:
            zq = rng.choice(outside, size=nz_extra, replace=False)
            for q in zq:
                q = int(q)
                cz[q // 64] |= 1 << (q % 64)
        key = tuple(cx) + tuple(cz)
        if key in seen:
            continue
        seen.add(key)
        out_x[got] = np.array(cx, dtype=np.uint64)
        out_z[got] = np.array(cz, dtype=np.uint64)
        got += 1
    return out_x, out_z


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def hamiltonian_dense(n_qubits: int, config: int):
    """Dense random-integral JW Hamiltonian on n_qubits (n_qubits/2 orbitals)."""
    h, g = integrals(n_qubits // 2, rng_for(config, PURPOSE_INTEGRALS))
    return jw_hamiltonian(h, g)


def hamiltonian_banded(n_qubits: int, config: int, band: int = 6, decay: float = 3.0):
    """Banded local-orbital JW Hamiltonian: (pq|rs) only for |p-q|,|r-s| <= band."""
    h, g = integrals(n_qubits // 2, rng_for(config, PURPOSE_INTEGRALS), band=band, decay=decay)
    return jw_hamiltonian(h, g)


def single_qubit_pauli(n_qubits: int, text: str):
    """Key of a Pauli word given as characters, character i acting on qubit i."""
    W = n_words(n_qubits)
    x = np.zeros(W, dtype=np.uint64)
    z = np.zeros(W, dtype=np.uint64)
    for i, ch in enumerate(text):
        b = np.uint64(1) << np.uint64(i % 64)
        if ch in "XY":
            x[i // 64] |= b
        if ch in "ZY":
            z[i // 64] |= b
    return x, z


def unique_rows(x: np.ndarray, z: np.ndarray, c: np.ndarray):
    """Distinct keys, keeping the first occurrence of each (stable)."""
    W = x.shape[1]
    keys = [z[:, w] for w in range(W)] + [x[:, w] for w in range(W)]
    order = np.lexsort(keys)
    xs, zs = x[order], z[order]
    # a row is a duplicate when all of its words equal the previous row's words
    same = np.ones(len(order) - 1, dtype=bool) if len(order) else np.zeros(0, bool)
    for w in range(W):
        same &= (xs[1:, w] == xs[:-1, w]) & (zs[1:, w] == zs[:-1, w])
    keep_sorted = np.ones(len(order), dtype=bool)
    keep_sorted[1:] = ~same
    # among equal keys lexsort is stable, so the kept row is the earliest one
    keep = np.sort(order[keep_sorted])
    return x[keep], z[keep], c[keep]


def expand_to(x, z, c, n_terms, gx, gz, rng):
    """Grow a Pauli sum to >= n_terms distinct words by XOR with generators.

    For a seeded half of the current words K, adds K xor P_j with coefficient
    c_K * u, u ~ U(-0.2, 0.2) (keys only; no phases or rotations), cycling
    through the generators; then keeps a seeded subset of exactly n_terms rows
    (also when the input is already larger).
    """
    j = 0
    while len(c) < n_terms:
        pick = rng.random(len(c)) < 0.5
        nx = x[pick] ^ gx[j % len(gx)]
        nz = z[pick] ^ gz[j % len(gz)]
        nc = c[pick] * rng.uniform(-0.2, 0.2, size=int(pick.sum()))
        x, z, c = unique_rows(np.concatenate([x, nx]), np.concatenate([z, nz]), np.concatenate([c, nc]))
        j += 1
    keep = np.sort(rng.permutation(len(c))[:n_terms])
    return np.ascontiguousarray(x[keep]), np.ascontiguousarray(z[keep]), np.ascontiguousarray(c[keep])


def hamiltonian_expanded(n_qubits: int, config: int, n_terms: int, band: int = 6,
                         w_max: int = 8):
    """A large Pauli sum with the structure of an iterated-dressing Hamiltonian.

    Starts from the banded JW Hamiltonian and repeatedly adds, for a seeded
    half of the current words K, the word K xor P_j of a DIS-form generator P_j
    with coefficient c_K * u, u ~ U(-0.2, 0.2) (keys only; no phases or
    rotations are evaluated).  Stops once at least n_terms distinct words exist
    and keeps a seeded subset of exactly n_terms rows.  Used as the stand-in
    Hamiltonian for batched DIS screening.
    """
    x, z, c = hamiltonian_banded(n_qubits, config, band=band)
    rng = rng_for(config, PURPOSE_SUBSET)
    gx, gz = dis_candidates(x, n_qubits, 64, w_max, rng_for(config, PURPOSE_ENTANGLERS))
    return expand_to(x, z, c, n_terms, gx, gz, rng)


def batch_hamiltonians(config: int, n_ham: int = 64, q_lo: int = 16, q_hi: int = 64,
                       size_lo: float = 1e3, size_hi: float = 1e6, band: int = 2):
    """Many independent Hamiltonians of uneven size for batched dressing.

    n_i ~ U{q_lo, q_lo+2, ..., q_hi} qubits, target sizes s_i log-uniform in
    [size_lo, size_hi]; each starts from the banded JW Hamiltonian on n_i/2
    orbitals (one per distinct n_i) and is grown or subset to exactly s_i
    distinct words by expand_to.  One DIS-form entangler (weight 2-8) and
    tau ~ U(-0.2, 0.2) per Hamiltonian.  Returns a list of dicts.
    """
    rng = rng_for(config, PURPOSE_SUBSET)
    qs = rng.integers(q_lo // 2, q_hi // 2 + 1, size=n_ham) * 2
    sizes = np.exp(rng.uniform(np.log(size_lo), np.log(size_hi), size=n_ham)).astype(np.int64)
    base = {}
    out = []
    for i in range(n_ham):
        nq = int(qs[i])
        if nq not in base:
            bx, bz, bc = hamiltonian_banded(nq, config + nq, band=band)
            gx, gz = dis_candidates(bx, nq, 16, 8, rng_for(config + nq, PURPOSE_ENTANGLERS))
            base[nq] = (bx, bz, bc, gx, gz)
        bx, bz, bc, gx, gz = base[nq]
        x, z, c = expand_to(bx, bz, bc, int(sizes[i]), gx, gz, rng)
        px, pz = dis_candidates(x, nq, 1, 8, rng)
        out.append({"n_qubits": nq, "x": x, "z": z, "c": c, "px": px[0], "pz": pz[0],
                    "tau": float(rng.uniform(-0.2, 0.2))})
    return out
