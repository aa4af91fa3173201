"""Plain CPU reference of one iQCC iteration (test infrastructure only).

Only the test-suite and the CPU-baseline leg of the benchmark use this module.
It follows the iterative procedure of Sec. II step by step, on the FP64 oracle
of ``iqcc_oracle.cpp`` (through ``oracle.py``) and plain numpy / Python:

1. DIS candidates (App. A): every distinct flip set F (the x part of a term,
   the qubits carrying X or Y) with 1 <= |F| <= w_max, and for each qubit q of
   F the generator with Y on q and X on the rest of F.  One Y gives odd Y
   parity; the flip set is that of a term of H.  These are the two DIS
   conditions.
2. Their energy gradients at tau = 0 (Eq. 7), by the oracle.
3. The n_select largest |g|; ties go to the smaller canonical key (x words,
   then z words, most significant word first).
4. For each selected P in that order, on the current Hamiltonian: Eq. 5 leaves
   the terms that commute with P unchanged and turns an anticommuting term A
   into cos(tau) A + (sin tau) (new term), so the QMF energy of the dressed
   Hamiltonian is E(tau) = a + b cos(tau) + c sin(tau) with
   b = sum over anticommuting terms of c_k <P_k>, a = E - b, and c = dE/dtau at
   0, the DIS gradient of P.  The minimum is at (cos tau, sin tau) = -(b, c) /
   |(b, c)|, i.e. tau = atan2(-c, -b).  Dress with that tau and compress.

Several generators at once (Eqs. 5 and 6): without compression, dressing with
P_1..P_n splits every term into branches that carry 1, cos(tau_k) or
sin(tau_k) per generator, so E(tau_1..tau_n) is a trigonometric polynomial with
3^n coefficients; they follow from the energies on the grid {0, pi/2, pi}^n by
inverting the 3x3 basis matrix along every axis.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O


def _popcount(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a.ravel()], dtype=np.int64).reshape(a.shape)


def canonical_key(x, z):
    """Sort key: x words, then z words, most significant word first."""
    W = len(x)
    return tuple(int(x[w]) for w in range(W - 1, -1, -1)) + tuple(int(z[w]) for w in range(W - 1, -1, -1))


def flip_sets(x, w_max):
    """Distinct x parts with 1 <= |F| <= w_max, ascending (most significant word first)."""
    x = np.ascontiguousarray(x, np.uint64)
    if x.ndim == 1:
        x = x[:, None]
    W = x.shape[1]
    wt = _popcount(x).sum(axis=1)
    rows = {tuple(int(v) for v in r) for r, k in zip(x, wt) if 1 <= k <= w_max}
    out = sorted(rows, key=lambda r: tuple(r[w] for w in range(W - 1, -1, -1)))
    return np.array(out, dtype=np.uint64).reshape(len(out), W)


def dis_generators(F):
    """For each flip set (in order) and each of its qubits (ascending): Y there, X elsewhere."""
    F = np.ascontiguousarray(F, np.uint64)
    W = F.shape[1] if F.ndim == 2 else 1
    cx, cz = [], []
    for row in F.reshape(-1, W):
        for w in range(W):
            v = int(row[w])
            for q in range(64):
                if (v >> q) & 1:
                    cx.append([int(t) for t in row])
                    z = [0] * W
                    z[w] = 1 << q
                    cz.append(z)
    return (np.array(cx, dtype=np.uint64).reshape(-1, W), np.array(cz, dtype=np.uint64).reshape(-1, W))


def anticommuting_mask(x, z, px, pz):
    """Terms K with {K, P} = 0: odd popcount of (x & pz) ^ (z & px) over all words."""
    x = np.ascontiguousarray(x, np.uint64).reshape(len(x), -1)
    z = np.ascontiguousarray(z, np.uint64).reshape(len(z), -1)
    t = (x & np.asarray(pz, np.uint64)) ^ (z & np.asarray(px, np.uint64))
    return (_popcount(t).sum(axis=1) % 2) == 1


def energy_anti(nq, x, z, c, px, pz, theta, phi):
    """sum over anticommuting terms of c_k <P_k> (exactly summed with math.fsum)."""
    if len(c) == 0:
        return 0.0
    ev = O.expectations(nq, x, z, theta, phi)
    m = anticommuting_mask(x, z, px, pz)
    return math.fsum((np.asarray(c)[m] * ev[m]).tolist())


def closed_form_tau(b, c):
    """Minimiser of b cos(tau) + c sin(tau)."""
    if b == 0.0 and c == 0.0:
        return 0.0
    return math.atan2(-c, -b)


def qcc_iteration(nq, x, z, c, theta, phi, w_max, n_select, eps):
    """One iteration; returns a dict like the library's and the dressed (x, z, c)."""
    x = np.ascontiguousarray(x, np.uint64).reshape(len(c), -1)
    z = np.ascontiguousarray(z, np.uint64).reshape(len(c), -1)
    W = x.shape[1]
    e = O.qmf_energy(nq, x, z, c, theta, phi)
    energies = [e]
    F = flip_sets(x, w_max)
    cx, cz = dis_generators(F)
    res = {"n_candidates": len(cx), "sel_x": [], "sel_z": [], "sel_g": [], "sel_tau": []}
    if len(cx) and n_select > 0:
        g = O.dis_gradients(nq, x, z, c, theta, phi, cx, cz)
        order = sorted(range(len(cx)), key=lambda i: (-abs(g[i]), canonical_key(cx[i], cz[i])))
        for k in range(min(n_select, len(cx))):
            i = order[k]
            if not abs(g[i]) > 0.0:
                break
            px, pz = cx[i], cz[i]
            b = energy_anti(nq, x, z, c, px, pz, theta, phi)
            cc = float(O.dis_gradients(nq, x, z, c, theta, phi, px[None, :], pz[None, :])[0])
            tau = closed_form_tau(b, cc)
            x, z, c = O.dress(nq, x, z, c, px, pz, tau, eps)
            energies.append(O.qmf_energy(nq, x, z, c, theta, phi))
            res["sel_x"].append(px)
            res["sel_z"].append(pz)
            res["sel_g"].append(float(g[i]))
            res["sel_tau"].append(tau)
    res["sel_x"] = np.array(res["sel_x"], dtype=np.uint64).reshape(-1, W)
    res["sel_z"] = np.array(res["sel_z"], dtype=np.uint64).reshape(-1, W)
    res["sel_g"] = np.array(res["sel_g"])
    res["sel_tau"] = np.array(res["sel_tau"])
    res["energy"] = np.array(energies)
    return res, (x, z, c)


# --- several generators at once -------------------------------------------

GRID = (0.0, 0.5 * math.pi, math.pi)


def energy_trig_poly(nq, x, z, c, pxs, pzs, theta, phi):
    """3^n coefficients of E(tau_1..tau_n) in the basis (1, cos, sin) per
    generator (index s = s_0 + 3 s_1 + ...), from the oracle energies of the
    dressed chains (no compression) on the grid {0, pi/2, pi}^n."""
    n = len(pxs)
    E = np.zeros([3] * n)
    for t in np.ndindex(*([3] * n)):
        hx, hz, hc = x, z, c
        for k in range(n):
            hx, hz, hc = O.dress(nq, hx, hz, hc, pxs[k], pzs[k], GRID[t[k]], 0.0)
        E[t] = O.qmf_energy(nq, hx, hz, hc, theta, phi)
    M = np.array([[1.0, math.cos(a), math.sin(a)] for a in GRID])
    Mi = np.linalg.inv(M)
    coef = E
    for k in range(n):
        coef = np.moveaxis(np.tensordot(Mi, coef, axes=([1], [k])), 0, k)
    # flatten with axis 0 least significant
    return np.transpose(coef, list(range(n))[::-1]).reshape(-1)


def trig_poly_eval(coef, tau):
    n = len(tau)
    f = [np.array([1.0, math.cos(t), math.sin(t)]) for t in tau]
    total = []
    for s in range(3 ** n):
        p, v = coef[s], s
        for k in range(n):
            p *= f[k][v % 3]
            v //= 3
        total.append(p)
    return math.fsum(total)
