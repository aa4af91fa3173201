"""Dense 2^n-matrix checker (test infrastructure only, n <= 8).

Builds every operator as an explicit complex matrix from Kronecker products of
the 2x2 Pauli matrices, so it pins the symplectic oracle to textbook linear
algebra:
  * dressing (Eq. 5): M = U^dagger H U with U = exp(-i tau P / 2)
    = cos(tau/2) I - i sin(tau/2) P, decomposed back into Pauli coefficients
    c_Q = Re tr(Q M) / 2^n;
  * QMF state (Eq. 3) as an explicit vector, energies <Omega|H|Omega>;
  * DIS gradient (Eq. 7) as Im <Omega|H P|Omega>.
Qubit j is bit j of the basis index (qubit 0 least significant).
"""
from __future__ import annotations

import itertools

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X2 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z2 = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def _bit(words, q):
    return int((int(words[q // 64]) >> (q % 64)) & 1)


def local_ops(nq, x, z):
    ops = []
    for q in range(nq):
        bx, bz = _bit(x, q), _bit(z, q)
        ops.append(Y2 if (bx and bz) else X2 if bx else Z2 if bz else I2)
    return ops


def pauli_matrix(nq, x, z):
    ops = local_ops(nq, x, z)
    M = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(range(nq)):          # qubit nq-1 is the most significant factor
        M = np.kron(M, ops[q])
    return M


def hamiltonian_matrix(nq, x, z, c):
    dim = 1 << nq
    H = np.zeros((dim, dim), dtype=np.complex128)
    for k in range(len(c)):
        H += c[k] * pauli_matrix(nq, x[k], z[k])
    return H


def all_pauli_keys(nq):
    W = max(1, (nq + 63) // 64)
    for xs in range(1 << nq):
        for zs in range(1 << nq):
            x = np.zeros(W, np.uint64); z = np.zeros(W, np.uint64)
            x[0] = np.uint64(xs); z[0] = np.uint64(zs)
            yield x, z


def decompose(nq, M, tol=0.0):
    """Pauli coefficients of a Hermitian matrix: c_Q = Re tr(Q M) / 2^n."""
    dim = 1 << nq
    xs, zs, cs = [], [], []
    for x, z in all_pauli_keys(nq):
        Q = pauli_matrix(nq, x, z)
        v = np.trace(Q @ M) / dim
        if abs(v) > tol:
            xs.append(x); zs.append(z); cs.append(v.real)
    W = max(1, (nq + 63) // 64)
    return (np.array(xs, np.uint64).reshape(-1, W), np.array(zs, np.uint64).reshape(-1, W),
            np.array(cs, np.float64))


def dress_matrix(nq, H, px, pz, tau):
    P = pauli_matrix(nq, px, pz)
    U = np.cos(tau / 2) * np.eye(1 << nq) - 1j * np.sin(tau / 2) * P
    return U.conj().T @ H @ U


def qmf_state(theta, phi):
    v = np.ones(1, dtype=np.complex128)
    for q in reversed(range(len(theta))):
        s = np.array([np.cos(theta[q] / 2), np.exp(1j * phi[q]) * np.sin(theta[q] / 2)])
        v = np.kron(v, s)
    return v


def qmf_state_dtheta(theta, phi, j):
    v = np.ones(1, dtype=np.complex128)
    for q in reversed(range(len(theta))):
        if q == j:
            s = np.array([-0.5 * np.sin(theta[q] / 2), 0.5 * np.exp(1j * phi[q]) * np.cos(theta[q] / 2)])
        else:
            s = np.array([np.cos(theta[q] / 2), np.exp(1j * phi[q]) * np.sin(theta[q] / 2)])
        v = np.kron(v, s)
    return v


def qmf_state_dphi(theta, phi, j):
    v = np.ones(1, dtype=np.complex128)
    for q in reversed(range(len(theta))):
        if q == j:
            s = np.array([0.0, 1j * np.exp(1j * phi[q]) * np.sin(theta[q] / 2)])
        else:
            s = np.array([np.cos(theta[q] / 2), np.exp(1j * phi[q]) * np.sin(theta[q] / 2)])
        v = np.kron(v, s)
    return v


def energy(H, psi):
    return float(np.real(np.vdot(psi, H @ psi)))


def grad_angles(H, theta, phi):
    psi = qmf_state(theta, phi)
    n = len(theta)
    dt = np.array([2 * np.real(np.vdot(psi, H @ qmf_state_dtheta(theta, phi, j))) for j in range(n)])
    dp = np.array([2 * np.real(np.vdot(psi, H @ qmf_state_dphi(theta, phi, j))) for j in range(n)])
    return dt, dp


def dis_gradient(nq, H, psi, px, pz):
    P = pauli_matrix(nq, px, pz)
    return float(np.imag(np.vdot(psi, H @ (P @ psi))))


def chain_energy_and_tau_grads(nq, H, ents, taus, psi):
    """E = <psi| U_K^+ ... U_1^+ H U_1 ... U_K |psi> and dE/dtau_k (exact, dense)."""
    dim = 1 << nq
    Us, dUs = [], []
    for (px, pz), t in zip(ents, taus):
        P = pauli_matrix(nq, px, pz)
        U = np.cos(t / 2) * np.eye(dim) - 1j * np.sin(t / 2) * P
        dU = -0.5 * np.sin(t / 2) * np.eye(dim) - 0.5j * np.cos(t / 2) * P
        Us.append(U); dUs.append(dU)

    def total(mats):
        V = np.eye(dim, dtype=np.complex128)
        for M in mats:
            V = V @ M
        return V

    V = total(Us)
    E = float(np.real(np.vdot(psi, V.conj().T @ H @ V @ psi)))
    grads = []
    for k in range(len(Us)):
        mats = list(Us)
        mats[k] = dUs[k]
        dV = total(mats)
        g = 2 * np.real(np.vdot(psi, V.conj().T @ H @ dV @ psi))
        grads.append(float(g))
    return E, np.array(grads)


def random_pauli_sum(nq, n_terms, rng, even_y=False):
    """Random distinct Pauli words with N(0,1) coefficients (W = 1)."""
    keys = set()
    xs, zs = [], []
    while len(xs) < n_terms:
        x = int(rng.integers(0, 1 << nq)); z = int(rng.integers(0, 1 << nq))
        if even_y and bin(x & z).count("1") % 2:
            continue
        if (x, z) in keys:
            continue
        keys.add((x, z))
        xs.append(x); zs.append(z)
    x = np.array(xs, np.uint64).reshape(-1, 1)
    z = np.array(zs, np.uint64).reshape(-1, 1)
    return x, z, rng.normal(size=n_terms)


def pauli_keys_small(nq):
    return list(itertools.product(range(1 << nq), repeat=2))


def pauli_basis(nq):
    """All 4^n Pauli matrices with their keys (x, z) as ints, n <= 5."""
    keys, mats = [], []
    for x, z in all_pauli_keys(nq):
        keys.append((int(x[0]), int(z[0])))
        mats.append(pauli_matrix(nq, x, z))
    return keys, np.array(mats)


def masked_chain_energy(nq, H, ents, taus, eps, psi, masks=None):
    """Energy of the dressing chain in dense arithmetic with compression.

    After each conjugation M <- U^dagger M U the Pauli components
    c_Q = Re tr(Q M) / 2^n with |c_Q| < eps are removed (strict, as the
    compression step of the iterative procedure).  With `masks` given (one
    boolean array over the 4^n basis per step) those kept/removed decisions are
    used instead of being taken from the coefficients, which defines the
    derivative with the compression decisions frozen.  Returns (E, masks,
    kept-key sets per step)."""
    dim = 1 << nq
    keys, B = pauli_basis(nq)
    M = H
    used, kept = [], []
    for j, ((px, pz), t) in enumerate(zip(ents, taus)):
        M = dress_matrix(nq, M, px, pz, t)
        coef = np.real(np.einsum("kab,ba->k", B, M)) / dim
        mask = (np.abs(coef) >= eps) if masks is None else masks[j]
        coef = np.where(mask, coef, 0.0)
        M = np.einsum("k,kab->ab", coef, B)
        used.append(mask)
        kept.append({keys[i] for i in np.flatnonzero(mask & (coef != 0.0))})
    return energy(M, psi), used, kept
