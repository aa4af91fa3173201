"""Pins of the oracle against dense 2^n linear algebra (n <= 8)."""
import numpy as np
import pytest

from oracle import dense as D
from paper_2603_08883_amd import inputs as I


def _c1():
    x, z, c = I.hamiltonian_dense(8, 0)
    px, pz = I.single_qubit_pauli(8, "XXXY")
    return 8, x, z, c, px, pz


def _mat(nq, x, z, c):
    return D.hamiltonian_matrix(nq, x, z, c)


def _random_case(seed, nq, nterms, even_y=False):
    rng = np.random.default_rng(seed)
    x, z, c = D.random_pauli_sum(nq, nterms, rng, even_y=even_y)
    while True:
        px = np.array([rng.integers(1, 1 << nq)], np.uint64)
        pz = np.array([rng.integers(0, 1 << nq)], np.uint64)
        if px[0] or pz[0]:
            break
    return x, z, c, px, pz, rng


def test_c1_generator_size():
    nq, x, z, c, px, pz = _c1()
    assert 250 <= len(c) <= 600
    assert px[0] == 0b1111 and pz[0] == 0b1000       # XXXY, Y on qubit 3


@pytest.mark.parametrize("tau", [0.1, -0.7, 2.0])
def test_dress_c1_against_dense_conjugation(oracle, tau):
    nq, x, z, c, px, pz = _c1()
    H = _mat(nq, x, z, c)
    M = D.dress_matrix(nq, H, px, pz, tau)
    ox, oz, oc = oracle.dress(nq, x, z, c, px, pz, tau, eps=0.0)
    Mo = _mat(nq, ox, oz, oc)
    scale = np.abs(c).sum()
    assert np.abs(Mo - M).max() <= 1e-12 * scale
    # the dressed operator is Hermitian and the coefficients are real
    assert np.allclose(M, M.conj().T, atol=1e-12 * scale)


@pytest.mark.parametrize("seed,nq", [(1, 3), (2, 5), (3, 6)])
def test_dress_random_against_dense_decomposition(oracle, seed, nq):
    x, z, c, px, pz, _ = _random_case(seed, nq, 3 * nq)
    tau = 0.37
    H = _mat(nq, x, z, c)
    dx, dz, dc = D.decompose(nq, D.dress_matrix(nq, H, px, pz, tau), tol=1e-13)
    ox, oz, oc = oracle.dress(nq, x, z, c, px, pz, tau, eps=0.0)
    keep = np.abs(oc) > 1e-13
    got = {(int(a[0]), int(b[0])): v for a, b, v in zip(ox[keep], oz[keep], oc[keep])}
    ref = {(int(a[0]), int(b[0])): v for a, b, v in zip(dx, dz, dc)}
    assert set(got) == set(ref)
    for k in ref:
        assert abs(got[k] - ref[k]) <= 1e-12 * np.abs(c).sum()


def test_dress_key_set_is_s_union_anti_xor_p(oracle):
    nq, x, z, c, px, pz = _c1()
    P = D.pauli_matrix(nq, px, pz)
    anti = []
    for k in range(len(c)):
        K = D.pauli_matrix(nq, x[k], z[k])
        anti.append(np.allclose(P @ K, -(K @ P)))
    anti = np.array(anti)
    expect = {(int(a[0]), int(b[0])) for a, b in zip(x, z)}
    expect |= {(int(a[0] ^ px[0]), int(b[0] ^ pz[0])) for a, b in zip(x[anti], z[anti])}
    ox, oz, oc = oracle.dress(nq, x, z, c, px, pz, 0.1, eps=0.0)
    got = {(int(a[0]), int(b[0])) for a, b in zip(ox, oz)}
    assert got == expect
    assert 0 < anti.sum() < len(c)


def test_energy_against_dense(oracle):
    nq, x, z, c, px, pz = _c1()
    th, ph = I.qmf_angles(nq, I.rng_for(0, I.PURPOSE_ANGLES))
    psi = D.qmf_state(th, ph)
    H = _mat(nq, x, z, c)
    assert abs(oracle.qmf_energy(nq, x, z, c, th, ph) - D.energy(H, psi)) <= 1e-12 * np.abs(c).sum()
    # dressed energy equals <Omega| U^+ H U |Omega>
    ox, oz, oc = oracle.dress(nq, x, z, c, px, pz, 0.1)
    Ed = D.energy(D.dress_matrix(nq, H, px, pz, 0.1), psi)
    assert abs(oracle.qmf_energy(nq, ox, oz, oc, th, ph) - Ed) <= 1e-12 * np.abs(c).sum()


@pytest.mark.parametrize("seed", [11, 12])
def test_dis_gradient_against_dense(oracle, seed):
    nq = 6
    x, z, c, _, _, rng = _random_case(seed, nq, 20)
    th = rng.uniform(0, np.pi, nq); ph = rng.uniform(0, 2 * np.pi, nq)
    psi = D.qmf_state(th, ph)
    H = _mat(nq, x, z, c)
    cx = rng.integers(0, 1 << nq, size=(30, 1)).astype(np.uint64)
    cz = rng.integers(0, 1 << nq, size=(30, 1)).astype(np.uint64)
    g = oracle.dis_gradients(nq, x, z, c, th, ph, cx, cz)
    for a in range(30):
        ref = D.dis_gradient(nq, H, psi, cx[a], cz[a])
        assert abs(g[a] - ref) <= 1e-12 * np.abs(c).sum()


def test_dis_gradient_c1_xxxy(oracle):
    nq, x, z, c, px, pz = _c1()
    th, ph = I.qmf_angles(nq, I.rng_for(0, I.PURPOSE_ANGLES))
    H = _mat(nq, x, z, c)
    ref = D.dis_gradient(nq, H, D.qmf_state(th, ph), px, pz)
    g = oracle.dis_gradients(nq, x, z, c, th, ph, px[None], pz[None])
    assert abs(g[0] - ref) <= 1e-12 * np.abs(c).sum()
    assert abs(ref) > 1e-6


def test_angle_gradients_against_dense(oracle):
    nq, x, z, c, _, _ = _c1()
    th, ph = I.qmf_angles(nq, I.rng_for(0, I.PURPOSE_ANGLES))
    H = _mat(nq, x, z, c)
    dt_ref, dp_ref = D.grad_angles(H, th, ph)
    dt, dp = oracle.qmf_grad_angles(nq, x, z, c, th, ph)
    s = np.abs(c).sum()
    assert np.abs(dt - dt_ref).max() <= 1e-12 * s
    assert np.abs(dp - dp_ref).max() <= 1e-12 * s


def test_chain_tau_gradients_against_dense(oracle):
    nq, x, z, c, _, _ = _c1()
    rng = np.random.default_rng(5)
    ents = []
    for _ in range(3):
        px = np.array([rng.integers(1, 256)], np.uint64)
        pz = np.array([rng.integers(0, 256)], np.uint64)
        ents.append((px, pz))
    taus = [0.11, -0.23, 0.31]
    th, ph = I.qmf_angles(nq, I.rng_for(0, I.PURPOSE_ANGLES))
    H = _mat(nq, x, z, c)
    E_ref, g_ref = D.chain_energy_and_tau_grads(nq, H, ents, taus, D.qmf_state(th, ph))
    ox, oz, oc = oracle.chain(nq, x, z, c, ents, taus, eps=0.0)
    s = np.abs(c).sum()
    assert abs(oracle.qmf_energy(nq, ox, oz, oc, th, ph) - E_ref) <= 1e-12 * s
    for k in range(3):
        gk, _ = oracle.chain_tau_gradient(nq, x, z, c, ents, taus, 0.0, th, ph, k)
        assert abs(gk - g_ref[k]) <= 1e-11 * s, (k, gk, g_ref[k])
