"""Pins of the oracle's iQCC iteration (candidates, closed-form amplitude,
sequential dressing) against dense 2^n algebra and the DIS conditions."""
import math

import numpy as np
import pytest

from oracle import dense as D
from oracle import oracle as O
from oracle import qcc as Q
from paper_2603_08883_amd import inputs as I


@pytest.fixture(scope="module")
def h8():
    x, z, c = I.hamiltonian_dense(8, 0)
    th, ph = I.qmf_angles(8, np.random.default_rng(21))
    return 8, x, z, c, th, ph


def test_generators_satisfy_dis_conditions(oracle):
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    F = Q.flip_sets(x, 6)
    xs = {int(v) for v in x[:, 0]}
    wt = [bin(int(v)).count("1") for v in x[:, 0]]
    expect = sorted({int(v) for v, k in zip(x[:, 0], wt) if 1 <= k <= 6})
    assert [int(v) for v in F[:, 0]] == expect
    cx, cz = Q.dis_generators(F)
    assert len(cx) == sum(bin(int(v)).count("1") for v in F[:, 0])
    for gx, gz in zip(cx[:, 0], cz[:, 0]):
        gx, gz = int(gx), int(gz)
        assert bin(gx & gz).count("1") == 1          # exactly one Y: odd parity
        assert gz & ~gx == 0                         # no Z outside the flip set
        assert gx in xs                              # flip set of a term of H
    assert len({(int(a), int(b)) for a, b in zip(cx[:, 0], cz[:, 0])}) == len(cx)


def test_energy_anti_is_the_cos_coefficient(oracle, h8):
    """b = (E(0) - E(pi)) / 2 from dense conjugation by e^{-i pi P/2}."""
    nq, x, z, c, th, ph = h8
    H = D.hamiltonian_matrix(nq, x, z, c)
    psi = D.qmf_state(th, ph)
    cx, cz = Q.dis_generators(Q.flip_sets(x, 4))
    for k in (0, 3, len(cx) - 1):
        b = Q.energy_anti(nq, x, z, c, cx[k], cz[k], th, ph)
        e0 = D.energy(H, psi)
        epi = D.energy(D.dress_matrix(nq, H, cx[k], cz[k], math.pi), psi)
        assert abs(b - (e0 - epi) / 2) <= 1e-12 * np.abs(c).sum()


def test_closed_form_tau_minimises_dense_energy(oracle, h8):
    nq, x, z, c, th, ph = h8
    H = D.hamiltonian_matrix(nq, x, z, c)
    psi = D.qmf_state(th, ph)
    cx, cz = Q.dis_generators(Q.flip_sets(x, 4))
    g = O.dis_gradients(nq, x, z, c, th, ph, cx, cz)
    k = int(np.argmax(np.abs(g)))
    b = Q.energy_anti(nq, x, z, c, cx[k], cz[k], th, ph)
    tau = Q.closed_form_tau(b, g[k])
    e0 = D.energy(H, psi)
    et = D.energy(D.dress_matrix(nq, H, cx[k], cz[k], tau), psi)
    s = np.abs(c).sum()
    assert abs(et - ((e0 - b) - math.hypot(b, g[k]))) <= 1e-12 * s
    for d in (1e-3, -1e-3, 0.3, -0.3):
        assert et <= D.energy(D.dress_matrix(nq, H, cx[k], cz[k], tau + d), psi) + 1e-13 * s
    assert et < e0 - 1e-6


def test_iteration_matches_dense_sequence(oracle, h8):
    """Selection order = dense |gradient| ranking; energies = dense conjugations."""
    nq, x, z, c, th, ph = h8
    res, (fx, fz, fc) = Q.qcc_iteration(nq, x, z, c, th, ph, w_max=4, n_select=3, eps=0.0)
    assert len(res["sel_tau"]) == 3
    H = D.hamiltonian_matrix(nq, x, z, c)
    psi = D.qmf_state(th, ph)
    cx, cz = Q.dis_generators(Q.flip_sets(x, 4))
    gd = np.array([D.dis_gradient(nq, H, psi, a, b) for a, b in zip(cx, cz)])
    first = max(range(len(cx)), key=lambda i: (abs(gd[i]), [-v for v in Q.canonical_key(cx[i], cz[i])]))
    assert np.array_equal(res["sel_x"][0], cx[first]) and np.array_equal(res["sel_z"][0], cz[first])
    s = np.abs(c).sum()
    assert abs(res["sel_g"][0] - gd[first]) <= 1e-12 * s
    M = H
    assert abs(res["energy"][0] - D.energy(M, psi)) <= 1e-12 * s
    for k in range(3):
        M = D.dress_matrix(nq, M, res["sel_x"][k], res["sel_z"][k], res["sel_tau"][k])
        assert abs(res["energy"][k + 1] - D.energy(M, psi)) <= 1e-12 * s
    assert all(b <= a + 1e-13 * s for a, b in zip(res["energy"], res["energy"][1:]))
    # the returned Hamiltonian is the dressed matrix
    assert np.abs(D.hamiltonian_matrix(nq, fx, fz, fc) - M).max() <= 1e-12 * s
