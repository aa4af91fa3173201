"""Invariant and closed-form pins of the oracle (sizes beyond dense reach)."""
import math

import numpy as np
import pytest

from oracle import dense as D
from paper_2603_08883_amd import inputs as I

ULP = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def h12():
    """12-qubit JW Hamiltonian (6 orbitals) and a DIS entangler."""
    x, z, c = I.hamiltonian_dense(12, 9)
    cx, cz = I.dis_candidates(x, 12, 4, 6, np.random.default_rng(3))
    return 12, x, z, c, cx, cz


def _as_dict(x, z, c):
    return {tuple(a.tolist()) + tuple(b.tolist()): v for a, b, v in zip(x, z, c)}


def test_sum_of_squares_preserved(oracle, h12):
    nq, x, z, c, cx, cz = h12
    for k in range(4):
        ox, oz, oc = oracle.dress(nq, x, z, c, cx[k], cz[k], 0.3 + 0.2 * k, eps=0.0)
        s0 = math.fsum((c * c).tolist()); s1 = math.fsum((oc * oc).tolist())
        assert abs(s1 - s0) <= 16 * ULP * s0
        x, z, c = ox, oz, oc


def test_involution(oracle, h12):
    nq, x, z, c, cx, cz = h12
    ox, oz, oc = oracle.dress(nq, x, z, c, cx[0], cz[0], 0.4)
    bx, bz, bc = oracle.dress(nq, ox, oz, oc, cx[0], cz[0], -0.4)
    keep = np.abs(bc) > 1e-14 * np.abs(c).max()
    got = _as_dict(bx[keep], bz[keep], bc[keep])
    ref = _as_dict(x, z, c)
    assert set(got) == set(ref)
    for k, v in ref.items():
        assert abs(got[k] - v) <= 8 * ULP * np.abs(c).max()


def test_additivity_same_generator(oracle, h12):
    nq, x, z, c, cx, cz = h12
    a = oracle.chain(nq, x, z, c, [(cx[1], cz[1])] * 2, [0.25, 0.5])
    b = oracle.dress(nq, x, z, c, cx[1], cz[1], 0.75)
    da, db = _as_dict(*a), _as_dict(*b)
    scale = np.abs(c).max()
    for k in set(da) | set(db):
        assert abs(da.get(k, 0.0) - db.get(k, 0.0)) <= 16 * ULP * scale


def test_commuting_generators_commute(oracle):
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    p1 = I.single_qubit_pauli(nq, "XYZIIIZZXXII")
    p2 = I.single_qubit_pauli(nq, "IIZXYIIIIIYX")
    _, _, e12 = oracle.pauli_product(nq, p1[0], p1[1], p2[0], p2[1])
    assert e12 % 2 == 0
    a = oracle.chain(nq, x, z, c, [p1, p2], [0.3, -0.45])
    b = oracle.chain(nq, x, z, c, [p2, p1], [-0.45, 0.3])
    da, db = _as_dict(*a), _as_dict(*b)
    scale = np.abs(c).max()
    for k in set(da) | set(db):
        assert abs(da.get(k, 0.0) - db.get(k, 0.0)) <= 16 * ULP * scale


def test_even_y_invariant(oracle, h12):
    nq, x, z, c, cx, cz = h12
    assert np.all(np.bitwise_count(x & z).sum(1) % 2 == 0)       # real JW H
    for k in range(4):
        assert np.bitwise_count(cx[k] & cz[k]).sum() % 2 == 1       # odd-Y generator
        x, z, c = oracle.dress(nq, x, z, c, cx[k], cz[k], 0.2)
        assert np.all(np.bitwise_count(x & z).sum(1) % 2 == 0)


def test_tau_zero(oracle, h12):
    nq, x, z, c, cx, cz = h12
    ox, oz, oc = oracle.dress(nq, x, z, c, cx[0], cz[0], 0.0)
    got = _as_dict(ox, oz, oc)
    ref = _as_dict(x, z, c)
    for k, v in ref.items():
        assert got[k] == v                           # bit-identical values
    for k in set(got) - set(ref):
        assert got[k] == 0.0                         # new keys carry +-0
    assert len(set(got) - set(ref)) > 0


def test_truncation_strict(oracle):
    x = np.array([[1], [2], [3]], np.uint64); z = np.zeros((3, 1), np.uint64)
    c = np.array([1e-8, -0.99e-8, 2.0])
    ox, oz, oc = oracle.merge_truncate(x, z, c, eps=1e-8)
    assert ox[:, 0].tolist() == [1, 3]
    # merging duplicates sums in input order before the cut
    x = np.array([[5], [5], [5], [4]], np.uint64); z = np.zeros((4, 1), np.uint64)
    c = np.array([1.0, 1e-16, -1.0, 3.0])
    ox, oz, oc = oracle.merge_truncate(x, z, c, eps=0.0)
    assert ox[:, 0].tolist() == [4, 5] and oc[1] == (1.0 + 1e-16) - 1.0


def test_energy_special_states(oracle, h12):
    nq, x, z, c, _, _ = h12
    rng = np.random.default_rng(4)
    occ = rng.integers(0, 2, size=nq)
    th = np.where(occ == 1, np.pi, 0.0)
    ph = rng.uniform(0, 2 * np.pi, nq)
    # z-eigenstate: only X-free terms survive, each with sign (-1)^{|z & occ|}
    occ_w = np.uint64(int("".join(str(b) for b in occ[::-1]), 2))
    diag = x[:, 0] == 0
    sign = np.where(np.bitwise_count(z[:, 0] & occ_w) % 2 == 1, -1.0, 1.0)
    ref = math.fsum((c[diag] * sign[diag]).tolist())
    E = oracle.qmf_energy(nq, x, z, c, th, ph)
    # sin(pi) is 1.2e-16 in FP64, so off-diagonal terms leak at that level
    assert abs(E - ref) <= 1e-13 * np.abs(c).sum()
    th2, ph2 = I.qmf_angles(nq, rng)
    assert oracle.qmf_energy(nq, x, z, c, th2, -ph2) == oracle.qmf_energy(nq, x, z, c, th2, ph2)


def test_closed_form_single_entangler(oracle):
    """E(tau) = a + b cos tau + c sin tau with a + b = E(0) and c = g_P (Eq. 7)."""
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, 1, 8, np.random.default_rng(8))
    th, ph = I.qmf_angles(nq, I.rng_for(1, I.PURPOSE_ANGLES))
    E0 = oracle.qmf_energy(nq, x, z, c, th, ph)
    g = oracle.dis_gradients(nq, x, z, c, th, ph, cx, cz)[0]
    taus = [0.5, -1.1, 2.3]
    Es = [oracle.qmf_energy(nq, *oracle.dress(nq, x, z, c, cx[0], cz[0], t), th, ph) for t in taus]
    A = np.array([[1, np.cos(t), np.sin(t)] for t in taus])
    a, b, cc = np.linalg.solve(A, Es)
    s = np.abs(c).sum()
    assert abs((a + b) - E0) <= 1e-11 * s
    assert abs(cc - g) <= 1e-11 * s
    assert abs(g) > 1e-8
    for t in (0.1, -0.2, 1.7, 0.1 + 2 * np.pi):
        Et = oracle.qmf_energy(nq, *oracle.dress(nq, x, z, c, cx[0], cz[0], t), th, ph)
        assert abs(Et - (a + b * np.cos(t) + cc * np.sin(t))) <= 1e-11 * s


def test_dis_gradient_is_derivative_at_zero(oracle):
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    cx, cz = I.dis_candidates(x, nq, 3, 6, np.random.default_rng(12))
    th, ph = I.qmf_angles(nq, np.random.default_rng(13))
    g = oracle.dis_gradients(nq, x, z, c, th, ph, cx, cz)
    h = 1e-4
    for k in range(3):
        Ep = oracle.qmf_energy(nq, *oracle.dress(nq, x, z, c, cx[k], cz[k], h), th, ph)
        Em = oracle.qmf_energy(nq, *oracle.dress(nq, x, z, c, cx[k], cz[k], -h), th, ph)
        fd = (Ep - Em) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k]))


def test_dis_conditions_at_z_eigenstates(oracle):
    """At theta in {0, pi}: a non-vanishing gradient needs odd #Y and a matching flip set."""
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    rng = np.random.default_rng(21)
    th = np.where(rng.integers(0, 2, nq) == 1, np.pi, 0.0)
    ph = rng.uniform(0, 2 * np.pi, nq)
    cx = rng.integers(0, 1 << nq, size=(400, 1)).astype(np.uint64)
    cz = rng.integers(0, 1 << nq, size=(400, 1)).astype(np.uint64)
    dcx, dcz = I.dis_candidates(x, nq, 40, 6, rng)
    cx = np.concatenate([cx, dcx]); cz = np.concatenate([cz, dcz])
    g = oracle.dis_gradients(nq, x, z, c, th, ph, cx, cz)
    flips = set(int(v) for v in x[:, 0])
    nonzero = np.abs(g) > 1e-10
    assert nonzero.sum() >= 3
    for a in np.flatnonzero(nonzero):
        assert bin(int(cx[a, 0] & cz[a, 0])).count("1") % 2 == 1
        assert int(cx[a, 0]) in flips


def test_angle_gradient_fd_and_phi_zero(oracle, h12):
    nq, x, z, c, _, _ = h12
    rng = np.random.default_rng(31)
    th, ph = I.qmf_angles(nq, rng)
    th[2] = 0.0
    dt, dp = oracle.qmf_grad_angles(nq, x, z, c, th, ph)
    assert dp[2] == 0.0
    h = 1e-6
    for j in (0, 5, 11):
        for arr, d in ((th, dt), (ph, dp)):
            a = arr.copy(); a[j] += h
            b = arr.copy(); b[j] -= h
            args_p = (a, ph) if arr is th else (th, a)
            args_m = (b, ph) if arr is th else (th, b)
            fd = (oracle.qmf_energy(nq, x, z, c, *args_p) - oracle.qmf_energy(nq, x, z, c, *args_m)) / (2 * h)
            assert abs(fd - d[j]) <= 1e-6 * max(1.0, abs(d[j]))


def test_tau_gradient_single_entangler_closed_form(oracle):
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    cx, cz = I.dis_candidates(x, nq, 1, 6, np.random.default_rng(41))
    th, ph = I.qmf_angles(nq, np.random.default_rng(42))
    taus = [0.4, -0.9, 1.3]
    Es = [oracle.qmf_energy(nq, *oracle.dress(nq, x, z, c, cx[0], cz[0], t), th, ph) for t in taus]
    A = np.array([[1, np.cos(t), np.sin(t)] for t in taus])
    a, b, cc = np.linalg.solve(A, Es)
    for t in (0.25, -0.6):
        g, _ = oracle.chain_tau_gradient(nq, x, z, c, [(cx[0], cz[0])], [t], 0.0, th, ph, 0)
        assert abs(g - (-b * np.sin(t) + cc * np.cos(t))) <= 1e-11 * np.abs(c).sum()


def test_tau_gradient_last_step_at_zero_is_dis_gradient(oracle):
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    cx, cz = I.dis_candidates(x, nq, 3, 6, np.random.default_rng(51))
    th, ph = I.qmf_angles(nq, np.random.default_rng(52))
    ents = [(cx[k], cz[k]) for k in range(3)]
    taus = [0.3, -0.2, 0.0]
    g, _ = oracle.chain_tau_gradient(nq, x, z, c, ents, taus, 0.0, th, ph, 2)
    hx, hz, hc = oracle.chain(nq, x, z, c, ents[:2], taus[:2])
    gd = oracle.dis_gradients(nq, hx, hz, hc, th, ph, cx[2:3], cz[2:3])[0]
    assert abs(g - gd) <= 1e-12 * np.abs(c).sum()


def test_chain_point_query_matches_full_chain(oracle):
    """The one-key-at-a-time evaluation of the chain reproduces the full chain."""
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, 5, 8, np.random.default_rng(61))
    taus = I.taus(5, np.random.default_rng(62))
    ents = list(zip(cx, cz))
    fx, fz, fc = oracle.chain(nq, x, z, c, ents, taus, 1e-8)
    rng = np.random.default_rng(63)
    idx = rng.integers(0, len(fc), 2000)
    found, val = oracle.chain_point(nq, x, z, c, ents, taus, 1e-8, fx[idx], fz[idx])
    assert found.all() and np.array_equal(val, fc[idx])
    table = {tuple(a) + tuple(b): v for a, b, v in zip(fx.tolist(), fz.tolist(), fc.tolist())}
    for j in (4, 2):
        qx = fx[idx] ^ cx[j]
        qz = fz[idx] ^ cz[j]
        f2, v2 = oracle.chain_point(nq, x, z, c, ents, taus, 1e-8, qx, qz)
        for a, b, f, v in zip(qx.tolist(), qz.tolist(), f2, v2):
            k = tuple(a) + tuple(b)
            assert f == (k in table)
            if f:
                assert v == table[k]
