"""The seeded input generators: JW image against a dense fermionic construction,
integral symmetries, DIS-candidate admissibility, determinism."""
import numpy as np
import pytest

from oracle import dense as D
from paper_2603_08883_amd import inputs as I


def _dense_fermion_hamiltonian(h, g):
    n = h.shape[0]
    nq = 2 * n

    def ann(j):
        M = np.ones((1, 1), complex)
        for q in reversed(range(nq)):
            op = D.Z2 if q < j else (np.array([[0, 1], [0, 0]], complex) if q == j else D.I2)
            M = np.kron(M, op)
        return M

    a = [ann(j) for j in range(nq)]
    ad = [m.conj().T for m in a]
    dim = 1 << nq
    H = np.zeros((dim, dim), complex)
    for p in range(n):
        for q in range(n):
            for s in range(2):
                H += h[p, q] * ad[2 * p + s] @ a[2 * q + s]
    for p in range(n):
        for q in range(n):
            for r in range(n):
                for t in range(n):
                    if g[p, q, r, t] == 0:
                        continue
                    for s in range(2):
                        for u in range(2):
                            H += 0.5 * g[p, q, r, t] * ad[2 * p + s] @ ad[2 * r + u] @ a[2 * t + u] @ a[2 * q + s]
    return H


@pytest.mark.parametrize("n_spatial,band", [(2, None), (3, None), (4, 1)])
def test_jw_matches_dense_fermions(n_spatial, band):
    h, g = I.integrals(n_spatial, np.random.default_rng(n_spatial), band=band, decay=3.0)
    x, z, c = I.jw_hamiltonian(h, g)
    nq = 2 * n_spatial
    Hp = D.hamiltonian_matrix(nq, x, z, c)
    Hf = _dense_fermion_hamiltonian(h, g)
    assert np.abs(Hp - Hf).max() <= 1e-13 * np.abs(c).sum()
    # unique keys, real JW image has an even number of Y's in every word
    keys = {tuple(a) + tuple(b) for a, b in zip(x.tolist(), z.tolist())}
    assert len(keys) == len(c)
    assert np.all(np.bitwise_count(x & z).sum(1) % 2 == 0)


def test_integral_symmetry_and_band():
    h, g = I.integrals(7, np.random.default_rng(1), band=2, decay=3.0)
    assert np.array_equal(h, h.T)
    for perm in ((1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)):
        assert np.array_equal(g, g.transpose(perm))
    p, q, r, s = np.nonzero(g)
    assert np.all(np.abs(p - q) <= 2) and np.all(np.abs(r - s) <= 2)


def test_generator_is_seeded():
    a = I.hamiltonian_dense(8, 0)
    b = I.hamiltonian_dense(8, 0)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_two_word_keys():
    # qubits above 63 land in the second word
    h, g = I.integrals(34, np.random.default_rng(2), band=1, decay=3.0)
    x, z, c = I.jw_hamiltonian(h, g)
    assert x.shape[1] == 2 and np.any(x[:, 1]) and np.any(z[:, 1])
    assert np.all(x[:, 1] >> np.uint64(4) == 0) and np.all(z[:, 1] >> np.uint64(4) == 0)


def test_dis_candidates_admissible():
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, 200, 8, I.rng_for(1, I.PURPOSE_CANDIDATES))
    flips = {tuple(r) for r in x.tolist()}
    seen = set()
    for a in range(200):
        ny = int(np.bitwise_count(cx[a] & cz[a]).sum())
        w = int(np.bitwise_count(cx[a] | cz[a]).sum())
        assert ny % 2 == 1
        assert tuple(cx[a].tolist()) in flips
        assert 2 <= w <= 8
        k = tuple(cx[a].tolist()) + tuple(cz[a].tolist())
        assert k not in seen
        seen.add(k)
