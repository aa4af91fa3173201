"""The all-cores form of the oracle step (CPU-baseline leg) against the serial
oracle: the same terms and coefficient bits, and the same energy bits, for any
thread count (Sec. II Eq. 5 dressing, App. D merge, App. A compression, Eq. 3
energy)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I


@pytest.mark.parametrize("eps", [0.0, 1e-8, 1e-3])
def test_parallel_step_equals_serial(eps):
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, 2, 8, np.random.default_rng(5))
    th, ph = I.qmf_angles(nq, np.random.default_rng(6))
    ref = O.canonical(*O.dress(nq, x, z, c, cx[0], cz[0], 0.17, eps))
    e_ref = O.qmf_energy(nq, *ref, th, ph)
    for T in (1, 2, 5):
        got = O.canonical(*O.dress_par(nq, x, z, c, cx[0], cz[0], 0.17, eps, T))
        assert got[0].shape == ref[0].shape
        for a, b in zip(got, ref):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert O.qmf_energy_par(nq, *ref, th, ph, T) == e_ref


def test_parallel_step_small_inputs():
    nq = 8
    x, z, c = I.hamiltonian_dense(nq, 0)
    px, pz = I.single_qubit_pauli(nq, "XXXY")
    for n in (0, 1, 5):
        ref = O.canonical(*O.dress(nq, x[:n], z[:n], c[:n], px, pz, 0.1, 0.0))
        got = O.canonical(*O.dress_par(nq, x[:n], z[:n], c[:n], px, pz, 0.1, 0.0, 3))
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)
