"""Pins of the oracle's term-limit selection: properties that any correct
"largest |c| first, smaller canonical key first among equals" selection has."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I


def _canon(x, z):
    W = len(x)
    return tuple(int(x[w]) for w in range(W - 1, -1, -1)) + tuple(int(z[w]) for w in range(W - 1, -1, -1))


def _tied_hamiltonian(nq, cfg, levels, seed):
    x, z, c = I.hamiltonian_dense(nq, cfg)
    rng = np.random.default_rng(seed)
    return x, z, rng.choice(levels, len(c)) * rng.choice([-1.0, 1.0], len(c))


@pytest.mark.parametrize("levels", [None, [0.5, 0.25, 0.125], [1.0]])
def test_selection_properties(oracle, levels):
    if levels is None:
        x, z, c = I.hamiltonian_dense(12, 9)
    else:
        x, z, c = _tied_hamiltonian(12, 9, levels, 3)
    n = len(c)
    allk = {_canon(a, b): v for a, b, v in zip(x, z, c)}
    for M in (0, 1, 7, n // 3, n // 2, n - 1, n, n + 5):
        kx, kz, kc = O.truncate_top(x, z, c, M)
        assert len(kc) == min(M, n)
        kept = {_canon(a, b): v for a, b, v in zip(kx, kz, kc)}
        assert len(kept) == len(kc)
        assert all(allk[k] == v for k, v in kept.items())          # coefficients untouched
        dropped = [k for k in allk if k not in kept]
        if kept and dropped:
            lo = min(abs(v) for v in kept.values())
            hi = max(abs(allk[k]) for k in dropped)
            assert lo >= hi
            if lo == hi:   # the boundary is a tie: kept keys precede dropped keys
                assert max(k for k, v in kept.items() if abs(v) == lo) < \
                    min(k for k in dropped if abs(allk[k]) == hi)


def test_selection_ignores_input_order(oracle):
    x, z, c = _tied_hamiltonian(12, 9, [0.5, 0.25], 5)
    p = np.random.default_rng(1).permutation(len(c))
    for M in (10, len(c) // 2):
        a = O.truncate_top(x, z, c, M)
        b = O.truncate_top(x[p], z[p], c[p], M)
        assert all(np.array_equal(u, v) for u, v in zip(a, b))


def test_worked_example(oracle):
    """Five one-qubit-word terms with hand-checked selections."""
    x = np.array([[1], [2], [3], [0], [1]], np.uint64)
    z = np.array([[0], [0], [1], [1], [1]], np.uint64)
    c = np.array([0.5, -0.5, 0.25, -1.0, 0.5])
    # |c| = .5 .5 .25 1 .5; keys (x, z): (1,0) (2,0) (3,1) (0,1) (1,1)
    kx, kz, kc = O.truncate_top(x, z, c, 3)
    # -1.0 first, then the two smallest keys among the three 0.5 terms: (1,0), (1,1)
    got = sorted(zip(kx[:, 0].tolist(), kz[:, 0].tolist(), kc.tolist()))
    assert got == [(0, 1, -1.0), (1, 0, 0.5), (1, 1, 0.5)]
