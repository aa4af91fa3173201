"""Pins of the oracle's Pauli algebra against explicit 2x2 / 2^n matrices."""
import itertools

import numpy as np

from oracle import dense as D

SINGLE = {"I": (0, 0), "X": (1, 0), "Y": (1, 1), "Z": (0, 1)}
MATS = {"I": D.I2, "X": D.X2, "Y": D.Y2, "Z": D.Z2}


def _key(nq, text):
    x = np.zeros(1, np.uint64); z = np.zeros(1, np.uint64)
    for i, ch in enumerate(text):
        bx, bz = SINGLE[ch]
        if bx:
            x[0] |= np.uint64(1 << i)
        if bz:
            z[0] |= np.uint64(1 << i)
    return x, z


def test_single_qubit_table(oracle):
    # XY = iZ, YZ = iX, ZX = iY, reverses carry -i, squares are I
    for a, b in itertools.product("IXYZ", repeat=2):
        x1, z1 = _key(1, a); x2, z2 = _key(1, b)
        x3, z3, e = oracle.pauli_product(1, x1, z1, x2, z2)
        lhs = MATS[a] @ MATS[b]
        rhs = (1j ** e) * D.pauli_matrix(1, x3, z3)
        assert np.allclose(lhs, rhs, atol=0), (a, b, e)
    expect = {("X", "Y"): ("Z", 1), ("Y", "X"): ("Z", 3), ("Y", "Z"): ("X", 1),
              ("Z", "Y"): ("X", 3), ("Z", "X"): ("Y", 1), ("X", "Z"): ("Y", 3)}
    for (a, b), (r, k) in expect.items():
        x1, z1 = _key(1, a); x2, z2 = _key(1, b)
        x3, z3, e = oracle.pauli_product(1, x1, z1, x2, z2)
        xr, zr = _key(1, r)
        assert e == k and x3[0] == xr[0] and z3[0] == zr[0]


def test_products_brute_force_n3(oracle):
    nq = 3
    for a in itertools.product("IXYZ", repeat=nq):
        for b in itertools.product("IXYZ", repeat=nq):
            x1, z1 = _key(nq, a); x2, z2 = _key(nq, b)
            x3, z3, e = oracle.pauli_product(nq, x1, z1, x2, z2)
            # key of the product is the XOR of the keys
            assert x3[0] == x1[0] ^ x2[0] and z3[0] == z1[0] ^ z2[0]
            M1 = D.pauli_matrix(nq, x1, z1); M2 = D.pauli_matrix(nq, x2, z2)
            assert np.array_equal(M1 @ M2, (1j ** e) * D.pauli_matrix(nq, x3, z3))
            anti = np.allclose(M1 @ M2, -(M2 @ M1))
            assert anti == (e % 2 == 1)


def test_multiword_products(oracle):
    # qubits straddling the 64-bit word boundary: compare against per-word products
    rng = np.random.default_rng(7)
    nq = 130
    for _ in range(50):
        x1, z1, x2, z2 = (rng.integers(0, 2**63, size=3, dtype=np.uint64) for _ in range(4))
        for arr in (x1, z1, x2, z2):
            arr[2] &= np.uint64(0x3)          # 130 qubits: two bits in word 2
        x3, z3, e = oracle.pauli_product(nq, x1, z1, x2, z2)
        assert np.array_equal(x3, x1 ^ x2) and np.array_equal(z3, z1 ^ z2)
        # phase: product of the three single-word (64-qubit) pieces
        tot = 0
        for w, nqw in ((0, 64), (1, 64), (2, 2)):
            _, _, ew = oracle.pauli_product(nqw, x1[w:w + 1], z1[w:w + 1], x2[w:w + 1], z2[w:w + 1])
            tot += ew
        assert e == tot % 4
