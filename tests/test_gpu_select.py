"""Term-limit selection on the GPU against the oracle: the kept set must be
identical (keys and coefficients bit for bit), including boundaries that fall
inside a run of equal |c|, and the result must be a valid dressing input."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import assert_same_terms, describe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


def _cases():
    x, z, c = I.hamiltonian_dense(40, 1)
    yield "40q", 40, x, z, c
    rng = np.random.default_rng(9)
    yield "40q-ties", 40, x, z, rng.choice([0.5, 0.25, 0.125, 1e-3], len(c)) * rng.choice([-1.0, 1.0], len(c))
    yield "40q-all-equal", 40, x, z, np.full(len(c), -0.75)
    x2, z2, c2 = I.hamiltonian_banded(124, 7, band=2)
    yield "124q", 124, x2, z2, c2
    yield "124q-ties", 124, x2, z2, np.round(c2, 3)


@pytest.mark.parametrize("case", list(range(5)))
def test_truncate_top_matches_oracle(ctx, case):
    name, nq, x, z, c = list(_cases())[case]
    n = len(c)
    keep = np.abs(c) > 0
    x, z, c = x[keep], z[keep], c[keep]
    n = len(c)
    a = iqcc.Store(ctx, nq, 2 * n).load_numpy(x, z, c)
    b = iqcc.Store(ctx, nq, 2 * n)
    for M in (0, 1, 1000, n // 3, n // 2, n - 1, n, n + 7):
        describe(M, "truncate_top", case=name, n=n)
        iqcc.iqcc_truncate_top(ctx.handle, a.handle, M, b.handle)
        assert b.count() == min(M, n)
        assert_same_terms(b.to_numpy(), O.truncate_top(x, z, c, M), f"{name} M={M}")
    a.close(); b.close()


def test_truncated_store_dresses_like_oracle(ctx):
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    M = len(c) // 3
    a = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
    b = iqcc.Store(ctx, nq, 2 * len(c))
    d = iqcc.Store(ctx, nq, 4 * len(c))
    iqcc.iqcc_truncate_top(ctx.handle, a.handle, M, b.handle)
    px, pz = I.dis_candidates(x, nq, 1, 8, np.random.default_rng(2))
    iqcc.iqcc_dress(ctx.handle, b.handle, px[0], pz[0], 0.13, 1e-8, d.handle)
    tx, tz, tc = O.truncate_top(x, z, c, M)
    assert_same_terms(d.to_numpy(), O.dress(nq, tx, tz, tc, px[0], pz[0], 0.13, 1e-8), "dress after truncation")
    a.close(); b.close(); d.close()


def test_truncate_top_rejects_bad_arguments(ctx):
    x, z, c = I.hamiltonian_dense(12, 9)
    a = iqcc.Store(ctx, 12, 2 * len(c)).load_numpy(x, z, c)
    small = iqcc.Store(ctx, 12, 8)
    for args in ((a.handle, 10, a.handle), (a.handle, -1, small.handle), (a.handle, 10, small.handle)):
        with pytest.raises(iqcc.IqccError):
            iqcc.iqcc_truncate_top(ctx.handle, *args)
    a.close(); small.close()
