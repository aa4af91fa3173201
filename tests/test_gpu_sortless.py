"""The sortless-dressing path (App. D) against the oracle: its output must be
the oracle's dressed Hamiltonian in canonical order, element by element (keys
and coefficients bit for bit), including the degenerate cases."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import describe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


def _run(ctx, nq, x, z, c, px, pz, tau, eps):
    x, z, c = O.canonical(x, z, c)
    ox, oz, oc = iqcc.iqcc_sortless_dress(ctx.handle, nq, iqcc.to_device_words(x), iqcc.to_device_words(z),
                                          torch.from_numpy(np.ascontiguousarray(c)).cuda(), px, pz, tau, eps)
    return iqcc.from_device_words(ox), iqcc.from_device_words(oz), oc.cpu().numpy()


def _check_exact(got, ref, what):
    gx, gz, gc = got
    rx, rz, rc = O.canonical(*ref)
    assert gx.shape == rx.shape, (what, gx.shape, rx.shape)
    assert np.array_equal(gx, rx) and np.array_equal(gz, rz), what      # same keys, same order
    assert np.array_equal(gc, rc), what                                   # bit for bit


@pytest.mark.parametrize("nq,kind,eps", [(12, "dense", 0.0), (40, "dense", 1e-8), (124, "banded", 1e-8)])
def test_sortless_step_matches_oracle(ctx, nq, kind, eps):
    if kind == "dense":
        x, z, c = I.hamiltonian_dense(nq, 9 if nq == 12 else 1)
    else:
        x, z, c = I.hamiltonian_banded(nq, 7, band=2)
    cx, cz = I.dis_candidates(x, nq, 3, 8, np.random.default_rng(nq + 3))
    for k, tau in enumerate((0.17, -0.4, 1.3)):
        describe(k, "sortless", nq=nq, n=len(c), eps=eps)
        got = _run(ctx, nq, x, z, c, cx[k], cz[k], tau, eps)
        _check_exact(got, O.dress(nq, x, z, c, cx[k], cz[k], tau, eps), f"{nq}q step {k}")


def test_sortless_chain_and_degenerate_cases(ctx):
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, 4, 8, np.random.default_rng(11))
    taus = [0.1, -0.2, 0.15, 0.05]
    gx, gz, gc = x, z, c
    ox, oz, oc = x, z, c
    for j in range(4):
        describe(j, "sortless chain", n=len(gc))
        gx, gz, gc = _run(ctx, nq, gx, gz, gc, cx[j], cz[j], taus[j], 1e-8)
        ox, oz, oc = O.dress(nq, ox, oz, oc, cx[j], cz[j], taus[j], 1e-8)
        _check_exact((gx, gz, gc), (ox, oz, oc), f"chain step {j}")
    zero = np.zeros(1, np.uint64)
    _check_exact(_run(ctx, nq, x, z, c, zero, zero, 0.3, 0.0), O.dress(nq, x, z, c, zero, zero, 0.3, 0.0), "identity")
    _check_exact(_run(ctx, nq, x, z, c, cx[0], cz[0], 0.0, 0.0), O.dress(nq, x, z, c, cx[0], cz[0], 0.0, 0.0), "tau 0")
    _check_exact(_run(ctx, nq, x, z, c, cx[0], cz[0], 0.3, 1e9), O.dress(nq, x, z, c, cx[0], cz[0], 0.3, 1e9), "all dropped")
    _check_exact(_run(ctx, nq, x[:1], z[:1], c[:1], cx[0], cz[0], 0.3, 0.0),
                 O.dress(nq, x[:1], z[:1], c[:1], cx[0], cz[0], 0.3, 0.0), "one term")


def test_sortless_rejects_bad_arguments(ctx):
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    x, z, c = O.canonical(x, z, c)
    dx, dz = iqcc.to_device_words(x), iqcc.to_device_words(z)
    dc = torch.from_numpy(np.ascontiguousarray(c)).cuda()
    wide = np.array([(1 << 21) - 1], np.uint64)          # flips 21 key bits
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_sortless_dress(ctx.handle, nq, dx, dz, dc, wide, np.zeros(1, np.uint64), 0.1, 0.0)
    with pytest.raises(iqcc.IqccError) as ei:            # no room for the result
        iqcc.iqcc_sortless_dress(ctx.handle, nq, dx, dz, dc, np.array([3], np.uint64),
                                 np.array([1], np.uint64), 0.1, 0.0, cap=10)
    assert ei.value.code == iqcc.IQCC_ERR_CAPACITY
