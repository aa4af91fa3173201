"""The multi-generator energy polynomial on the GPU against the oracle's:
coefficients within 1e-10 of the 1-norm scale, and the polynomial against
oracle chain energies at off-grid amplitudes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import qcc as Q
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import describe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("nq,cfg,n", [(12, 9, 3), (20, 1, 2)])
def test_energy_polynomial_matches_oracle(ctx, nq, cfg, n):
    x, z, c = I.hamiltonian_dense(nq, cfg)
    th, ph = I.qmf_angles(nq, np.random.default_rng(nq))
    cx, cz = Q.dis_generators(Q.flip_sets(x, 4))
    pick = np.random.default_rng(nq + 1).choice(len(cx), n, replace=False)
    pxs, pzs = cx[pick], cz[pick]
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
    work = [iqcc.Store(ctx, nq, 2 * len(c) * 2 ** (k + 1)) for k in range(n)]
    describe(0, "trig poly", nq=nq, n_terms=len(c), n=n)
    got = iqcc.iqcc_energy_trig_poly(ctx.handle, h.handle, pxs, pzs, tht, pht, work)
    ref = Q.energy_trig_poly(nq, x, z, c, pxs, pzs, th, ph)
    s = np.abs(c).sum()
    assert np.abs(got - ref).max() <= 1e-12 * s
    for tau in np.random.default_rng(3).uniform(-2, 2, (3, n)):
        hx, hz, hc = x, z, c
        for k in range(n):
            hx, hz, hc = O.dress(nq, hx, hz, hc, pxs[k], pzs[k], tau[k], 0.0)
        assert abs(iqcc.iqcc_trig_poly_eval(got, tau) - O.qmf_energy(nq, hx, hz, hc, th, ph)) <= 1e-11 * s
    tau, e = iqcc.iqcc_trig_poly_minimize(got, np.zeros(n), sweeps=200)
    assert e <= iqcc.iqcc_trig_poly_eval(got, np.zeros(n)) + 1e-12
    h.close()
    for w in work:
        w.close()


def test_energy_polynomial_rejects_bad_arguments(ctx):
    x, z, c = I.hamiltonian_dense(12, 9)
    th, ph = I.qmf_angles(12, np.random.default_rng(1))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, 12, 2 * len(c)).load_numpy(x, z, c)
    w = iqcc.Store(ctx, 12, 8 * len(c))
    cx, cz = Q.dis_generators(Q.flip_sets(x, 2))
    with pytest.raises(iqcc.IqccError):        # the same work store twice
        iqcc.iqcc_energy_trig_poly(ctx.handle, h.handle, cx[:2], cz[:2], tht, pht, [w, w])
    with pytest.raises(iqcc.IqccError):        # more than 8 generators
        iqcc.iqcc_energy_trig_poly(ctx.handle, h.handle, cx[:9], cz[:9], tht, pht, [w] * 9)
    h.close(); w.close()
