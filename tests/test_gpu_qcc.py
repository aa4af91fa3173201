"""The iQCC iteration on the GPU against the oracle's plain loop.

Flip sets exactly; the anticommuting energy within 1e-10 (relative to the
1-norm of the coefficients); candidates, the selected generators and their
order exactly; gradients, closed-form amplitudes and energies within 1e-10;
the dressed Hamiltonian with the same keys and coefficients within 1e-12
relative (the amplitudes come from sums whose rounding order differs, so the
coefficients are not bit-identical)."""
import numpy as np
import pytest
import torch

from oracle import qcc as Q
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from paper_2603_08883_amd import qcc as G
from tests.gpu_util import describe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


def _assert_close_terms(got, ref, rtol=1e-12):
    gx, gz, gc = got
    rx, rz, rc = ref
    ga = {tuple(a.tolist()) + tuple(b.tolist()): v for a, b, v in zip(gx, gz, gc)}
    ra = {tuple(a.tolist()) + tuple(b.tolist()): v for a, b, v in zip(rx, rz, rc)}
    assert ga.keys() == ra.keys()
    k = np.array(list(ra.keys()), dtype=object)
    g = np.array([ga[t] for t in ra]); r = np.array([ra[t] for t in ra])
    assert np.all(np.abs(g - r) <= rtol * np.abs(r) + 1e-300), np.abs(g - r).max()


@pytest.mark.parametrize("nq,cfg,band", [(40, 1, None), (124, 7, 2)])
def test_flip_sets_and_energy_anti(ctx, nq, cfg, band):
    if band is None:
        x, z, c = I.hamiltonian_dense(nq, cfg)
    else:
        x, z, c = I.hamiltonian_banded(nq, cfg, band=band)
    describe(0, "flip sets", nq=nq, n=len(c))
    h = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
    for w_max in (2, 4, 64):
        F = iqcc.iqcc_flip_sets(ctx.handle, h.handle, w_max)
        assert np.array_equal(F, Q.flip_sets(x, w_max)), w_max
    th, ph = I.qmf_angles(nq, np.random.default_rng(4))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    cx, cz = Q.dis_generators(Q.flip_sets(x, 2))
    s = np.abs(c).sum()
    for k in (0, len(cx) // 2, len(cx) - 1):
        b = iqcc.iqcc_qmf_energy_anti(ctx.handle, h.handle, cx[k], cz[k], tht, pht).item()
        assert abs(b - Q.energy_anti(nq, x, z, c, cx[k], cz[k], th, ph)) <= 1e-12 * max(1.0, s)
    h.close()


@pytest.mark.parametrize("nq,cfg,w_max,n_select,eps,iters",
                         [(12, 9, 6, 4, 0.0, 2), (20, 1, 2, 3, 1e-8, 2)])
def test_iteration_matches_oracle(ctx, nq, cfg, w_max, n_select, eps, iters):
    x, z, c = I.hamiltonian_dense(nq, cfg)
    th, ph = I.qmf_angles(nq, np.random.default_rng(30 + nq))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    cap = 4 * len(c) * 4 ** iters
    h = iqcc.Store(ctx, nq, cap).load_numpy(x, z, c)
    spare = iqcc.Store(ctx, nq, cap)
    ox, oz, oc = x, z, c
    for it in range(iters):
        describe(it, "qcc iteration", nq=nq, n=len(oc), w_max=w_max, n_select=n_select)
        got = iqcc.iqcc_qcc_iteration(ctx.handle, h, spare, tht, pht, w_max, n_select, eps)
        ref, (ox, oz, oc) = Q.qcc_iteration(nq, ox, oz, oc, th, ph, w_max, n_select, eps)
        assert got["n_candidates"] == ref["n_candidates"]
        assert np.array_equal(got["sel_x"], ref["sel_x"]) and np.array_equal(got["sel_z"], ref["sel_z"])
        assert np.abs(got["sel_g"] - ref["sel_g"]).max() <= 1e-10
        assert np.abs(got["sel_tau"] - ref["sel_tau"]).max() <= 1e-10
        assert np.abs(got["energy"] - ref["energy"]).max() <= 1e-10
        assert len(got["sel_tau"]) == n_select
        _assert_close_terms(h.to_numpy(), (ox, oz, oc))
    h.close(); spare.close()


def test_outer_loop_converges(ctx):
    """Energies fall monotonically and the loop stops on the tolerance or the cap."""
    nq = 12
    x, z, c = I.hamiltonian_dense(nq, 9)
    th, ph = I.qmf_angles(nq, np.random.default_rng(5))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, nq, 1 << 20).load_numpy(x, z, c)
    spare = iqcc.Store(ctx, nq, 1 << 20)
    hist = G.run(ctx, h, spare, tht, pht, w_max=6, n_select=2, eps=1e-10, max_iter=6, tol=1e-6)
    es = np.concatenate([r["energy"] for r in hist])
    assert all(b <= a + 1e-12 for a, b in zip(es, es[1:]))
    assert es[-1] < es[0] - 1e-3
    last = hist[-1]
    assert len(hist) == 6 or abs(last["energy"][-1] - last["energy"][0]) < 1e-6 or len(last["sel_tau"]) == 0
    h.close(); spare.close()


def test_iteration_rejects_bad_arguments(ctx):
    x, z, c = I.hamiltonian_dense(12, 9)
    th, ph = I.qmf_angles(12, np.random.default_rng(1))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, 12, 4 * len(c)).load_numpy(x, z, c)
    with pytest.raises(iqcc.IqccError):        # h and spare are the same store
        iqcc.iqcc_qcc_iteration(ctx.handle, h, h, tht, pht, 4, 2, 1e-8)
    spare = iqcc.Store(ctx, 12, 4 * len(c))
    with pytest.raises(iqcc.IqccError):        # w_max < 1
        iqcc.iqcc_qcc_iteration(ctx.handle, h, spare, tht, pht, 0, 2, 1e-8)
    assert iqcc.iqcc_flip_sets(ctx.handle, h.handle, 64).shape[1] == 1
    h.close(); spare.close()
