"""The allocation-free QMF energy entry point (iqcc_qmf_energy_noalloc) against
iqcc_qmf_energy, which allocates its own scratch: two calls in a row on one
context, the second on a smaller Hamiltonian, each equal to the allocating
entry point bit for bit and to the oracle within 1e-10 (Eq. 3)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import describe

pytestmark = pytest.mark.gpu


def test_noalloc_energy_matches_allocating_entry_point():
    ctx = iqcc.Context(0)
    cases = [(40, I.hamiltonian_dense(40, 1)), (8, I.hamiltonian_dense(8, 0))]   # larger first
    for nq, (x, z, c) in cases:
        th, ph = I.qmf_angles(nq, np.random.default_rng(nq))
        tht, pht = torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()
        s = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
        describe(0, "qmf_energy_noalloc", nq=nq, n=len(c))
        e_na = iqcc.iqcc_qmf_energy_noalloc(ctx.handle, s.handle, tht, pht)
        e_ref = iqcc.iqcc_qmf_energy(ctx.handle, s.handle, tht, pht)
        e_na2 = iqcc.iqcc_qmf_energy_noalloc(ctx.handle, s.handle, tht, pht)
        torch.cuda.synchronize()
        a, b, a2 = float(e_na.item()), float(e_ref.item()), float(e_na2.item())
        assert a == b and a2 == b, (nq, a, b, a2)
        assert abs(a - O.qmf_energy(nq, x, z, c, th, ph)) <= 1e-10
        s.close()
    # a grid larger than the fixed scratch holds is refused before any launch
    old = iqcc.iqcc_get_param(ctx.handle, "energy_grid_per_cu")
    try:
        iqcc.iqcc_set_param(ctx.handle, "energy_grid_per_cu", 32)
        n_cu = iqcc.iqcc_get_param(ctx.handle, "n_cu")
        x, z, c = cases[1][1]
        s = iqcc.Store(ctx, 8, 2 * len(c)).load_numpy(x, z, c)
        th, ph = I.qmf_angles(8, np.random.default_rng(8))
        tht, pht = torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()
        if 32 * n_cu > iqcc.NOALLOC_MAX_PARTIALS:
            with pytest.raises(iqcc.IqccError) as e:
                iqcc.iqcc_qmf_energy_noalloc(ctx.handle, s.handle, tht, pht)
            assert e.value.code == iqcc.IQCC_ERR_CAPACITY
        s.close()
    finally:
        iqcc.iqcc_set_param(ctx.handle, "energy_grid_per_cu", old)
    ctx.close()
