"""Batched DIS screening at the full workload (1e7-term 100-qubit screening
Hamiltonian, 1e4 candidates of weight 2-12) against oracle gradients of a
seeded sample of 32 candidates (tests/golden/c4a_dis.json): the sampled
entries of the full 1e4-candidate launch (many candidate tiles, bucket-prefix
search over several chunks per range), a launch on the sample alone and the
plain per-candidate form all agree with the oracle within 1e-10 Ha."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import describe
from tests.golden.multiset_hash import multiset_hash

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c4a_dis.json")


def test_dis_full_workload_against_oracle_sample():
    gold = json.load(open(GOLDEN))
    nq, config = 100, 3
    x, z, c = I.hamiltonian_expanded(nq, config, 10**7)
    assert f"{multiset_hash(x, z, c):016x}" == gold["initial_digest"], "input generator changed"
    cx, cz = I.dis_candidates(x, nq, 10**4, 12, I.rng_for(config, I.PURPOSE_CANDIDATES))
    th, ph = I.qmf_angles(nq, I.rng_for(config, I.PURPOSE_ANGLES))
    idx = np.array(gold["sample_index"])
    ref = np.array([v["value"] for v in gold["grad"]])
    ctx = iqcc.Context(0)
    h = iqcc.Store(ctx, nq, len(c)).load_numpy(x, z, c)
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    describe(0, "dis full", n=len(c), n_cand=len(cx))
    g = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, iqcc.to_device_words(cx),
                                iqcc.to_device_words(cz), iqcc.IQCC_DIS_BATCHED).cpu().numpy()
    assert np.abs(g[idx] - ref).max() <= 1e-10
    # fewer ranges than the default: each holds several 512-bucket chunks
    try:
        iqcc.iqcc_set_param(ctx.handle, "dis_bucket_ranges", 16)
        describe(1, "dis full, 16 bucket ranges")
        g16 = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, iqcc.to_device_words(cx),
                                      iqcc.to_device_words(cz), iqcc.IQCC_DIS_BATCHED).cpu().numpy()
    finally:
        iqcc.iqcc_set_param(ctx.handle, "dis_bucket_ranges", 0)
    assert np.abs(g16[idx] - ref).max() <= 1e-10
    sx, sz = iqcc.to_device_words(cx[idx]), iqcc.to_device_words(cz[idx])
    describe(2, "dis sample batched + plain", n_cand=len(idx))
    gs = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, sx, sz, iqcc.IQCC_DIS_BATCHED).cpu().numpy()
    gp = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, sx, sz, iqcc.IQCC_DIS_PLAIN).cpu().numpy()
    assert np.abs(gs - ref).max() <= 1e-10
    assert np.abs(gp - ref).max() <= 1e-10
    h.close(); ctx.close()
