"""Batched dressing of many uneven Hamiltonians: one persistent launch, and
the same launch captured in a HIP graph and replayed."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import assert_same_terms, describe
from tests.golden.multiset_hash import multiset_hash_torch

pytestmark = pytest.mark.gpu
EPS = 1e-8


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def hams():
    hs = I.batch_hamiltonians(41, n_ham=12, q_lo=16, q_hi=40, size_lo=1e3, size_hi=1e5)
    # degenerate members: a single term and an empty Hamiltonian
    one = dict(hs[0]); one.update(x=hs[0]["x"][:1], z=hs[0]["z"][:1], c=hs[0]["c"][:1])
    empty = dict(hs[1]); empty.update(x=hs[1]["x"][:0], z=hs[1]["z"][:0], c=hs[1]["c"][:0])
    return hs + [one, empty]


def _stores(ctx, hs):
    ins, outs = [], []
    for h in hs:
        cap = max(4 * len(h["c"]), 64)
        ins.append(iqcc.Store(ctx, h["n_qubits"], cap).load_numpy(h["x"], h["z"], h["c"]))
        outs.append(iqcc.Store(ctx, h["n_qubits"], cap))
    return ins, outs


def _refs(hs):
    return [O.dress(h["n_qubits"], h["x"], h["z"], h["c"], h["px"], h["pz"], h["tau"], EPS) for h in hs]


def _args(hs):
    W = 1
    pxs = np.array([np.asarray(h["px"], np.uint64).reshape(W) for h in hs])
    pzs = np.array([np.asarray(h["pz"], np.uint64).reshape(W) for h in hs])
    return pxs, pzs, [h["tau"] for h in hs]


def test_batched_matches_oracle(ctx, hams):
    ins, outs = _stores(ctx, hams)
    pxs, pzs, taus = _args(hams)
    describe(0, "dress_batched", n_ham=len(hams), terms=sum(len(h["c"]) for h in hams))
    iqcc.iqcc_dress_batched(ctx.handle, [s.handle for s in ins], [s.handle for s in outs], pxs, pzs, taus, EPS)
    for i, (o, r) in enumerate(zip(outs, _refs(hams))):
        assert_same_terms(o.to_numpy(), r, f"item {i}")


def test_batched_graph_replays(ctx, hams):
    ins, outs = _stores(ctx, hams)
    pxs, pzs, taus = _args(hams)
    refs = _refs(hams)
    describe(0, "batch graph", n_ham=len(hams))
    b = iqcc.iqcc_batch_create(ctx.handle, [s.handle for s in ins], [s.handle for s in outs], pxs, pzs, taus, EPS)
    try:
        for rep in range(3):
            describe(rep, "batch graph replay")
            iqcc.iqcc_batch_launch(ctx.handle, b)
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(outs, refs)):
                assert_same_terms(o.to_numpy(), r, f"replay {rep} item {i}")
            # unrelated eager work between replays
            t = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
            assert torch.isfinite(t.sum()).item()
            torch.cuda.synchronize()
    finally:
        iqcc.iqcc_batch_destroy(ctx.handle, b)


def test_batch_rejects_aliasing(ctx, hams):
    ins, outs = _stores(ctx, hams[:2])
    pxs, pzs, taus = _args(hams[:2])
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_dress_batched(ctx.handle, [ins[0].handle, ins[1].handle], [outs[0].handle, outs[0].handle],
                                pxs, pzs, taus, EPS)
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_dress_batched(ctx.handle, [ins[0].handle, ins[1].handle], [outs[0].handle, ins[0].handle],
                                pxs, pzs, taus, EPS)


def test_full_batch_graph_against_oracle_digests(ctx):
    """The 64-Hamiltonian batch of the benchmark (16-64 qubits, 1e3-1e6 terms),
    captured once and replayed twice: each output's size and digest equal the
    oracle's (tests/golden/c4b_batch.json)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "c4b_batch.json")))["items"]
    hs = I.batch_hamiltonians(4)
    assert [len(h["c"]) for h in hs] == [g["n_in"] for g in gold]
    ins = [iqcc.Store(ctx, h["n_qubits"], max(2 * len(h["c"]), 64)).load_numpy(h["x"], h["z"], h["c"])
           for h in hs]
    outs = [iqcc.Store(ctx, h["n_qubits"], max(2 * len(h["c"]), 64)) for h in hs]
    pxs, pzs, taus = _args(hs)
    b = iqcc.iqcc_batch_create(ctx.handle, [s.handle for s in ins], [s.handle for s in outs], pxs, pzs,
                               taus, EPS)
    try:
        for rep in range(2):
            describe(rep, "full batch graph replay", n_ham=len(hs))
            iqcc.iqcc_batch_launch(ctx.handle, b)
            torch.cuda.synchronize()
            for i, (o, g) in enumerate(zip(outs, gold)):
                n_anti, _ = iqcc.iqcc_store_stats(ctx.handle, o.handle)
                assert (o.count(), n_anti) == (g["n_out"], g["n_anti"]), (rep, i)
                gx, gz, gc = iqcc.iqcc_store_export(ctx.handle, o.handle)
                assert f"{multiset_hash_torch(gx, gz, gc):016x}" == g["digest"], (rep, i)
    finally:
        iqcc.iqcc_batch_destroy(ctx.handle, b)
    for s_ in ins + outs:
        s_.close()


@pytest.mark.parametrize("unit_pairs", [1, 3, 1000])
def test_batch_work_units(ctx, hams, unit_pairs):
    """Work units of one bucket pair, of an odd count that splits Hamiltonians
    unevenly, and of more pairs than any Hamiltonian has: the same terms as the
    oracle."""
    old = iqcc.iqcc_get_param(ctx.handle, "batch_unit_pairs")
    iqcc.iqcc_set_param(ctx.handle, "batch_unit_pairs", unit_pairs)
    try:
        ins, outs = _stores(ctx, hams)
        pxs, pzs, taus = _args(hams)
        describe(0, "dress_batched work units", unit_pairs=unit_pairs)
        iqcc.iqcc_dress_batched(ctx.handle, [s.handle for s in ins], [s.handle for s in outs], pxs, pzs,
                                taus, EPS)
        for i, (o, r) in enumerate(zip(outs, _refs(hams))):
            assert_same_terms(o.to_numpy(), r, f"unit_pairs {unit_pairs} item {i}")
    finally:
        iqcc.iqcc_set_param(ctx.handle, "batch_unit_pairs", old)


def test_autotuned_batch_bit_identical(ctx, hams, tmp_path, monkeypatch):
    """The autotuner's pick for the batch changes timing only: every output has
    the same (key, coefficient bits) multiset as under the default knobs."""
    from paper_2603_08883_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "autotune.json"))
    pxs, pzs, taus = _args(hams)
    defaults = {k: iqcc.iqcc_get_param(ctx.handle, k) for k in autotune.BATCH_SPACE}
    ins, outs = _stores(ctx, hams)
    hin, hout = [s.handle for s in ins], [s.handle for s in outs]
    describe(0, "batch under default knobs")
    iqcc.iqcc_dress_batched(ctx.handle, hin, hout, pxs, pzs, taus, EPS)
    ref = [f"{multiset_hash_torch(*iqcc.iqcc_store_export(ctx.handle, o.handle)):016x}" for o in outs]
    try:
        describe(0, "batch autotune")
        params, secs = autotune.tune_batch(ctx, hin, hout, pxs, pzs, taus, EPS, 1,
                                           sum(len(h["c"]) for h in hams), use_cache=False)
        assert secs > 0 and set(params) == set(autotune.BATCH_SPACE)
        assert all(iqcc.iqcc_get_param(ctx.handle, k) == v for k, v in params.items())
        ins2, outs2 = _stores(ctx, hams)
        iqcc.iqcc_dress_batched(ctx.handle, [s.handle for s in ins2], [s.handle for s in outs2], pxs, pzs,
                                taus, EPS)
        got = [f"{multiset_hash_torch(*iqcc.iqcc_store_export(ctx.handle, o.handle)):016x}" for o in outs2]
        assert got == ref
        # the choice is cached and re-applied without timing
        autotune.apply(ctx, defaults)
        again, _ = autotune.tune_batch(ctx, hin, hout, pxs, pzs, taus, EPS, 1,
                                       sum(len(h["c"]) for h in hams))
        assert again == params
    finally:
        autotune.apply(ctx, defaults)
