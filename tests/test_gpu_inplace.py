"""In-place dressing (iqcc_dress_inplace) against the FP64 oracle.

The in-place step must leave exactly the terms and coefficients the oracle's
dressing + merge + compression gives (Sec. II Eq. 5, App. D, App. A), bit for
bit, and the QMF energy (Eq. 3) within 1e-10, on every path of the kernel:
rows rewritten in place, new keys appended, rows freed by compression and
refilled, buckets moved to the pool when their region is full, and
anticommuting sets larger than a wavefront's LDS stash (hash rounds).  The
same input layout must give the same rows and bits on every run.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2603_08883_amd import inputs as I
from paper_2603_08883_amd import iqcc
from tests.gpu_util import assert_same_terms, describe

pytestmark = pytest.mark.gpu

E_TOL = 1e-10
INPLACE = iqcc.IQCC_STORE_INPLACE


@pytest.fixture(scope="module")
def ctx():
    c = iqcc.Context(0)
    yield c
    c.close()


def _angles(nq, seed):
    th, ph = I.qmf_angles(nq, np.random.default_rng(seed))
    return th, ph, torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()


class _Params:
    def __init__(self, ctx, **kv):
        self.ctx, self.kv = ctx, kv

    def __enter__(self):
        self.old = {k: iqcc.iqcc_get_param(self.ctx.handle, k) for k in self.kv}
        for k, v in self.kv.items():
            iqcc.iqcc_set_param(self.ctx.handle, k, v)

    def __exit__(self, *a):
        for k, v in self.old.items():
            iqcc.iqcc_set_param(self.ctx.handle, k, v)


def _inplace_chain(ctx, nq, x, z, c, ents, taus, eps, th, ph, max_terms, params=None, carry=True,
                   compare=True):
    """Dress an in-place store step by step; compare every step with the oracle
    (terms, energy, anticommuting and new counts).  Returns the store."""
    params = params or {}
    tht, pht = torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda()
    with _Params(ctx, **params):
        s = iqcc.Store(ctx, nq, max_terms, INPLACE).load_numpy(x, z, c)
        e = torch.zeros(1, dtype=torch.float64, device="cuda")
        ox, oz, oc = x, z, c
        for j, ((px, pz), t) in enumerate(zip(ents, taus)):
            describe(j, "dress_inplace", nq=nq, n=len(oc), tau=t, eps=eps, params=params, carry=carry)
            iqcc.iqcc_dress_inplace(ctx.handle, s.handle, px, pz, t, eps, tht, pht,
                                    e if (carry and j > 0) else None, e)
            torch.cuda.synchronize()
            n_in = len(oc)
            rx, rz, rc = O.dress_raw(nq, ox, oz, oc, px, pz, t)
            n_anti = len(rc) - n_in
            ox, oz, oc = O.merge_truncate(rx, rz, rc, eps=eps)
            if compare:
                assert s.count() == len(oc), (j, s.count(), len(oc))
                assert_same_terms(s.to_numpy(), (ox, oz, oc), f"in-place step {j}")
                Eo = O.qmf_energy(nq, ox, oz, oc, th, ph)
                assert abs(float(e.item()) - Eo) <= E_TOL * max(1.0, abs(Eo)), (j, e.item(), Eo)
                a, _ = iqcc.iqcc_store_stats(ctx.handle, s.handle)
                assert a == n_anti, (j, a, n_anti)
    return s, (ox, oz, oc)


def test_inplace_chain_40q_matches_oracle(ctx):
    nq, steps = 40, 6
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(1, I.PURPOSE_ENTANGLERS))
    taus = I.taus(steps, I.rng_for(1, I.PURPOSE_TAUS))
    th, ph, _, _ = _angles(nq, 11)
    s, _ = _inplace_chain(ctx, nq, x, z, c, list(zip(cx, cz)), taus, 1e-8, th, ph, 8 * len(c))
    st = iqcc.iqcc_store_inplace_stats(ctx.handle, s.handle)
    assert st["relocated"] == 0, st     # default regions leave room for this growth
    s.close()


def test_inplace_chain_124q_matches_oracle(ctx):
    """Two-word keys: a small banded 124-qubit Hamiltonian, four steps."""
    nq, steps = 124, 4
    x, z, c = I.hamiltonian_banded(nq, 2, band=2, decay=3.0)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(2, I.PURPOSE_ENTANGLERS))
    taus = I.taus(steps, I.rng_for(2, I.PURPOSE_TAUS))
    th, ph, _, _ = _angles(nq, 12)
    s, _ = _inplace_chain(ctx, nq, x, z, c, list(zip(cx, cz)), taus, 1e-8, th, ph, 6 * len(c))
    s.close()


@pytest.mark.parametrize("eps", [0.0, 1e-3, 1e9])
def test_inplace_compression_refills_rows(ctx, eps):
    """eps = 0 keeps exact zeros; 1e-3 frees many rows (refilled from the end
    of each bucket); 1e9 empties the store.  The energy is summed in full."""
    nq, steps = 40, 3
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, np.random.default_rng(31))
    taus = [0.15, -0.11, 0.07]
    th, ph, _, _ = _angles(nq, 13)
    s, ref = _inplace_chain(ctx, nq, x, z, c, list(zip(cx, cz)), taus, eps, th, ph, 8 * len(c),
                            carry=False)
    if eps >= 1e9:
        assert s.count() == 0
    elif eps > 0:
        st = iqcc.iqcc_store_inplace_stats(ctx.handle, s.handle)
        assert st["freed"] > 0, st
    s.close()


def test_inplace_relocation_to_pool(ctx):
    """Regions of 16 rows: growing buckets move to the pool."""
    nq, steps = 40, 5
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, np.random.default_rng(41))
    taus = I.taus(steps, np.random.default_rng(42))
    th, ph, _, _ = _angles(nq, 14)
    s, _ = _inplace_chain(ctx, nq, x, z, c, list(zip(cx, cz)), taus, 1e-8, th, ph, 16 * len(c),
                          params={"inplace_region_rows": 16, "inplace_bucket_terms": 8})
    st = iqcc.iqcc_store_inplace_stats(ctx.handle, s.handle)
    assert st["pool_used"] > 0, st
    s.close()


def test_inplace_hash_rounds(ctx):
    """A stash of 16 entries per wavefront: most work items take the pool path
    with several residue classes of the pair hash."""
    nq, steps = 40, 3
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, np.random.default_rng(51))
    taus = I.taus(steps, np.random.default_rng(52))
    th, ph, _, _ = _angles(nq, 15)
    s, _ = _inplace_chain(ctx, nq, x, z, c, list(zip(cx, cz)), taus, 1e-8, th, ph, 16 * len(c),
                          params={"inplace_cap": 16})
    st = iqcc.iqcc_store_inplace_stats(ctx.handle, s.handle)
    assert st["relocated"] > 0, st
    s.close()


def test_inplace_small_cases(ctx):
    """8 qubits (the XXXY step of the smallest workload), an identity
    entangler, a single term and an empty store."""
    nq = 8
    x, z, c = I.hamiltonian_dense(nq, 0)
    px, pz = I.single_qubit_pauli(nq, "XXXY")
    th, ph, tht, pht = _angles(nq, 16)
    s, _ = _inplace_chain(ctx, nq, x, z, c, [(px, pz)], [0.1], 0.0, th, ph, 4 * len(c))
    s.close()
    zero = np.zeros(1, np.uint64)
    s, _ = _inplace_chain(ctx, nq, x, z, c, [(zero, zero)], [0.3], 0.0, th, ph, 4 * len(c))
    s.close()
    s, _ = _inplace_chain(ctx, nq, x[:1], z[:1], c[:1], [(px, pz)], [0.2], 0.0, th, ph, 64)
    s.close()
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = iqcc.Store(ctx, nq, 64, INPLACE).load_numpy(x[:0], z[:0], c[:0])
    iqcc.iqcc_dress_inplace(ctx.handle, s.handle, px, pz, 0.2, 0.0, tht, pht, None, e)
    assert s.count() == 0 and float(e.item()) == 0.0
    s.close()


def test_inplace_same_rows_every_run(ctx):
    """Two chains from copies of one loaded store: identical rows (export
    order) and identical energy bits."""
    nq, steps = 40, 4
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, np.random.default_rng(61))
    taus = I.taus(steps, np.random.default_rng(62))
    th, ph, tht, pht = _angles(nq, 17)
    h0 = iqcc.Store(ctx, nq, 8 * len(c), INPLACE).load_numpy(x, z, c)
    runs = []
    for r in range(2):
        w = iqcc.Store(ctx, nq, 8 * len(c), INPLACE)
        describe(r, "copy + chain", nq=nq)
        iqcc.iqcc_store_copy(ctx.handle, h0.handle, w.handle)
        e = torch.zeros(steps, dtype=torch.float64, device="cuda")
        for j in range(steps):
            iqcc.iqcc_dress_inplace(ctx.handle, w.handle, cx[j], cz[j], taus[j], 1e-8, tht, pht,
                                    e[j - 1:j] if j else None, e[j:j + 1])
        gx, gz, gc = w.to_numpy()
        runs.append((gx, gz, gc.view(np.uint64), e.cpu().numpy().view(np.uint64)))
        w.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    h0.close()


def test_load_rows_independent_of_input_order(ctx):
    """A load writes each bucket's terms in ascending key order: the same terms
    in two input orders give identical rows, for packed stores (buckets of up
    to ~256 terms, and a few buckets of thousands when the bucket count is
    held down) and in-place stores (a few terms per bucket); and chains from
    two separately loaded stores agree bit for bit."""
    nq = 124
    x, z, c = I.hamiltonian_banded(nq, 2, band=6, decay=3.0)
    perm = np.random.default_rng(5).permutation(len(c))
    cases = [(0, len(c), {}), (0, len(c), {"load_bucket_terms": 4096}), (INPLACE, 64 * len(c), {})]
    for flags, max_terms, params in cases:
        describe(0, "load order", flags=flags, max_terms=max_terms, **params)
        rows = []
        with _Params(ctx, **params):
            for order in (slice(None), perm):
                s = iqcc.Store(ctx, nq, max_terms, flags).load_numpy(x[order], z[order], c[order])
                assert s.count() == len(c)
                gx, gz, gc = s.to_numpy()
                rows.append((gx, gz, gc.view(np.uint64)))
                s.close()
        for a, b in zip(*rows):
            assert np.array_equal(a, b)
        # the same multiset as the input
        key_in = np.concatenate([x, z, c.view(np.uint64)[:, None]], axis=1)
        key_out = np.concatenate([rows[0][0], rows[0][1], rows[0][2][:, None]], axis=1)
        assert np.array_equal(np.unique(key_in, axis=0), np.unique(key_out, axis=0))
    # chains from two loads (input in two orders) give the same energy bits
    steps = 6
    cx, cz = I.dis_candidates(x, nq, steps, 8, np.random.default_rng(63))
    taus = I.taus(steps, np.random.default_rng(64))
    th, ph, tht, pht = _angles(nq, 18)
    out = []
    for order in (slice(None), perm):
        describe(1, "chain after load", nq=nq, steps=steps)
        s = iqcc.Store(ctx, nq, 64 * len(c), INPLACE).load_numpy(x[order], z[order], c[order])
        e = torch.zeros(steps, dtype=torch.float64, device="cuda")
        for j in range(steps):
            iqcc.iqcc_dress_inplace(ctx.handle, s.handle, cx[j], cz[j], taus[j], 1e-8, tht, pht,
                                    e[j - 1:j] if j else None, e[j:j + 1])
        out.append(e.cpu().numpy().view(np.uint64))
        s.close()
    assert np.array_equal(out[0], out[1])


def test_store_copy_rebuckets(ctx):
    """Copies from an ordinary store into in-place stores with fewer, about
    as many and more buckets keep the terms, and the copy dresses like the
    original; a destination whose arena cannot hold the regions is reported
    invalid (IQCC_ERR_CAPACITY) instead of being written."""
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    px, pz = I.dis_candidates(x, nq, 1, 8, np.random.default_rng(71))
    src = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
    ref = O.dress(nq, x, z, c, px[0], pz[0], 0.12, 1e-8)
    for bucket_terms in (8192, 128, 4):          # fewer, similar, more buckets than src
        with _Params(ctx, inplace_bucket_terms=bucket_terms):
            dst = iqcc.Store(ctx, nq, 4 * len(c), INPLACE)
            describe(0, "store_copy", bucket_terms=bucket_terms)
            iqcc.iqcc_store_copy(ctx.handle, src.handle, dst.handle)
            assert_same_terms(dst.to_numpy(), (x, z, c), f"copy, {bucket_terms} terms per bucket")
            iqcc.iqcc_dress_inplace(ctx.handle, dst.handle, px[0], pz[0], 0.12, 1e-8)
            assert_same_terms(dst.to_numpy(), ref, f"dressed copy, {bucket_terms} terms per bucket")
            dst.close()
    small = iqcc.Store(ctx, nq, len(c) // 8, INPLACE)
    iqcc.iqcc_store_copy(ctx.handle, src.handle, small.handle)
    with pytest.raises(iqcc.IqccError) as e:
        small.count()
    assert e.value.code == iqcc.IQCC_ERR_CAPACITY
    small.close()
    src.close()


def test_inplace_argument_checks(ctx):
    nq = 8
    x, z, c = I.hamiltonian_dense(nq, 0)
    px, pz = I.single_qubit_pauli(nq, "XXXY")
    plain = iqcc.Store(ctx, nq, 4 * len(c)).load_numpy(x, z, c)
    with pytest.raises(iqcc.IqccError) as e:
        iqcc.iqcc_dress_inplace(ctx.handle, plain.handle, px, pz, 0.1, 0.0)
    assert e.value.code == iqcc.IQCC_ERR_INVALID_ARG
    ip = iqcc.Store(ctx, nq, 4 * len(c), INPLACE)
    iqcc.iqcc_dress(ctx.handle, plain.handle, px, pz, 0.1, 0.0, ip.handle)   # out-of-place output
    with pytest.raises(iqcc.IqccError) as e:
        iqcc.iqcc_dress_inplace(ctx.handle, ip.handle, px, pz, 0.1, 0.0)
    assert e.value.code == iqcc.IQCC_ERR_INVALID_ARG
    iqcc.iqcc_store_copy(ctx.handle, plain.handle, ip.handle)               # region layout again
    iqcc.iqcc_dress_inplace(ctx.handle, ip.handle, px, pz, 0.1, 0.0)
    ref = O.dress(nq, x, z, c, px, pz, 0.1, 0.0)
    assert_same_terms(ip.to_numpy(), ref, "after copy")
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_dress_inplace(ctx.handle, ip.handle, px, pz, float("nan"), 0.0)
    with pytest.raises(iqcc.IqccError):
        iqcc.iqcc_store_copy(ctx.handle, ip.handle, plain.handle)          # not an in-place store
    plain.close(); ip.close()


def test_autotuned_inplace_chain_bit_identical(ctx, tmp_path, monkeypatch):
    """The autotuner's pick for the in-place chain changes timing only: the
    final store holds the same (key, coefficient bits) multiset as under the
    default knobs.  The energies are sums whose order follows the work items,
    which the knobs resize, so they agree to rounding."""
    from paper_2603_08883_amd import autotune
    from tests.golden.multiset_hash import multiset_hash_torch
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "autotune.json"))
    nq, steps = 40, 5
    x, z, c = I.hamiltonian_dense(nq, 3)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(3, I.PURPOSE_ENTANGLERS))
    ents = list(zip(cx, cz))
    taus = I.taus(steps, I.rng_for(3, I.PURPOSE_TAUS))
    th, ph, tht, pht = _angles(nq, 13)
    defaults = {k: iqcc.iqcc_get_param(ctx.handle, k) for k in autotune.INPLACE_SPACE}
    h0 = iqcc.Store(ctx, nq, 8 * len(c), INPLACE).load_numpy(x, z, c)
    work = iqcc.Store(ctx, nq, 8 * len(c), INPLACE)

    def run():
        e = torch.zeros(steps, dtype=torch.float64, device="cuda")
        iqcc.iqcc_store_copy(ctx.handle, h0.handle, work.handle)
        for j, ((px, pz), t) in enumerate(zip(ents, taus)):
            iqcc.iqcc_dress_inplace(ctx.handle, work.handle, px, pz, t, 1e-8, tht, pht,
                                    e[j - 1:j] if j else None, e[j:j + 1])
        return (f"{multiset_hash_torch(*iqcc.iqcc_store_export(ctx.handle, work.handle)):016x}",
                e.cpu().numpy())

    describe(0, "in-place chain under default knobs", nq=nq)
    ref = run()
    try:
        describe(0, "in-place autotune", nq=nq)
        params, secs = autotune.tune_inplace(ctx, h0, work, ents, taus, 1e-8, tht, pht, 1, len(c),
                                             use_cache=False)
        assert secs > 0 and set(params) == set(autotune.INPLACE_SPACE)
        got = run()
        assert got[0] == ref[0]
        assert np.abs(got[1] - ref[1]).max() <= 1e-12 * np.abs(ref[1]).max()
    finally:
        autotune.apply(ctx, defaults)
    h0.close(); work.close()


def test_sum_squares_per_step(ctx):
    """iqcc_store_sum_squares equals the sum of the exported coefficients'
    squares, and across in-place steps at eps = 0 it stays at the H0 value to
    rounding (a dressing step keeps sum c^2, Eq. 5)."""
    nq, steps = 40, 4
    x, z, c = I.hamiltonian_dense(nq, 5)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(5, I.PURPOSE_ENTANGLERS))
    taus = I.taus(steps, I.rng_for(5, I.PURPOSE_TAUS))
    s = iqcc.Store(ctx, nq, 8 * len(c), INPLACE).load_numpy(x, z, c)
    ref0 = float(np.sum(c * c))
    describe(0, "sum of squares", nq=nq)
    got0 = float(iqcc.iqcc_store_sum_squares(ctx.handle, s.handle).item())
    assert abs(got0 - ref0) <= 1e-12 * ref0
    for j, ((px, pz), t) in enumerate(zip(zip(cx, cz), taus)):
        iqcc.iqcc_dress_inplace(ctx.handle, s.handle, px, pz, t, 0.0)
        got = float(iqcc.iqcc_store_sum_squares(ctx.handle, s.handle).item())
        ex = s.to_numpy()[2]
        assert abs(got - float(np.sum(ex * ex))) <= 1e-12 * ref0, j
        assert abs(got - ref0) <= 1e-11 * ref0, (j, got, ref0)
    s.close()
