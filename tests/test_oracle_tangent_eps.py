"""Pins of the oracle's tau-gradient when compression removes terms (eps > 0).

The tau-derivative of the compressed chain is read as the derivative with
every step's drop decisions frozen at the forward pass (Eq. 6 chain with the
optional compression step of the iterative procedure; the paper is silent on
differentiating through it).  The oracle computes it in forward mode, dropping
a row's tangent together with the row.  Two independent checks:

* a 4-qubit chain in dense 2^n arithmetic where terms are dropped in the
  middle of the chain: the same frozen masks are applied to conjugated dense
  matrices and the derivative is taken by central differences;
* the 40-qubit workload at eps = 1e-8: central differences of the oracle's own
  chain energy, with h small enough that the kept key set of every step is the
  same at tau - h, tau and tau + h (asserted), so no coefficient crosses eps.
"""
import numpy as np

from oracle import dense as D
from paper_2603_08883_amd import inputs as I


def _dense_case():
    nq = 4
    rng = np.random.default_rng(2024)
    x, z, c = D.random_pauli_sum(nq, 14, rng)
    ents = []
    while len(ents) < 3:
        px = np.array([rng.integers(1, 1 << nq)], np.uint64)
        pz = np.array([rng.integers(0, 1 << nq)], np.uint64)
        ents.append((px, pz))
    taus = [0.35, -0.3, 0.45]
    th = rng.uniform(0.2, np.pi - 0.2, nq)
    ph = rng.uniform(0, 2 * np.pi, nq)
    return nq, x, z, c, ents, taus, th, ph


def _key_set(x, z):
    return {(int(a), int(b)) for a, b in zip(x[:, 0], z[:, 0])}


def test_frozen_mask_tangent_against_dense_masked_chain(oracle):
    nq, x, z, c, ents, taus, th, ph = _dense_case()
    eps = 0.12
    H = D.hamiltonian_matrix(nq, x, z, c)
    psi = D.qmf_state(th, ph)
    E, masks, kept = D.masked_chain_energy(nq, H, ents, taus, eps, psi)
    # the oracle's chain keeps the same keys at every step and has the same energy
    hx, hz, hc = x, z, c
    for j, ((px, pz), t) in enumerate(zip(ents, taus)):
        raw = oracle.dress_raw(nq, hx, hz, hc, px, pz, t)
        ux, uz, uc = oracle.merge_truncate(*raw, eps=0.0)
        hx, hz, hc = oracle.merge_truncate(ux, uz, uc, eps=eps)
        assert _key_set(hx, hz) == kept[j], j
        # margin: no coefficient within 1e-3 of eps, so finite differences with
        # h = 1e-6 cannot flip a decision
        assert np.all(np.abs(np.abs(uc) - eps) > 1e-3), j
        if j < len(ents) - 1:
            dropped = len(uc) - len(hc)
            assert dropped > 0, f"step {j} drops nothing: the case does not test a mid-chain drop"
    s = np.abs(c).sum()
    assert abs(oracle.qmf_energy(nq, hx, hz, hc, th, ph) - E) <= 1e-12 * s
    h = 1e-6
    for k in range(len(ents)):
        tp = list(taus); tp[k] += h
        tm = list(taus); tm[k] -= h
        Ep, _, _ = D.masked_chain_energy(nq, H, ents, tp, eps, psi, masks)
        Em, _, _ = D.masked_chain_energy(nq, H, ents, tm, eps, psi, masks)
        fd = (Ep - Em) / (2 * h)
        g, _ = oracle.chain_tau_gradient(nq, x, z, c, ents, taus, eps, th, ph, k)
        assert abs(g - fd) <= 1e-8 * s, (k, g, fd)
        # the drops matter: without compression the gradient is different
        g0, _ = oracle.chain_tau_gradient(nq, x, z, c, ents, taus, 0.0, th, ph, k)
        if k < len(ents) - 1:
            assert abs(g - g0) > 1e-4 * s, (k, g, g0)


def test_frozen_mask_tangent_matches_finite_differences_40q(oracle):
    nq, steps, eps = 40, 4, 1e-8
    x, z, c = I.hamiltonian_dense(nq, 1)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(1, I.PURPOSE_ENTANGLERS))
    taus = np.asarray(I.taus(steps, I.rng_for(1, I.PURPOSE_TAUS)), np.float64)
    th, ph = I.qmf_angles(nq, I.rng_for(1, I.PURPOSE_ANGLES))
    ents = list(zip(cx, cz))
    h = 2e-6

    def run(tv):
        keys = []
        hx, hz, hc = x, z, c
        for (px, pz), t in zip(ents, tv):
            hx, hz, hc = oracle.dress(nq, hx, hz, hc, px, pz, t, eps)
            keys.append((hx.tobytes(), hz.tobytes()))
        return oracle.qmf_energy(nq, hx, hz, hc, th, ph), keys

    _, keys0 = run(taus)
    for k in (0, steps - 2, steps - 1):
        tp = taus.copy(); tp[k] += h
        tm = taus.copy(); tm[k] -= h
        Ep, kp = run(tp)
        Em, km = run(tm)
        assert kp == keys0 and km == keys0, f"tau_{k}: a coefficient crosses eps within h"
        fd = (Ep - Em) / (2 * h)
        g, _ = oracle.chain_tau_gradient(nq, x, z, c, ents, list(taus), eps, th, ph, k)
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(g)), (k, g, fd)
