"""Differentiable QMF energy of an iteratively dressed Hamiltonian.

E(theta, phi, tau) = <Omega(theta, phi)| H^(K) |Omega(theta, phi)>,
H^(j) = compress(e^{i tau_j P_j/2} H^(j-1) e^{-i tau_j P_j/2})   (Sec. II, Eqs. 3-6).

Forward: the dressing chain runs on the GPU through iqcc_dress_taped, which
keeps every intermediate Hamiltonian and a tape of output rows in HBM, then
iqcc_qmf_energy evaluates the energy.  Backward: iqcc_qmf_energy_backward gives
dE/dtheta and dE/dphi and, in the same pass, the coefficient cotangent
lambda = dE/dc = <P_K>; iqcc_dress_backward carries it back through the
steps in reverse, producing dE/dtau_j.  Compression decisions of the forward
pass are held fixed (the derivative of the chain with frozen drop masks).
All arithmetic runs in libiqcc; this module only sequences calls.
"""
from __future__ import annotations

import numpy as np
import torch

from . import iqcc


class DressingChain:
    """HBM-resident dressing chain H0 -> H^(K) with per-step tapes."""

    def __init__(self, ctx: "iqcc.Context", n_qubits: int, x, z, c, entanglers, eps: float):
        self.ctx = ctx
        self.nq = n_qubits
        self.eps = float(eps)
        self.ents = [(np.asarray(px, np.uint64), np.asarray(pz, np.uint64)) for px, pz in entanglers]
        self.h0 = iqcc.Store(ctx, n_qubits, max(2 * len(c), 16)).load_numpy(x, z, c)
        self.h0_max = max(2 * len(c), 16)
        self.stores = [None] * len(self.ents)      # output store of step j
        self.caps = [0] * len(self.ents)
        self.tapes = [None] * len(self.ents)       # (tape_self, tape_partner) of step j
        self.version = 0                           # bumped by every run()

    def _input(self, j):
        return self.h0 if j == 0 else self.stores[j - 1]

    def run(self, taus):
        """Dress H0 through every step; returns the final store.

        The chain owns one set of device stores and tapes, so each run replaces
        the previous one; `version` identifies the current contents.
        """
        self.version += 1
        prev_cap = self.h0_max
        for j, ((px, pz), t) in enumerate(zip(self.ents, taus)):
            src = self._input(j)
            n_in = src.count()
            need = max(n_in, prev_cap)
            if self.stores[j] is None or self.caps[j] < need:
                if self.stores[j] is not None:
                    self.stores[j].close()
                self.stores[j] = iqcc.Store(self.ctx, self.nq, need)
                self.caps[j] = need
            rows = iqcc.iqcc_store_rows(src.handle)
            tp = self.tapes[j]
            if tp is None or tp[0].numel() < rows:
                tp = (torch.empty(rows, dtype=torch.int32, device="cuda"),
                      torch.empty(rows, dtype=torch.int32, device="cuda"))
                self.tapes[j] = tp
            iqcc.iqcc_dress_taped(self.ctx.handle, src.handle, px, pz, float(t), self.eps,
                                  self.stores[j].handle, tp[0], tp[1])
            prev_cap = self.caps[j]
        return self.stores[-1] if self.ents else self.h0

    def backward_taus(self, taus, lam_final):
        """Reverse sweep: returns dE/dtau (device tensor) given dE/dc of the final rows."""
        K = len(self.ents)
        dtau = torch.zeros(K, dtype=torch.float64, device="cuda")
        lam = lam_final
        for j in reversed(range(K)):
            src = self._input(j)
            lam_in = torch.empty(iqcc.iqcc_store_rows(src.handle), dtype=torch.float64, device="cuda")
            px, pz = self.ents[j]
            iqcc.iqcc_dress_backward(self.ctx.handle, src.handle, px, pz, float(taus[j]),
                                     self.tapes[j][0], self.tapes[j][1], lam, lam_in, dtau[j:j + 1],
                                     store_out=self.stores[j].handle)
            lam = lam_in
        return dtau

    def close(self):
        for s in self.stores:
            if s is not None:
                s.close()
        self.h0.close()


class QMFChainEnergy(torch.autograd.Function):
    """E(theta, phi, tau) for a DressingChain; differentiable in all three."""

    @staticmethod
    def forward(fctx, theta, phi, taus, chain: DressingChain):
        tau_list = [float(v) for v in taus.detach().cpu().tolist()]
        final = chain.run(tau_list)
        E = iqcc.iqcc_qmf_energy(chain.ctx.handle, final.handle, theta, phi)
        fctx.chain = chain
        fctx.version = chain.version
        fctx.tau_list = tau_list
        fctx.save_for_backward(theta, phi, taus)
        return E

    @staticmethod
    def backward(fctx, gE):
        theta, phi, taus = fctx.saved_tensors
        chain = fctx.chain
        if chain.version != fctx.version:
            # another forward ran on this chain since: recompute this one's tape
            final = chain.run(fctx.tau_list)
        else:
            final = chain.stores[-1] if chain.ents else chain.h0
        g = gE.detach().to(device="cuda", dtype=torch.float64).reshape(())
        lam = torch.empty(iqcc.iqcc_store_rows(final.handle), dtype=torch.float64, device="cuda")
        dth, dph = iqcc.iqcc_qmf_energy_backward(chain.ctx.handle, final.handle, theta, phi, g, lam)
        dtau = chain.backward_taus(fctx.tau_list, lam)
        return dth, dph, dtau.to(taus.device), None


def qmf_chain_energy(theta, phi, taus, chain: DressingChain):
    return QMFChainEnergy.apply(theta, phi, taus, chain)


def optimize(chain: DressingChain, theta, phi, taus, steps: int = 50, lr: float = 0.1,
             shrink: float = 0.5, c1: float = 1e-4, max_backtracks: int = 30, stats=None):
    """Gradient descent with Armijo backtracking on (theta, phi, tau) jointly
    (the joint optimisation of amplitudes and QMF parameters, App. A).

    Every trial point runs the taped forward once; an accepted trial is
    differentiated from that same forward.  Returns the list of accepted
    energies (non-increasing) and the final parameters; `stats`, if a dict,
    receives the number of forward and backward passes."""
    params = [theta.detach().clone(), phi.detach().clone(), taus.detach().clone()]
    energies = []
    n_fwd = n_bwd = 0

    def forward(p):
        nonlocal n_fwd
        n_fwd += 1
        q = [t.detach().clone().requires_grad_(True) for t in p]
        return qmf_chain_energy(q[0], q[1], q[2], chain), q

    def gradient(E_t, q):
        nonlocal n_bwd
        n_bwd += 1
        E_t.backward()
        return [t.grad.detach() for t in q]

    E_t, q = forward(params)
    E = float(E_t.item())
    grads = gradient(E_t, q)
    energies.append(E)
    for _ in range(steps):
        gnorm2 = sum(float((g * g).sum().item()) for g in grads)
        if gnorm2 == 0.0:
            break
        step = lr
        for _ in range(max_backtracks):
            trial = [p - step * g for p, g in zip(params, grads)]
            Et_t, qt = forward(trial)
            Et = float(Et_t.item())
            if Et <= E - c1 * step * gnorm2:
                break
            step *= shrink
        else:
            break
        params = trial
        E = Et
        grads = gradient(Et_t, qt)
        energies.append(E)
    if isinstance(stats, dict):
        stats.update({"forward_passes": n_fwd, "backward_passes": n_bwd})
    return energies, params
