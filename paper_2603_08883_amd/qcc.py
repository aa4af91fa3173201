"""The iQCC outer loop (Sec. II, iterative procedure) as a sequence of libiqcc
calls: each iteration screens the DIS candidates of the current Hamiltonian,
takes the largest gradients, applies each with its closed-form amplitude and
compresses (iqcc_qcc_iteration); the loop stops when an iteration lowers the
energy by less than `tol` or applies no generator.  All arithmetic runs in
libiqcc; this module only sequences calls."""
from __future__ import annotations

from . import iqcc


def run(ctx, h: "iqcc.Store", spare: "iqcc.Store", theta, phi, w_max: int = 4, n_select: int = 4,
        eps: float = 1e-8, max_iter: int = 10, tol: float = 1e-6):
    """Iterate in place on h (spare is the ping-pong partner); returns the per-iteration records."""
    history = []
    for _ in range(max_iter):
        rec = iqcc.iqcc_qcc_iteration(ctx.handle, h, spare, theta, phi, w_max, n_select, eps)
        history.append(rec)
        if len(rec["sel_tau"]) == 0 or abs(rec["energy"][-1] - rec["energy"][0]) < tol:
            break
    return history
