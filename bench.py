#!/usr/bin/env python3
"""Benchmark of the iQCC hot path on one MI355X.

Timed step: one full 20-step dressing chain of a 124-qubit Hamiltonian
(dress + merge + compression |c| < 1e-8 + fused QMF energy after every step,
carried forward from the previous step's energy),
replayed from the HBM-resident initial Hamiltonian.  Value: dressed+merged
output terms per second over the chain.  Also measured: the dominant kernel
against the HBM roofline (HIP events on the library's stream), batched versus
plain DIS screening of 1e4 candidates against a 1e7-term 100-qubit
Hamiltonian, and the FP64 CPU oracle on a bounded sample of the same chain.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "dressed+merged Pauli terms/s & HBM GB/s @124q; DIS grads/s batched vs plain"
HBM_PEAK_GBPS = 8000.0
# VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
N_QUBITS = 124
N_STEPS_CHAIN = 20
EPS = 1e-8
CONFIG = 2          # seed family of the 124-qubit workload
DIS_CONFIG = 3      # seed family of the DIS workload
BATCH_CONFIG = 4    # seed family of the 64-Hamiltonian batch


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload_chain():
    from paper_2603_08883_amd import inputs as I
    x, z, c = I.hamiltonian_banded(N_QUBITS, CONFIG, band=6, decay=3.0)
    cx, cz = I.dis_candidates(x, N_QUBITS, N_STEPS_CHAIN, 8, I.rng_for(CONFIG, I.PURPOSE_ENTANGLERS))
    taus = I.taus(N_STEPS_CHAIN, I.rng_for(CONFIG, I.PURPOSE_TAUS))
    th, ph = I.qmf_angles(N_QUBITS, I.rng_for(CONFIG, I.PURPOSE_ANGLES))
    return x, z, c, list(zip(cx, cz)), taus, th, ph


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, z, c, ents, taus, th, ph, budget_s=20.0, single_budget_s=8.0):
    """The oracle as it stands on the host: its bucket-parallel form on every
    core this process may use (the same terms and energies as the serial
    oracle), over the chain's steps in order until about budget_s is spent,
    and the serial oracle on one core over the first steps."""
    from oracle import oracle as O
    O.lib()
    cores = len(os.sched_getaffinity(0))

    def run(step_fn, energy_fn, budget):
        hx, hz, hc = x, z, c
        t0 = time.perf_counter()
        n_out = steps = 0
        largest = 0
        for (px, pz), t in zip(ents, taus):
            largest = max(largest, len(hc))
            hx, hz, hc = step_fn(hx, hz, hc, px, pz, t)
            energy_fn(hx, hz, hc)
            n_out += len(hc)
            steps += 1
            if time.perf_counter() - t0 > budget:
                break
        return n_out, steps, time.perf_counter() - t0, largest, len(hc)

    n_out, steps, dt, largest, final = run(
        lambda a, b, cc, px, pz, t: O.dress_par(N_QUBITS, a, b, cc, px, pz, t, EPS, cores),
        lambda a, b, cc: O.qmf_energy_par(N_QUBITS, a, b, cc, th, ph, cores), budget_s)
    s_out, s_steps, s_dt, _, s_final = run(
        lambda a, b, cc, px, pz, t: O.dress(N_QUBITS, a, b, cc, px, pz, t, EPS),
        lambda a, b, cc: O.qmf_energy(N_QUBITS, a, b, cc, th, ph), single_budget_s)
    return {"value": n_out / dt, "unit": "dressed+merged terms/s", "cores": cores, "kind": "oracle",
            "sample": f"first {steps} of {N_STEPS_CHAIN} dressing steps (+energy) of the 124-qubit chain "
                      f"on {cores} threads (bucket-parallel oracle: same terms and energies as the serial "
                      f"one), {len(c)} -> {final} terms, largest step input {largest} terms, {dt:.1f} s",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(),
            "single_thread": {"value": s_out / s_dt, "unit": "dressed+merged terms/s", "cores": 1,
                              "sample": f"first {s_steps} steps, {len(c)} -> {s_final} terms, "
                                        f"{s_dt:.1f} s"}}


def profiled_traffic(ctx):
    """HBM bytes per k_dress_inplace launch from the committed hardware-counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a kernel of known traffic), or None
    when the kernel source or the launch knobs differ from the profiled ones."""
    import hashlib
    from paper_2603_08883_amd import iqcc
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "k_dress_inplace_124q_chain_pmc.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ("kernels_inplace.hip", "iqcc_internal.h"):
        with open(os.path.join(here, "paper_2603_08883_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    knobs = " ".join(f"{k}={iqcc.iqcc_get_param(ctx.handle, k)}"
                     for k in ("inplace_bucket_terms", "inplace_item_terms", "inplace_cap",
                               "inplace_region_rows"))
    if fields.get("kernel_source_sha256") != h.hexdigest() or fields.get("knobs") != knobs:
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def dis_ops_per_pair():
    """VALU lane-operations per (term, candidate) pair of k_dis_batched from the
    committed counter summary (SQ_INSTS_VALU * 64 / pairs), or None when the
    kernel source differs from the profiled one."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "k_dis_batched_100q_pmc.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    with open(os.path.join(here, "paper_2603_08883_amd", "csrc", "kernels_dis.hip"), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(fields["valu_lane_ops_per_pair"])
    except (KeyError, ValueError):
        return None


def measured_copy_gbps():
    """Bandwidth of a plain device-to-device copy of 4 GiB (bytes read + bytes
    written per second): the practical HBM ceiling next to the 8 TB/s peak."""
    import torch
    src = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 5
    nbytes = 2 * src.numel() * 8
    del src, dst
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


def extended_chain_leg(ctx, stream, wl, steps=4, max_terms=4.0e8):
    """The chain carried past its 20 steps, to the 12-GB-class footprint of the
    largest workloads: H0 loaded into an in-place store sized for 4e8 terms
    (2^21 buckets), the 20 steps of the chain (untimed), then `steps` more
    seeded DIS entanglers timed with HIP events; per step sizes, time and
    algorithmic bandwidth, energy carried.  Run last: its 58 GB store is
    allocated after every other leg."""
    import torch
    from paper_2603_08883_amd import inputs as I
    from paper_2603_08883_amd import iqcc
    x, z, c, ents, taus, th, ph = wl
    cx, cz = I.dis_candidates(x, N_QUBITS, steps, 8, I.rng_for(CONFIG + 50, I.PURPOSE_ENTANGLERS))
    taus2 = I.taus(steps, I.rng_for(CONFIG + 50, I.PURPOSE_TAUS))
    tht = torch.from_numpy(th).cuda()
    pht = torch.from_numpy(ph).cuda()
    big = iqcc.Store(ctx, N_QUBITS, int(max_terms), iqcc.IQCC_STORE_INPLACE)
    K = len(ents)
    e = torch.zeros(K + steps, dtype=torch.float64, device="cuda")

    def chain20():
        big.load_numpy(x, z, c)
        for j, ((px, pz), t) in enumerate(zip(ents, taus)):
            iqcc.iqcc_dress_inplace(ctx.handle, big.handle, px, pz, t, EPS, tht, pht,
                                    e[j - 1:j] if j else None, e[j:j + 1])

    def step(j):
        k = K + j
        iqcc.iqcc_dress_inplace(ctx.handle, big.handle, cx[j], cz[j], taus2[j], EPS, tht, pht,
                                e[k - 1:k], e[k:k + 1])

    sizes = []   # untimed pass: sizes of every extra step
    chain20()
    n_in = big.count()
    for j in range(steps):
        step(j)
        n_out = big.count()
        n_anti, n_new = iqcc.iqcc_store_stats(ctx.handle, big.handle)
        sizes.append((n_in, n_anti, n_new, n_out))
        n_in = n_out
    chain20()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    for j in range(steps):
        evs[j].record(stream)
        step(j)
    evs[steps].record(stream)
    torch.cuda.synchronize()
    ms = [evs[j].elapsed_time(evs[j + 1]) for j in range(steps)]
    bt = 16 * x.shape[1] + 8
    alg = [bt * s_[0] + 8 * s_[1] + bt * s_[2] for s_ in sizes]
    st = iqcc.iqcc_store_inplace_stats(ctx.handle, big.handle)
    out = {"workload": f"the 124-qubit chain continued by {steps} more seeded DIS entanglers past its "
                       f"20 steps, in an in-place store for {max_terms:.1e} terms",
           "arena_gb": iqcc.iqcc_store_bytes(N_QUBITS, int(max_terms), iqcc.IQCC_STORE_INPLACE) / 1e9,
           "final_terms": sizes[-1][3], "final_term_bytes_gb": sizes[-1][3] * bt / 1e9,
           "steps_ms": sum(ms), "alg_gbps": sum(alg) / (sum(ms) * 1e-3) / 1e9,
           "roofline_frac": sum(alg) / (sum(ms) * 1e-3) / 1e9 / HBM_PEAK_GBPS,
           "relocated_items_last_step": st["relocated"],
           "per_step": [{"n_in": s_[0], "n_anti": s_[1], "n_new": s_[2], "n_out": s_[3],
                         "energy": float(e[K + j].item()), "ms": round(ms[j], 4),
                         "alg_gbps": alg[j] / (ms[j] * 1e-3) / 1e9} for j, s_ in enumerate(sizes)]}
    big.close()
    torch.cuda.empty_cache()
    log(f"extended chain: {sizes[0][0]} -> {sizes[-1][3]} terms in {sum(ms):.2f} ms, "
        f"{out['alg_gbps']:.0f} GB/s algorithmic")
    return out


def angle_backward_leg(ctx, stream, final, tht, pht, bt, reps=5):
    """dE/dtheta, dE/dphi and the per-term cotangents of the final 124-qubit
    Hamiltonian (in-place store) in one call, timed with HIP events on the
    library's stream; checks that two calls give the same bits."""
    import torch
    from paper_2603_08883_amd import iqcc
    n = final.count()
    lam = torch.empty(iqcc.iqcc_store_rows(final.handle), dtype=torch.float64, device="cuda")
    d1 = iqcc.iqcc_qmf_energy_backward(ctx.handle, final.handle, tht, pht, None, lam)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        d2 = iqcc.iqcc_qmf_energy_backward(ctx.handle, final.handle, tht, pht, None, lam)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    same = bool(torch.equal(d1[0], d2[0]) and torch.equal(d1[1], d2[1]))
    del lam
    torch.cuda.empty_cache()
    nbytes = (bt + 8) * n   # read each term, write its cotangent
    log(f"angle backward {ms:.3f} ms over {n} terms")
    return {"workload": f"final 124-qubit Hamiltonian ({n} terms, in-place store): dE/dtheta, "
                        "dE/dphi and the per-term cotangents in one call",
            "ms": ms, "alg_bytes": int(nbytes),
            "hbm_gbps_algorithmic": nbytes / (ms * 1e-3) / 1e9,
            "roofline_frac_hbm": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "bit_identical_calls": same,
            "bound": "VALU and LDS: 44 group lookups, prefix/suffix products and an exact "
                     "fixed-point add per 3-qubit group of every term"}


def autograd_leg(ctx, stream, wl):
    """dE/d(theta, phi, tau) of the full 124-qubit chain through the autograd
    Function (taped forward + reverse sweep), against the same gradient from
    plain per-call central differences (h = 1e-6): two untaped chains per tau,
    two energy calls per angle."""
    import torch
    from paper_2603_08883_amd import iqcc
    from paper_2603_08883_amd.autograd import DressingChain, qmf_chain_energy
    x, z, c, ents, taus, th, ph = wl
    K = len(ents)
    chain = DressingChain(ctx, N_QUBITS, x, z, c, ents, EPS)

    def fwd_bwd():
        q = [torch.tensor(th, device="cuda", requires_grad=True),
             torch.tensor(ph, device="cuda", requires_grad=True),
             torch.tensor(taus, device="cuda", requires_grad=True)]
        E = qmf_chain_energy(q[0], q[1], q[2], chain)
        E.backward()
        return float(E.item()), [v.grad for v in q]

    fwd_bwd()
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        E, grads = fwd_bwd()
    torch.cuda.synchronize()
    t_ad = (time.perf_counter() - t0) / reps
    tape_rows = sum(iqcc.iqcc_store_rows(s.handle) for s in chain.stores)
    n_final = chain.stores[-1].count()
    chain.close()
    torch.cuda.empty_cache()
    log(f"autograd fwd+bwd {t_ad*1e3:.1f} ms")

    # plain per-call form: central differences, untaped ping-pong chains
    h = 1e-6
    h0 = iqcc.Store(ctx, N_QUBITS, 2 * len(c)).load_numpy(x, z, c)
    s1 = iqcc.Store(ctx, N_QUBITS, 2 * n_final)
    s2 = iqcc.Store(ctx, N_QUBITS, 2 * n_final)
    tht = torch.from_numpy(th).cuda()
    pht = torch.from_numpy(ph).cuda()
    e = torch.zeros(2, dtype=torch.float64, device="cuda")

    def energy_of(tau_vec, slot):
        src = h0
        for j, ((px, pz), t) in enumerate(zip(ents, tau_vec)):
            dst = (s1, s2)[j % 2]
            iqcc.iqcc_dress(ctx.handle, src.handle, px, pz, float(t), EPS, dst.handle)
            src = dst
        iqcc.iqcc_qmf_energy(ctx.handle, src.handle, tht, pht, e[slot:slot + 1])
        return src

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_tau = np.zeros(K)
    for k in range(K):
        tp = np.array(taus, dtype=np.float64); tp[k] += h
        tm = np.array(taus, dtype=np.float64); tm[k] -= h
        energy_of(tp, 0)
        energy_of(tm, 1)
        g_tau[k] = float((e[0] - e[1]).item()) / (2 * h)
    final = energy_of(np.asarray(taus, np.float64), 0)
    g_ang = [np.zeros(N_QUBITS), np.zeros(N_QUBITS)]
    ev = torch.zeros(2 * 2 * N_QUBITS, dtype=torch.float64, device="cuda")
    for which in (0, 1):
        for j in range(N_QUBITS):
            for sgn, slot in ((1.0, 0), (-1.0, 1)):
                a = tht.clone(); b = pht.clone()
                (a if which == 0 else b)[j] += sgn * h
                k = (which * N_QUBITS + j) * 2 + slot
                iqcc.iqcc_qmf_energy(ctx.handle, final.handle, a, b, ev[k:k + 1])
    evn = ev.cpu().numpy().reshape(2, N_QUBITS, 2)
    for which in (0, 1):
        g_ang[which] = (evn[which, :, 0] - evn[which, :, 1]) / (2 * h)
    torch.cuda.synchronize()
    t_fd = time.perf_counter() - t0
    # the angle backward alone on the final Hamiltonian, as the autograd backward
    # calls it (dE/dtheta, dE/dphi and the per-row cotangents)
    n_fin = final.count()
    lam = torch.empty(iqcc.iqcc_store_rows(final.handle), dtype=torch.float64, device="cuda")
    iqcc.iqcc_qmf_energy_backward(ctx.handle, final.handle, tht, pht, None, lam)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        iqcc.iqcc_qmf_energy_backward(ctx.handle, final.handle, tht, pht, None, lam)
    ev1.record()
    torch.cuda.synchronize()
    bwd_ms = ev0.elapsed_time(ev1) / 5
    bwd_bytes = (16 * x.shape[1] + 8 + 8) * n_fin   # read each term, write its cotangent
    del lam
    h0.close(); s1.close(); s2.close()
    ad_tau = grads[2].cpu().numpy()
    ad_th = grads[0].cpu().numpy(); ad_ph = grads[1].cpu().numpy()
    ang_err = max(np.abs(ad_th - g_ang[0]).max(), np.abs(ad_ph - g_ang[1]).max())
    tau_rel = np.abs(ad_tau - g_tau) / np.maximum(1.0, np.abs(g_tau))
    log(f"plain central differences {t_fd*1e3:.1f} ms; angle max|diff| {ang_err:.2e}, "
        f"tau max rel diff {tau_rel.max():.2e}")
    return {
        "workload": "124-qubit 20-step chain as timed above; gradient w.r.t. 248 Bloch angles "
                    "and 20 tau (compression masks of the forward held fixed)",
        "energy": E, "fwd_bwd_ms": t_ad * 1e3, "taped_rows": int(tape_rows),
        "plain_central_diff_ms": t_fd * 1e3, "speedup_autograd_vs_plain": t_fd / t_ad,
        "plain_calls": 2 * K * (K + 1) + 4 * N_QUBITS,
        "angle_grad_max_abs_diff_vs_fd": float(ang_err),
        "tau_grad_max_rel_diff_vs_fd": float(tau_rel.max()),
        "tau_grad_median_rel_diff_vs_fd": float(np.median(tau_rel)),
        "angle_backward": {
            "workload": f"final 124-qubit Hamiltonian ({n_fin} terms): dE/dtheta, dE/dphi and "
                        "the per-term cotangents in one call",
            "ms": bwd_ms, "alg_bytes": int(bwd_bytes),
            "hbm_gbps_algorithmic": bwd_bytes / (bwd_ms * 1e-3) / 1e9,
            "roofline_frac_hbm": bwd_bytes / (bwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "bound": "valu (counters: VALU issue about 70% of SIMD time)"},
    }


def c5_leg(ctx, wl, steps=50, lr=0.1):
    """Joint gradient-based optimisation of the 248 Bloch angles and 20 tau of
    the 124-qubit chain (App. A iterative procedure): gradient descent with
    Armijo backtracking, each trial a full taped forward, each accepted point
    differentiated by the reverse sweep."""
    import torch
    from paper_2603_08883_amd.autograd import DressingChain, optimize
    x, z, c, ents, taus, th, ph = wl
    chain = DressingChain(ctx, N_QUBITS, x, z, c, ents, EPS)
    stats = {}
    torch.cuda.empty_cache()
    chain.run(list(taus))   # untimed: the chain allocates its stores and tapes
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies, params = optimize(chain, torch.from_numpy(th).cuda(), torch.from_numpy(ph).cuda(),
                                torch.tensor(taus, dtype=torch.float64, device="cuda"),
                                steps=steps, lr=lr, stats=stats)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_final = chain.stores[-1].count()
    chain.close()
    torch.cuda.empty_cache()
    taken = len(energies) - 1
    log(f"C5 optimisation: {taken} steps, E {energies[0]:.10f} -> {energies[-1]:.10f}, "
        f"{dt / max(taken, 1) * 1e3:.1f} ms/step")
    return {"workload": "124-qubit 20-step chain (eps 1e-8): gradient descent with Armijo "
                        "backtracking on (theta, phi, tau) jointly, lr 0.1",
            "steps_requested": steps, "steps_taken": taken,
            "energy_first": energies[0], "energy_last": energies[-1],
            "energies": energies,
            "non_increasing": all(b <= a for a, b in zip(energies, energies[1:])),
            "seconds": dt, "ms_per_step": dt / max(taken, 1) * 1e3,
            "final_terms": int(n_final), **stats}


def sortless_leg(ctx, wl, fused_chain_ms, fused_final_terms):
    """The same 124-qubit chain through the sortless-dressing path (flat, globally
    sorted Hamiltonian; partition by flipped bits, per-partition merges, multiway
    merge), against the fused bucket-pair kernel timed above (energy excluded)."""
    import torch
    from paper_2603_08883_amd import iqcc
    x, z, c, ents, taus, th, ph = wl
    W = x.shape[1]
    order = np.lexsort([z[:, w] for w in range(W)] + [x[:, w] for w in range(W)])
    dx = iqcc.to_device_words(x[order]); dz = iqcc.to_device_words(z[order])
    dc = torch.from_numpy(np.ascontiguousarray(c[order])).cuda()

    def chain():
        hx, hz, hc = dx, dz, dc
        for (px, pz), t in zip(ents, taus):
            hx, hz, hc = iqcc.iqcc_sortless_dress(ctx.handle, N_QUBITS, hx, hz, hc, px, pz, t, EPS)
        return hc.numel()

    n_final = chain()          # also warms the allocator
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chain()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": "the 124-qubit 20-step chain, dressing + merge + compression only",
            "chain_ms": dt * 1e3, "final_terms": int(n_final),
            "same_final_count_as_fused": int(n_final) == int(fused_final_terms),
            "fused_chain_ms_with_energy": fused_chain_ms,
            "fused_over_sortless_speedup": dt * 1e3 / fused_chain_ms}


def poly_leg(ctx, n_gen=4, budget_s=10.0):
    """Exact energy polynomial of the 4 largest-gradient DIS generators of the
    40-qubit Hamiltonian (3^4 grid chains sharing prefixes, no compression) and
    its coordinate-descent minimum, against the oracle on a bounded number of
    grid chains."""
    import torch
    from paper_2603_08883_amd import inputs as I
    from paper_2603_08883_amd import iqcc
    from oracle import oracle as O
    from oracle import qcc as Q
    nq = 40
    x, z, c = I.hamiltonian_dense(nq, 1)
    th, ph = I.qmf_angles(nq, I.rng_for(1, I.PURPOSE_ANGLES))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)
    cx, cz = Q.dis_generators(Q.flip_sets(x, 2))
    g = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, iqcc.to_device_words(cx),
                                iqcc.to_device_words(cz)).cpu().numpy()
    pick = np.argsort(-np.abs(g), kind="stable")[:n_gen]
    pxs, pzs = cx[pick], cz[pick]
    work = [iqcc.Store(ctx, nq, 2 * len(c) * 2 ** (k + 1)) for k in range(n_gen)]
    iqcc.iqcc_energy_trig_poly(ctx.handle, h.handle, pxs, pzs, tht, pht, work)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    coef = iqcc.iqcc_energy_trig_poly(ctx.handle, h.handle, pxs, pzs, tht, pht, work)
    tau, e = iqcc.iqcc_trig_poly_minimize(coef, np.zeros(n_gen), sweeps=200)
    dt = time.perf_counter() - t0
    # oracle: full chains for a few grid points
    k, t1 = 0, time.perf_counter()
    while time.perf_counter() - t1 < budget_s and k < 3 ** n_gen:
        hx, hz, hc = x, z, c
        for j in range(n_gen):
            hx, hz, hc = O.dress(nq, hx, hz, hc, pxs[j], pzs[j], Q.GRID[(k // 3 ** j) % 3], 0.0)
        O.qmf_energy(nq, hx, hz, hc, th, ph)
        k += 1
    odt = time.perf_counter() - t1
    h.close()
    for w in work:
        w.close()
    return {"workload": f"40-qubit dense JW Hamiltonian ({len(c)} terms), {n_gen} largest-gradient DIS "
                        f"generators, {3 ** n_gen} grid chains without compression",
            "ms": dt * 1e3, "energy_at_zero": float(iqcc.iqcc_trig_poly_eval(coef, np.zeros(n_gen))),
            "minimum": e, "taus": [float(v) for v in tau],
            "cpu_oracle": {"kind": "oracle", "cores": 1, "sample": f"{k} of {3 ** n_gen} grid chains, {odt:.1f} s",
                           "ms_extrapolated": odt / max(k, 1) * 3 ** n_gen * 1e3}}


def qcc_leg(ctx, budget_s=10.0):
    """One iQCC iteration (screen all DIS candidates of the flip sets with
    |F| <= 4, take the 4 largest gradients, closed-form amplitude and dressing
    for each) on the 40-qubit Hamiltonian, against the oracle's screening rate
    on a bounded candidate sample."""
    import torch
    from paper_2603_08883_amd import inputs as I
    from paper_2603_08883_amd import iqcc
    nq, w_max, n_sel = 40, 4, 4
    x, z, c = I.hamiltonian_dense(nq, 1)
    th, ph = I.qmf_angles(nq, I.rng_for(1, I.PURPOSE_ANGLES))
    tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
    h = iqcc.Store(ctx, nq, 64 * len(c)).load_numpy(x, z, c)
    spare = iqcc.Store(ctx, nq, 64 * len(c))
    h0 = iqcc.Store(ctx, nq, 2 * len(c)).load_numpy(x, z, c)

    def one():
        # restart from H0 so every timed iteration does the same work
        iqcc.iqcc_dress(ctx.handle, h0.handle, np.zeros(1, np.uint64), np.zeros(1, np.uint64), 0.0, 0.0,
                        h.handle)
        return iqcc.iqcc_qcc_iteration(ctx.handle, h, spare, tht, pht, w_max, n_sel, 1e-8)

    one()
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        rec = one()
    torch.cuda.synchronize()
    t_gpu = (time.perf_counter() - t0) / reps
    nc = rec["n_candidates"]
    out = {"workload": f"40-qubit dense JW Hamiltonian ({len(c)} terms), DIS candidates of every flip set "
                       f"with |F| <= {w_max} ({nc}), {n_sel} generators with closed-form amplitudes, "
                       "eps=1e-8",
           "iteration_ms": t_gpu * 1e3, "n_candidates": nc,
           "screening_pairs_per_s": nc * len(c) / t_gpu,
           "energy_before": float(rec["energy"][0]), "energy_after": float(rec["energy"][-1]),
           "taus": [float(v) for v in rec["sel_tau"]]}
    # the oracle's screening on a bounded sample of the same candidates
    from oracle import oracle as O
    from oracle import qcc as Q
    cx, cz = Q.dis_generators(Q.flip_sets(x, w_max))
    k = 16
    t0 = time.perf_counter()
    while True:
        O.dis_gradients(nq, x, z, c, th, ph, cx[:k], cz[:k])
        dt = time.perf_counter() - t0
        if dt > budget_s / 4 or k >= len(cx):
            break
        k = min(len(cx), k * 2)
        t0 = time.perf_counter()
    out["cpu_oracle"] = {"kind": "oracle", "cores": 1, "pairs_per_s": k * len(c) / dt,
                         "sample": f"DIS gradients of the first {k} of {len(cx)} candidates, {dt:.1f} s",
                         "iteration_s_extrapolated": len(cx) * dt / k}
    h.close(); spare.close(); h0.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dis", action="store_true")
    ap.add_argument("--no-chain", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-autograd", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the 50-step joint optimisation")
    ap.add_argument("--no-extended", action="store_true",
                    help="skip the chain continued to ~3e8 terms (12-GB-class footprint)")
    ap.add_argument("--no-qcc", action="store_true")
    ap.add_argument("--no-sortless", action="store_true")
    ap.add_argument("--no-poly", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip the autotuner (batch and DIS knobs; in-place chain knobs reported)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 1 GiB device copy first (scale for profiler byte counters)")
    ap.add_argument("--dis-plain-sample", type=int, default=1024)
    ap.add_argument("--only", choices=("chain", "angle-backward", "dis", "batch"),
                    help="run one leg alone (for profiling): the timed in-place chain; the "
                         "angle backward on the chain's final Hamiltonian; DIS; the batch")
    ap.add_argument("--max-terms", type=float, default=1.3e8,
                    help="max_terms of the in-place stores of the 124-qubit chain")
    args = ap.parse_args()
    if args.only is not None:
        for leg in ("cpu_baseline", "dis", "chain", "batch", "autograd", "c5", "qcc", "sortless",
                    "poly", "extended"):
            setattr(args, "no_" + leg, True)
        if args.only in ("chain", "angle-backward"):
            args.no_chain = False
        else:
            setattr(args, "no_" + args.only, False)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not a built path)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_08883_amd import inputs as I
    from paper_2603_08883_amd import iqcc

    torch.cuda.init()
    dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream()
    ctx = iqcc.Context(dev)
    result = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
              "data": "synthetic"}

    if args.calib_copy:
        # known traffic for the profiler's byte counters: a fill kernel writes
        # 1 GiB, then an elementwise kernel reads 1 GiB and writes 1 GiB
        src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        torch.neg(src_t, out=dst_t)
        torch.cuda.synchronize()
        result["calib_copy_bytes"] = 2 * src_t.numel() * 8
        del src_t, dst_t

    copy_gbps = measured_copy_gbps()
    log(f"device copy {copy_gbps:.0f} GB/s (read + write)")

    wl = None
    if not (args.no_chain and args.no_autograd and args.no_extended):
        t = time.perf_counter()
        wl = workload_chain()
        log(f"124-qubit workload: {len(wl[2])} terms generated in {time.perf_counter() - t:.1f}s")

    if not args.no_chain:
        x, z, c, ents, taus, th, ph = wl
        W = x.shape[1]
        bt = 16 * W + 8
        INPLACE = iqcc.IQCC_STORE_INPLACE
        max_ip = int(args.max_terms)
        # resident H0 and the working store, both laid out in bucket regions
        h0 = iqcc.Store(ctx, N_QUBITS, max_ip, INPLACE).load_numpy(x, z, c)
        work = iqcc.Store(ctx, N_QUBITS, max_ip, INPLACE)
        tht = torch.from_numpy(th).cuda()
        pht = torch.from_numpy(ph).cuda()
        energies = torch.zeros(N_STEPS_CHAIN, dtype=torch.float64, device="cuda")

        def chain(events=None, carry=True):
            """Copy H0 into the working store, then 20 in-place dressing steps;
            the energy of step 0 is summed in full, later steps carry it
            forward (carry=False: every step sums in full)."""
            if events is not None:
                events[0].record(stream)
            iqcc.iqcc_store_copy(ctx.handle, h0.handle, work.handle)
            for j, ((px, pz), tau) in enumerate(zip(ents, taus)):
                if events is not None:
                    events[j + 1].record(stream)
                iqcc.iqcc_dress_inplace(ctx.handle, work.handle, px, pz, tau, EPS, tht, pht,
                                        energies[j - 1:j] if (carry and j > 0) else None,
                                        energies[j:j + 1])
            if events is not None:
                events[-1].record(stream)
            return work

        # untimed pass that records the per-step sizes (the same on every replay)
        sizes, relocated, sum_c2 = [], 0, []
        iqcc.iqcc_store_copy(ctx.handle, h0.handle, work.handle)
        sum_c2_h0 = float(iqcc.iqcc_store_sum_squares(ctx.handle, work.handle).item())
        n_in = len(c)
        for j, ((px, pz), tau) in enumerate(zip(ents, taus)):
            iqcc.iqcc_dress_inplace(ctx.handle, work.handle, px, pz, tau, EPS, tht, pht, None,
                                    energies[j:j + 1])
            n_out = work.count()
            n_anti, n_new = iqcc.iqcc_store_stats(ctx.handle, work.handle)
            relocated += iqcc.iqcc_store_inplace_stats(ctx.handle, work.handle)["relocated"]
            sizes.append((n_in, n_anti, n_new, n_out))
            sum_c2.append(float(iqcc.iqcc_store_sum_squares(ctx.handle, work.handle).item()))
            n_in = n_out
        ip_stats = iqcc.iqcc_store_inplace_stats(ctx.handle, work.handle)
        log("step sizes (N_in, N_anti, N_new, N_out):", sizes[0], "...", sizes[-1],
            f"relocated items {relocated}")
        e_full = energies.clone()
        if args.only == "angle-backward":
            result["angle_backward"] = angle_backward_leg(ctx, stream, work, tht, pht, bt)
            print(json.dumps(result), flush=True)
            return
        for _ in range(max(0, args.warmup)):
            chain()
        torch.cuda.synchronize()
        per_step = np.zeros(N_STEPS_CHAIN)
        copy_s = 0.0
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(N_STEPS_CHAIN + 2)]
               for _ in range(args.steps)]
        finals = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            chain(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for k in range(args.steps):
            copy_s += evs[k][0].elapsed_time(evs[k][1]) * 1e-3
            for j in range(N_STEPS_CHAIN):
                per_step[j] += evs[k][j + 1].elapsed_time(evs[k][j + 2]) * 1e-3
        per_step /= args.steps
        copy_s /= args.steps
        chain_s = wall / args.steps
        e_carry = energies.clone()
        carry_err = float((e_carry - e_full).abs().max().item())
        # bit-identical replays: the final store and energies of two more chains
        digests = []
        for _ in range(2):
            chain()
            ex, ez, ec = iqcc.iqcc_store_export(ctx.handle, work.handle)
            digests.append((ex.cpu().numpy().tobytes(), ez.cpu().numpy().tobytes(),
                            ec.cpu().numpy().tobytes(), energies.cpu().numpy().tobytes()))
            del ex, ez, ec
        identical = digests[0] == digests[1] and digests[0][3] == e_carry.cpu().numpy().tobytes()
        del digests
        torch.cuda.empty_cache()
        # the same chain with the energy summed in full after every step
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            chain(carry=False)
        torch.cuda.synchronize()
        full_s = (time.perf_counter() - t0) / args.steps
        total_out = sum(s_[3] for s_ in sizes)
        total_in = sum(s_[0] for s_ in sizes)
        alg = [bt * s_[0] + 8 * s_[1] + bt * s_[2] for s_ in sizes]
        alg_bytes = sum(alg)
        stream_bytes = sum(bt * (s_[0] + s_[3]) for s_ in sizes)
        kernel_s = per_step.sum()
        achieved = alg_bytes / kernel_s / 1e9
        traffic = profiled_traffic(ctx)
        result.update({
            "value": total_out / chain_s,
            "unit": "dressed+merged terms/s",
            "ms_per_step": chain_s * 1e3,
            "config": {
                "workload": "124-qubit banded JW Hamiltonian (62 orbitals, band 6, decay 3), "
                            f"{len(c)} initial terms, 20 seeded DIS entanglers (weight 2-8), "
                            "tau~U(-0.2,0.2), |c|<1e-8 dropped after each step, QMF energy "
                            "fused after each step; one step = the whole 20-entangler chain "
                            "(copy of the resident H0 + 20 in-place dressings)",
                "n_qubits": N_QUBITS, "initial_terms": len(c), "final_terms": sizes[-1][3],
                "terms_processed": total_in, "terms_produced": total_out,
                "parallelism": "1 GPU"},
            "hbm_gbps_algorithmic": achieved,
            "hbm_gbps_stream_model": stream_bytes / kernel_s / 1e9,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS,
                         "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                         "traffic": traffic,
                         "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                         "copy-calibrated)",
                         "kernel": "k_dress_inplace (in-place dress+merge+truncate+energy)",
                         "alg_bytes_per_chain": alg_bytes,
                         "alg_bytes_per_launch": alg_bytes / N_STEPS_CHAIN,
                         "traffic_over_alg_bytes": (traffic / (alg_bytes / N_STEPS_CHAIN)
                                                    if traffic else None),
                         "avg_launch_ms": kernel_s / N_STEPS_CHAIN * 1e3,
                         "measured_copy_gbps": copy_gbps,
                         "frac_of_measured_copy": achieved / copy_gbps},
            "per_step": [{"n_in": s_[0], "n_anti": s_[1], "n_new": s_[2], "n_out": s_[3],
                          "sum_c2": sum_c2[j],
                          "energy": float(e_carry[j].item()), "ms": round(per_step[j] * 1e3, 4),
                          "alg_gbps": alg[j] / per_step[j] / 1e9}
                         for j, s_ in enumerate(sizes)],
            "sum_c2_h0": sum_c2_h0,
            "h0_copy_ms": copy_s * 1e3,
            "final_energy": float(e_carry[-1].item()),
            "bit_identical_replays": bool(identical),
            "inplace": {"relocated_items": int(relocated), "region_rows": ip_stats["region_rows"],
                        "pool_rows_used": ip_stats["pool_used"],
                        "bucket_terms_at_max": iqcc.iqcc_get_param(ctx.handle, "inplace_bucket_terms"),
                        "max_terms": max_ip},
            "energy": {"mode": "carried forward from step to step (only changed terms "
                               "evaluated); step 0 summed in full",
                       "max_abs_diff_vs_full_sum": carry_err,
                       "chain_ms_full_sum_every_step": full_s * 1e3},
        })
        log(f"chain {chain_s*1e3:.2f} ms, kernels {kernel_s*1e3:.2f} ms, {achieved:.0f} GB/s algorithmic")
        if args.only == "chain":
            print(json.dumps(result), flush=True)
            return
        if not args.no_autotune:
            # the tuner's pick for this chain is reported; the headline above
            # keeps the default knobs, which the committed counter profile names
            from paper_2603_08883_amd import autotune
            before = {k: iqcc.iqcc_get_param(ctx.handle, k) for k in autotune.INPLACE_SPACE}
            tp_, ts_ = autotune.tune_inplace(ctx, h0, work, ents, taus, EPS, tht, pht, W, len(c))
            result["inplace_autotune"] = {"params": tp_, "chain_ms_at_tuning": ts_ * 1e3,
                                          "default_params": before,
                                          "headline_chain_ms_default_params": chain_s * 1e3}
            autotune.apply(ctx, before)
            chain()   # the final store again under the default knobs
        final = work
        result["angle_backward"] = angle_backward_leg(ctx, stream, work, tht, pht, bt)
        # stand-alone QMF energy of the final Hamiltonian (HBM bound: 40 B per term)
        e1 = torch.zeros(1, dtype=torch.float64, device="cuda")
        iqcc.iqcc_qmf_energy(ctx.handle, final.handle, tht, pht, e1)
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True); ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(5):
            iqcc.iqcc_qmf_energy(ctx.handle, final.handle, tht, pht, e1)
        ev1.record(stream)
        torch.cuda.synchronize()
        t_e = ev0.elapsed_time(ev1) * 1e-3 / 5
        n_fin0 = final.count()
        result["qmf_energy"] = {
            "workload": f"stand-alone energy of the final 124-qubit Hamiltonian ({n_fin0} terms)",
            "ms": t_e * 1e3, "hbm_gbps_algorithmic": bt * n_fin0 / t_e / 1e9,
            "roofline_frac": bt * n_fin0 / t_e / 1e9 / HBM_PEAK_GBPS,
            "frac_of_measured_copy": bt * n_fin0 / t_e / 1e9 / copy_gbps,
            "matches_fused_energy": abs(float(e1.item()) - float(e_carry[-1].item())) <= 1e-10}
        # the out-of-place kernel on the same chain (every kept term rewritten
        # into a fresh store), for comparison
        s1 = iqcc.Store(ctx, N_QUBITS, max_ip)
        s2 = iqcc.Store(ctx, N_QUBITS, max_ip)
        h0p = iqcc.Store(ctx, N_QUBITS, 2 * len(c)).load_numpy(x, z, c)
        e_oop = torch.zeros(N_STEPS_CHAIN, dtype=torch.float64, device="cuda")

        def chain_oop():
            src = h0p
            for j, ((px, pz), tau) in enumerate(zip(ents, taus)):
                dst = (s1, s2)[j % 2]
                if j > 0:
                    iqcc.iqcc_dress_energy_update(ctx.handle, src.handle, px, pz, tau, EPS, dst.handle,
                                                  tht, pht, e_oop[j - 1:j], e_oop[j:j + 1])
                else:
                    iqcc.iqcc_dress(ctx.handle, src.handle, px, pz, tau, EPS, dst.handle, tht, pht,
                                    e_oop[j:j + 1])
                src = dst
            return src

        oop_final = chain_oop()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            oop_final = chain_oop()
        torch.cuda.synchronize()
        oop_s = (time.perf_counter() - t0) / args.steps
        result["out_of_place_chain"] = {
            "workload": "the same 20-step chain through the out-of-place kernel (k_dress: every kept "
                        "term written to a fresh store)",
            "chain_ms": oop_s * 1e3, "final_terms": oop_final.count(),
            "energy_max_abs_diff_vs_inplace": float((e_oop - e_carry).abs().max().item()),
            "inplace_speedup": oop_s / chain_s}
        log(f"out-of-place chain {oop_s*1e3:.2f} ms")
        # term-limit compression of the final Hamiltonian to 80 % of its terms
        n_fin = final.count()
        limit = int(0.8 * n_fin)
        other = s1 if oop_final is s2 else s2
        iqcc.iqcc_truncate_top(ctx.handle, oop_final.handle, limit, other.handle)
        torch.cuda.synchronize()
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            iqcc.iqcc_truncate_top(ctx.handle, oop_final.handle, limit, other.handle)
        torch.cuda.synchronize()
        t_lim = (time.perf_counter() - t0) / reps
        # two |c| digit passes over every term (the later ones read only the
        # terms that share the first digit) + copy of the kept terms
        lim_bytes = 2 * 8 * n_fin + bt * (n_fin + limit)
        result["term_limit"] = {
            "workload": f"final 124-qubit Hamiltonian ({n_fin} terms) limited to {limit} terms "
                        "(largest |c|, canonical-key tie-break)",
            "ms": t_lim * 1e3, "terms_per_s": n_fin / t_lim,
            "hbm_gbps_algorithmic": lim_bytes / t_lim / 1e9,
            "alg_bytes": lim_bytes, "kept": other.count()}
        log(f"term limit {n_fin} -> {limit}: {t_lim*1e3:.2f} ms")
        if not args.no_cpu_baseline:
            from oracle import oracle as O
            t0 = time.perf_counter()
            O.truncate_top(x, z, c, int(0.8 * len(c)))
            dt = time.perf_counter() - t0
            result["term_limit"]["cpu_oracle"] = {
                "kind": "oracle", "cores": 1, "terms_per_s": len(c) / dt,
                "sample": f"the initial Hamiltonian ({len(c)} terms) limited to 80 %, {dt:.2f} s"}
        h0.close(); work.close(); s1.close(); s2.close(); h0p.close()
        if not args.no_cpu_baseline:
            log("CPU baseline (oracle)...")
            result["cpu_baseline"] = cpu_baseline(x, z, c, ents, taus, th, ph)
        del x, z, c
        torch.cuda.empty_cache()

    if not args.no_sortless and "roofline" in result:
        result["sortless_dressing"] = sortless_leg(ctx, wl, result["ms_per_step"],
                                                   result["config"]["final_terms"])
        log(f"sortless chain {result['sortless_dressing']['chain_ms']:.1f} ms")
        torch.cuda.empty_cache()

    if not args.no_autograd:
        result["autograd"] = autograd_leg(ctx, stream, wl)
        torch.cuda.empty_cache()
    if not args.no_c5:
        result["c5_optimisation"] = c5_leg(ctx, wl)
    wl_ext = wl if not args.no_extended else None
    del wl

    if not args.no_dis:
        t = time.perf_counter()
        nq = 100
        x, z, c = I.hamiltonian_expanded(nq, DIS_CONFIG, 10**7)
        cx, cz = I.dis_candidates(x, nq, 10**4, 12, I.rng_for(DIS_CONFIG, I.PURPOSE_CANDIDATES))
        th, ph = I.qmf_angles(nq, I.rng_for(DIS_CONFIG, I.PURPOSE_ANGLES))
        log(f"DIS workload generated in {time.perf_counter() - t:.1f}s")
        h = iqcc.Store(ctx, nq, len(c)).load_numpy(x, z, c)
        tht = torch.from_numpy(th).cuda(); pht = torch.from_numpy(ph).cuda()
        dcx = iqcc.to_device_words(cx); dcz = iqcc.to_device_words(cz)
        dis_tuned = None
        dis_defaults = {k: iqcc.iqcc_get_param(ctx.handle, k) for k in ("dis_tile", "dis_bucket_ranges")}
        if not args.no_autotune:
            from paper_2603_08883_amd import autotune
            ns_t = min(2048, cx.shape[0])
            tp_, ts_ = autotune.tune_dis(ctx, h, tht, pht, dcx[:, :ns_t].contiguous(),
                                         dcz[:, :ns_t].contiguous(), x.shape[1], len(c))
            dis_tuned = {"params": tp_, "sample_candidates": ns_t, "sample_s_at_tuning": ts_}
        g = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, dcx, dcz, iqcc.IQCC_DIS_BATCHED)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        reps = 2
        e0.record(stream)
        for _ in range(reps):
            g = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, dcx, dcz, iqcc.IQCC_DIS_BATCHED)
        e1.record(stream)
        torch.cuda.synchronize()
        tb = e0.elapsed_time(e1) * 1e-3 / reps
        ns = min(args.dis_plain_sample, cx.shape[0])
        pcx = iqcc.to_device_words(cx[:ns]); pcz = iqcc.to_device_words(cz[:ns])
        gp = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, pcx, pcz, iqcc.IQCC_DIS_PLAIN)
        torch.cuda.synchronize()
        e0.record(stream)
        gp = iqcc.iqcc_dis_gradients(ctx.handle, h.handle, tht, pht, pcx, pcz, iqcc.IQCC_DIS_PLAIN)
        e1.record(stream)
        torch.cuda.synchronize()
        tp = e0.elapsed_time(e1) * 1e-3
        agree = float((g[:ns] - gp).abs().max().item())
        pairs = float(len(c)) * cx.shape[0]
        plain_bytes = (16 * x.shape[1] + 8) * len(c)   # every term read once per candidate
        plain_gbps = plain_bytes / (tp / ns) / 1e9
        ops = dis_ops_per_pair()
        result["dis"] = {
            "workload": "1e7-term 100-qubit Hamiltonian (banded JW, expanded by XOR with DIS-form "
                        "generators), 1e4 seeded DIS candidates of weight 2-12",
            "n_terms": len(c), "n_candidates": int(cx.shape[0]),
            "batched_grads_per_s": cx.shape[0] / tb, "batched_s": tb,
            "batched_pairs_per_s": pairs / tb,
            "batched_roofline": {"bound": "alu", "valu_lane_ops_per_pair": ops,
                                 "achieved": pairs / tb * ops if ops else None,
                                 "peak": VALU_LANE_OPS_PEAK, "unit": "VALU lane-ops/s",
                                 "frac": pairs / tb * ops / VALU_LANE_OPS_PEAK if ops else None},
            "plain_grads_per_s": ns / tp, "plain_sample": ns,
            "plain_ms_per_candidate": tp / ns * 1e3,
            "plain_hbm_gbps_algorithmic": plain_gbps,
            "plain_roofline_frac_hbm": plain_gbps / HBM_PEAK_GBPS,
            "speedup_batched_vs_plain": (cx.shape[0] / tb) / (ns / tp),
            "max_abs_diff_batched_vs_plain": agree,
            "knobs": {k: iqcc.iqcc_get_param(ctx.handle, k) for k in ("dis_tile", "dis_bucket_ranges")},
            "autotuned": dis_tuned,
        }
        log(f"DIS batched {cx.shape[0]/tb:.0f} grads/s, plain {ns/tp:.0f} grads/s")
        h.close()
        # the tuned DIS knobs fit this workload only: later legs get the defaults
        for k_, v_ in dis_defaults.items():
            iqcc.iqcc_set_param(ctx.handle, k_, v_)
        if "value" not in result:
            result.update({"value": cx.shape[0] / tb, "unit": "DIS grads/s", "ms_per_step": tb * 1e3,
                           "config": {"workload": result["dis"]["workload"]}})

    if not args.no_batch:
        t = time.perf_counter()
        hs = I.batch_hamiltonians(BATCH_CONFIG)
        log(f"batch workload: {len(hs)} Hamiltonians, {sum(len(h['c']) for h in hs)} terms, "
            f"{time.perf_counter() - t:.1f}s")
        ins = [iqcc.Store(ctx, h["n_qubits"], max(2 * len(h["c"]), 64)).load_numpy(h["x"], h["z"], h["c"])
               for h in hs]
        outs = [iqcc.Store(ctx, h["n_qubits"], max(2 * len(h["c"]), 64)) for h in hs]
        pxs = np.array([np.asarray(h["px"], np.uint64).reshape(1) for h in hs])
        pzs = np.array([np.asarray(h["pz"], np.uint64).reshape(1) for h in hs])
        btaus = [h["tau"] for h in hs]
        hin = [s.handle for s in ins]
        hout = [s.handle for s in outs]
        n_terms = sum(len(h["c"]) for h in hs)
        tuned = None
        batch_defaults = {k: iqcc.iqcc_get_param(ctx.handle, k)
                          for k in ("batch_anti_cap", "batch_split_bucket_terms", "batch_unit_pairs",
                                    "grid_per_cu")}
        if not args.no_autotune:
            from paper_2603_08883_amd import autotune
            tp_, ts_ = autotune.tune_batch(ctx, hin, hout, pxs, pzs, btaus, EPS, 1, n_terms)
            tuned = {"params": tp_, "graph_ms_at_tuning": ts_ * 1e3}

        def plain():
            for i in range(len(hs)):
                iqcc.iqcc_dress(ctx.handle, hin[i], pxs[i], pzs[i], btaus[i], EPS, hout[i])

        b = iqcc.iqcc_batch_create(ctx.handle, hin, hout, pxs, pzs, btaus, EPS)

        def timed(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) * 1e-3 / reps

        tp = timed(plain)
        tg = timed(lambda: iqcc.iqcc_batch_launch(ctx.handle, b))
        n_out = sum(o.count() for o in outs)
        iqcc.iqcc_batch_destroy(ctx.handle, b)
        # every input term read once and every output term written once (24 B each, W = 1)
        b_bytes = 24 * (n_terms + n_out)
        result["batch"] = {
            "workload": f"{len(hs)} Hamiltonians, 16-64 qubits, {n_terms} terms (log-uniform "
                        "1e3-1e6 each), one entangler each, eps=1e-8",
            "graph_ms": tg * 1e3, "plain_calls_ms": tp * 1e3, "speedup_graph_vs_plain": tp / tg,
            "terms_per_s_graph": n_out / tg, "output_terms": int(n_out),
            "alg_bytes": int(b_bytes), "hbm_gbps_algorithmic": b_bytes / tg / 1e9,
            "roofline_frac_hbm": b_bytes / tg / 1e9 / HBM_PEAK_GBPS,
            "knobs": {k: iqcc.iqcc_get_param(ctx.handle, k)
                      for k in ("batch_anti_cap", "batch_split_bucket_terms", "batch_unit_pairs",
                                "grid_per_cu")},
            "autotuned": tuned}
        log(f"batch: graph {tg*1e3:.3f} ms vs {len(hs)} plain calls {tp*1e3:.3f} ms")
        for s_ in ins + outs:
            s_.close()
        for k_, v_ in batch_defaults.items():
            iqcc.iqcc_set_param(ctx.handle, k_, v_)

    if not args.no_poly:
        result["energy_polynomial"] = poly_leg(ctx)
        log(f"energy polynomial {result['energy_polynomial']['ms']:.1f} ms")
        torch.cuda.empty_cache()

    if not args.no_qcc:
        result["qcc_iteration"] = qcc_leg(ctx)
        log(f"iQCC iteration {result['qcc_iteration']['iteration_ms']:.1f} ms "
            f"({result['qcc_iteration']['n_candidates']} candidates)")
        torch.cuda.empty_cache()

    if wl_ext is not None:
        result["extended_chain"] = extended_chain_leg(ctx, stream, wl_ext)

    ctx.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
