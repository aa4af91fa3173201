#!/usr/bin/env python3
"""Write the expected values of the full-size parity tests (CPU only).

Every number written here comes from the FP64 CPU oracle (`oracle/`) applied
to the seeded inputs of `paper_2603_08883_amd/inputs.py`; nothing from the HIP
library is read.  Files (JSON, floats also as exact hex strings):

  c3_chain.json   124-qubit chain (banded JW H0, 20 DIS entanglers, eps=1e-8):
                  per step N_in, N_anti, N_out, the Neumaier QMF energy
                  (Eq. 3) and the multiset digest of the output terms (Eq. 5
                  dressing, App. D merge, compression); for the final
                  Hamiltonian the 248 angle gradients, and dE/dtau_k for
                  k in {0, 9, 19} with the compression masks frozen (Eq. 6).
  c4a_dis.json    DIS gradients (Eq. 7) of a seeded sample of 32 of the 1e4
                  screening candidates against the 1e7-term 100-qubit H.
  c4b_batch.json  the 64 Hamiltonians of the batched-dressing workload, each
                  dressed by its entangler (count and digest of the output).

Usage: python tests/golden/make_goldens.py [--only c3,c4a,c4b]
Takes about 20 minutes and up to ~30 GB of host memory for c3.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O                     # noqa: E402
from paper_2603_08883_amd import inputs as I       # noqa: E402
from tests.golden.multiset_hash import multiset_hash  # noqa: E402

EPS = 1e-8
TAU_K = (0, 9, 19)
DIS_SAMPLE = 32
DIS_SAMPLE_SEED = 4242


def log(*a):
    print("[golden]", *a, flush=True)


def fl(v):
    v = float(v)
    return {"value": v, "hex": v.hex()}


def write(name, obj):
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        json.dump(obj, f, indent=1)
    os.replace(path + ".tmp", path)
    log("wrote", path)


def c3():
    nq, steps, config = 124, 20, 2
    t0 = time.time()
    x, z, c = I.hamiltonian_banded(nq, config, band=6, decay=3.0)
    cx, cz = I.dis_candidates(x, nq, steps, 8, I.rng_for(config, I.PURPOSE_ENTANGLERS))
    taus = [float(t) for t in I.taus(steps, I.rng_for(config, I.PURPOSE_TAUS))]
    th, ph = I.qmf_angles(nq, I.rng_for(config, I.PURPOSE_ANGLES))
    ents = list(zip(cx, cz))
    log(f"c3 inputs: {len(c)} terms ({time.time() - t0:.0f} s)")
    out = {"workload": "124-qubit banded JW Hamiltonian (62 orbitals, band 6, decay 3), "
                       "20 seeded DIS entanglers, tau~U(-0.2,0.2), eps=1e-8",
           "n_qubits": nq, "eps": EPS, "initial_terms": int(len(c)),
           "initial_digest": f"{multiset_hash(x, z, c):016x}", "steps": []}
    keep = {}
    hx, hz, hc = x, z, c
    for j, ((px, pz), t) in enumerate(zip(ents, taus)):
        if j in TAU_K:
            keep[j] = (hx, hz, hc)
        n_in = len(hc)
        rx, rz, rc = O.dress_raw(nq, hx, hz, hc, px, pz, t)
        n_anti = len(rc) - n_in
        hx, hz, hc = O.merge_truncate(rx, rz, rc, eps=EPS)
        del rx, rz, rc
        e = O.qmf_energy(nq, hx, hz, hc, th, ph)
        out["steps"].append({"n_in": int(n_in), "n_anti": int(n_anti), "n_out": int(len(hc)),
                             "energy": fl(e), "digest": f"{multiset_hash(hx, hz, hc):016x}"})
        log(f"c3 step {j}: {n_in} -> {len(hc)} terms, E = {e:.15f} ({time.time() - t0:.0f} s)")
    dt, dp = O.qmf_grad_angles(nq, hx, hz, hc, th, ph)
    out["grad_theta"] = [fl(v) for v in dt]
    out["grad_phi"] = [fl(v) for v in dp]
    log(f"c3 angle gradients ({time.time() - t0:.0f} s)")
    del hx, hz, hc
    out["grad_tau"] = {}
    for k in TAU_K:
        sx, sz, sc = keep.pop(k)
        # the tangent is zero before step k, so the chain from H^(k) (the input
        # of step k) gives the same derivative as the chain from H0
        g, _ = O.chain_tau_gradient(nq, sx, sz, sc, ents[k:], taus[k:], EPS, th, ph, 0)
        out["grad_tau"][str(k)] = fl(g)
        log(f"c3 dE/dtau_{k} = {g:.15e} ({time.time() - t0:.0f} s)")
    write("c3_chain.json", out)


def c4a():
    nq, config = 100, 3
    t0 = time.time()
    x, z, c = I.hamiltonian_expanded(nq, config, 10**7)
    cx, cz = I.dis_candidates(x, nq, 10**4, 12, I.rng_for(config, I.PURPOSE_CANDIDATES))
    th, ph = I.qmf_angles(nq, I.rng_for(config, I.PURPOSE_ANGLES))
    idx = np.sort(np.random.default_rng(DIS_SAMPLE_SEED).choice(len(cx), DIS_SAMPLE, replace=False))
    log(f"c4a inputs ({time.time() - t0:.0f} s)")
    g = O.dis_gradients(nq, x, z, c, th, ph, cx[idx], cz[idx])
    write("c4a_dis.json", {
        "workload": "1e7-term 100-qubit screening Hamiltonian, 1e4 DIS candidates (weight 2-12)",
        "n_terms": int(len(c)), "initial_digest": f"{multiset_hash(x, z, c):016x}",
        "sample_index": [int(i) for i in idx], "grad": [fl(v) for v in g]})
    log(f"c4a done ({time.time() - t0:.0f} s)")


def c4b():
    config = 4
    t0 = time.time()
    hs = I.batch_hamiltonians(config)
    items = []
    for i, h in enumerate(hs):
        nq = h["n_qubits"]
        rx, rz, rc = O.dress_raw(nq, h["x"], h["z"], h["c"], h["px"], h["pz"], h["tau"])
        n_anti = len(rc) - len(h["c"])
        ox, oz, oc = O.merge_truncate(rx, rz, rc, eps=EPS)
        items.append({"n_qubits": nq, "n_in": int(len(h["c"])), "n_anti": int(n_anti),
                      "n_out": int(len(oc)), "digest": f"{multiset_hash(ox, oz, oc):016x}"})
    write("c4b_batch.json", {
        "workload": "64 Hamiltonians, 16-64 qubits, log-uniform 1e3-1e6 terms, one DIS entangler "
                    "each, eps=1e-8", "items": items})
    log(f"c4b done ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="c4b,c4a,c3")
    args = ap.parse_args()
    O.lib()
    for part in args.only.split(","):
        {"c3": c3, "c4a": c4a, "c4b": c4b}[part.strip()]()
