"""Autotuner for bucket and tile sizes of the dressing kernels.

Times candidate settings of the library's knobs ("anti_cap", "grid_per_cu",
"split_bucket_terms", their batched-dressing counterparts "batch_anti_cap",
"batch_split_bucket_terms" and "batch_unit_pairs", and the DIS tile "dis_tile") on the caller's own workload through
the C ABI, keeps the fastest, and caches the choice in a JSON file keyed by
(device architecture, words per key, log2 of the term count, workload kind).
Only timing and bookkeeping happen here; every measured call runs in libiqcc.
"""
from __future__ import annotations

import itertools
import json
import math
import os

import torch

from . import iqcc

CACHE = os.environ.get("IQCC_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "iqcc", "autotune.json"))

BATCH_SPACE = {"batch_anti_cap": [512, 1024], "grid_per_cu": [1, 2, 4],
               "batch_split_bucket_terms": [384, 768], "batch_unit_pairs": [4, 8, 32]}
CHAIN_SPACE = {"anti_cap": [512, 1024], "grid_per_cu": [1, 2, 4],
               "split_bucket_terms": [256, 384, 768]}
# the stash size (inplace_cap) is not searched: the knob can only lower it
# below what the LDS holds, and a smaller stash only relocates more items
INPLACE_SPACE = {"inplace_item_terms": [0, 128, 192, 256, 384]}
DIS_SPACE = {"dis_tile": [64, 128, 256], "dis_bucket_ranges": [0, 512, 1024]}


def _arch():
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _key(kind, W, n_terms, extra=""):
    return f"{_arch()}|{kind}|W{W}|n2^{int(math.log2(max(n_terms, 1)))}|{extra}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except Exception:
        return {}


def _save(d):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def apply(ctx, params: dict):
    for k, v in params.items():
        iqcc.iqcc_set_param(ctx.handle, k, int(v))


def _time(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def tune_batch(ctx, ins, outs, pxs, pzs, taus, eps, W, n_terms, space=None, use_cache=True):
    """Pick knobs for a batched dressing (graph replay time); returns (params, seconds)."""
    space = space or BATCH_SPACE
    cache = _load()
    key = _key("batch", W, n_terms, f"h{len(ins)}")
    if use_cache and key in cache:
        apply(ctx, cache[key]["params"])
        return cache[key]["params"], cache[key]["seconds"]
    best = None
    names = sorted(space)
    for vals in itertools.product(*[space[k] for k in names]):
        params = dict(zip(names, vals))
        try:
            apply(ctx, params)
            b = iqcc.iqcc_batch_create(ctx.handle, ins, outs, pxs, pzs, taus, eps)
        except iqcc.IqccError:
            continue
        try:
            t = _time(lambda: iqcc.iqcc_batch_launch(ctx.handle, b))
            for o in outs:   # a setting whose outputs overflowed does not count
                iqcc.iqcc_store_count(ctx.handle, o)
        except iqcc.IqccError:
            continue
        finally:
            iqcc.iqcc_batch_destroy(ctx.handle, b)
        if best is None or t < best[1]:
            best = (params, t)
    apply(ctx, best[0])
    cache[key] = {"params": best[0], "seconds": best[1]}
    _save(cache)
    return best


def tune_chain(ctx, h0, stores, entanglers, taus, eps, W, n_terms, steps=4, space=None,
               use_cache=True):
    """Pick knobs for the dressing chain (first `steps` steps); returns (params, seconds)."""
    space = space or CHAIN_SPACE
    cache = _load()
    key = _key("chain", W, n_terms, f"s{steps}")
    if use_cache and key in cache:
        apply(ctx, cache[key]["params"])
        return cache[key]["params"], cache[key]["seconds"]
    best = None
    names = sorted(space)
    for vals in itertools.product(*[space[k] for k in names]):
        params = dict(zip(names, vals))
        try:
            apply(ctx, params)
        except iqcc.IqccError:
            continue

        def run():
            src = h0
            for j in range(steps):
                dst = stores[j % 2]
                px, pz = entanglers[j]
                iqcc.iqcc_dress(ctx.handle, src.handle, px, pz, float(taus[j]), eps, dst.handle)
                src = dst

        try:
            t = _time(run)
        except iqcc.IqccError:
            continue
        if best is None or t < best[1]:
            best = (params, t)
    apply(ctx, best[0])
    cache[key] = {"params": best[0], "seconds": best[1]}
    _save(cache)
    return best


def _search(ctx, space, key, run, use_cache, check=None):
    """Time `run` under every setting of `space` (cached under `key`); a
    setting for which `check()` raises (e.g. a capacity error of the last
    run) is skipped.  The best setting is applied and run once more, so the
    caller's outputs come from it."""
    cache = _load()
    if use_cache and key in cache:
        apply(ctx, cache[key]["params"])
        return cache[key]["params"], cache[key]["seconds"]
    before = {k: iqcc.iqcc_get_param(ctx.handle, k) for k in space}
    best = None
    names = sorted(space)
    for vals in itertools.product(*[space[k] for k in names]):
        params = dict(zip(names, vals))
        try:
            apply(ctx, params)
            t = _time(run)
            if check is not None:
                check()
        except iqcc.IqccError:
            continue
        if best is None or t < best[1]:
            best = (params, t)
    if best is None:
        apply(ctx, before)
        raise RuntimeError("no setting of the search space ran")
    apply(ctx, best[0])
    run()
    if check is not None:
        check()
    cache[key] = {"params": best[0], "seconds": best[1]}
    _save(cache)
    return best


def tune_inplace(ctx, h0, work, entanglers, taus, eps, theta, phi, W, n_terms, space=None,
                 use_cache=True):
    """Pick the in-place dressing knobs for a chain (copy of H0 + every step with
    the fused energy); returns (params, seconds)."""
    space = space or INPLACE_SPACE
    e = torch.zeros(max(len(entanglers), 1), dtype=torch.float64, device="cuda")

    def run():
        iqcc.iqcc_store_copy(ctx.handle, h0.handle, work.handle)
        for j, ((px, pz), t) in enumerate(zip(entanglers, taus)):
            iqcc.iqcc_dress_inplace(ctx.handle, work.handle, px, pz, float(t), eps, theta, phi,
                                    e[j - 1:j] if j else None, e[j:j + 1])

    return _search(ctx, space, _key("inplace", W, n_terms, f"s{len(entanglers)}"), run, use_cache,
                   check=lambda: iqcc.iqcc_store_count(ctx.handle, work.handle))


def tune_dis(ctx, store, theta, phi, cx, cz, W, n_terms, space=None, use_cache=True):
    """Pick the batched DIS tile and bucket ranges on the caller's candidates
    (cx, cz device words, a sample is enough); returns (params, seconds)."""
    space = space or DIS_SPACE

    def run():
        iqcc.iqcc_dis_gradients(ctx.handle, store.handle, theta, phi, cx, cz, iqcc.IQCC_DIS_BATCHED)

    return _search(ctx, space, _key("dis", W, n_terms, f"c{cx.shape[1]}"), run, use_cache)
