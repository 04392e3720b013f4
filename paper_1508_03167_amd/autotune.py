"""Autotuner for batched calls.

For each (element size, size bucket [2^k, 2^(k+1))) it times a batch of
arrays of that bucket under every candidate of three knobs -- the cutoff B,
the merge levels fused into one HBM pass, and the leaf workgroup shape
(64 KiB super-blocks of 512 threads, or 128 KiB ones of 1024) -- each
candidate as a batched call captured in a HIP graph and timed over replays,
and keeps the fastest.  For a given batch, tune_for_batch then times the
whole batch under that per-bucket table and under every uniform setting of
the three knobs, since arrays of different knobs split the batch's shared
launches, and keeps the fastest table.  The choices go to a JSON cache and
into the library's tuning table (ms_tune_set): calls made with tuned=True
then use them, and ms_leaf_B_for reports the cutoff they use.  The cutoff is
Algorithm MergeShuffle's parameter, so it changes the permutation (a replay
elsewhere needs ms_leaf_B_for's value); the other two knobs never do.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import _lib

CUTOFFS = (1024, 2048, 4096)
LEVELS_PER_PASS = (2, 3, 4)
SHAPES = (False, True)


def cache_path() -> str:
    """MS_TUNE_CACHE, else ~/.cache/mergeshuffle/tune.json."""
    return os.environ.get("MS_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "mergeshuffle",
                                                           "tune.json")


def bucket_sizes(k: int, budget: int, seed: int = 17):
    """Seeded sizes log-uniform in [2^k, 2^(k+1)), about `budget` elements in
    all (at least one array, at most 2048)."""
    count = max(1, min(2048, budget >> k))
    u = np.random.default_rng(seed * 64 + k).random(count)
    return [int(np.floor(2.0 ** (k + x))) for x in u]


def candidates(eb: int, k: int):
    """(cutoff, levels per pass, big leaf) triples worth timing for the bucket:
    levels per pass only where the bucket's largest size has HBM levels."""
    out = []
    for B in CUTOFFS:
        hbm = _lib.plan((1 << (k + 1)) - 1, eb, leaf_B=B)["hbm_levels"]
        for lpp in (LEVELS_PER_PASS if hbm else (0,)):
            for big in SHAPES:
                out.append((B, lpp, big))
    return out


def time_candidate(torch, tensors, seeds, B: int, lpp: int, big: bool, reps: int) -> float:
    """Milliseconds per replay of the batched call with these knobs."""
    cfgs = [_lib.config(leaf_B=B, levels_per_pass=lpp, leaf_big=big)] * len(tensors)
    g = _lib.BatchGraph(tensors, seeds, cfgs=cfgs)
    try:
        g.launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.launch()
        e1.record()
        torch.cuda.synchronize()
        if g.status() != 0:
            raise _lib.MSError(_lib.MS_ERR_CAPACITY, "a plan pool overflowed while tuning")
        return e0.elapsed_time(e1) / reps
    finally:
        g.destroy()


def tune_bucket(eb: int, k: int, budget: int = 1 << 23, reps: int = 5) -> dict:
    import torch

    sizes = bucket_sizes(k, budget)
    words = eb // 4
    offs = np.concatenate([[0], np.cumsum([(n * words + 3) // 4 * 4 for n in sizes])])
    buf = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    tensors = []
    for i, n in enumerate(sizes):
        v = buf[int(offs[i]):int(offs[i]) + n * words]
        tensors.append(v if eb == 4 else v.view(torch.int64).view(n, eb // 8) if eb == 16 else v.view(torch.int64))
    seeds = list(range(len(sizes)))
    timed = {}
    for B, lpp, big in candidates(eb, k):
        timed[(B, lpp, big)] = time_candidate(torch, tensors, seeds, B, lpp, big, reps)
    (B, lpp, big), ms = min(timed.items(), key=lambda kv: kv[1])
    default = timed.get((4096, 3, False), timed.get((4096, 0, False)))
    del buf, tensors
    return {"elem_bytes": eb, "log2_n": k, "leaf_B": B, "levels_per_pass": lpp, "leaf_big": big,
            "ms": round(ms, 4), "default_ms": round(default, 4), "arrays": len(sizes),
            "elements": int(sum(sizes)), "candidates": len(timed)}


def tune(buckets, budget: int = 1 << 23, reps: int = 5) -> dict:
    """Tune every (elem_bytes, k) of `buckets`; returns the cache record."""
    import torch

    t0 = time.perf_counter()
    entries = [tune_bucket(eb, k, budget, reps) for eb, k in buckets]
    return {"device": torch.cuda.get_device_name(0), "budget": budget, "reps": reps,
            "seconds": round(time.perf_counter() - t0, 2), "entries": entries}


def save(record: dict, path: str | None = None) -> str:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(record, f, indent=1)
    return path


def load(path: str | None = None) -> dict | None:
    path = path or cache_path()
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def install(record: dict):
    """Hand the record's entries to the library's tuning table."""
    _lib.tune_set(record["entries"])


def ensure_tuned(buckets, path: str | None = None, budget: int = 1 << 23, reps: int = 5) -> dict:
    """Load the cache, tune the buckets it lacks (for this device), save it and
    install the table."""
    import torch

    rec = load(path)
    dev = torch.cuda.get_device_name(0)
    if not rec or rec.get("device") != dev:
        rec = {"device": dev, "budget": budget, "reps": reps, "seconds": 0.0, "entries": []}
    have = {(e["elem_bytes"], e["log2_n"]) for e in rec["entries"]}
    missing = [b for b in buckets if tuple(b) not in have]
    if missing:
        new = tune(missing, budget, reps)
        rec["entries"] += new["entries"]
        rec["seconds"] = round(rec.get("seconds", 0.0) + new["seconds"], 2)
        save(rec, path)
    install(rec)
    return rec


def _time_table(torch, tensors, seeds, entries, reps: int) -> float:
    _lib.tune_set(entries)
    cfgs = [_lib.config(tuned=True)] * len(tensors)
    g = _lib.BatchGraph(tensors, seeds, cfgs=cfgs)
    try:
        g.launch()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            g.launch()
        e1.record()
        torch.cuda.synchronize()
        if g.status() != 0:
            raise _lib.MSError(_lib.MS_ERR_CAPACITY, "a plan pool overflowed while tuning")
        return e0.elapsed_time(e1) / reps
    finally:
        g.destroy()


def tune_for_batch(tensors, seeds, path: str | None = None, budget: int = 1 << 22, reps: int = 3) -> dict:
    """Tune for this batch of device tensors (tensor a shuffled with seeds[a]):
    the per-bucket table of its sizes, then the whole batch timed under that
    table and under each uniform (cutoff, levels per pass, leaf shape); the
    fastest table is saved, installed and returned with the timings.  The
    tensors' contents are shuffled many times over."""
    import torch

    def eb_of(t):
        return t.element_size() * (t[0].numel() if t.dim() > 1 else 1)

    buckets = sorted({(eb_of(t), int(t.shape[0]).bit_length() - 1) for t in tensors if t.shape[0] > 1})
    rec = ensure_tuned(buckets, path=path, budget=budget, reps=reps)
    per_bucket = [e for e in rec["entries"] if (e["elem_bytes"], e["log2_n"]) in set(buckets)]
    options = {"per-bucket": per_bucket}
    for B in CUTOFFS:
        for lpp in (0,) + LEVELS_PER_PASS:
            for big in SHAPES:
                options[f"uniform B={B} lpp={lpp} {'1024' if big else '512'} thr"] = [
                    {"elem_bytes": eb, "log2_n": k, "leaf_B": B, "levels_per_pass": lpp, "leaf_big": big}
                    for eb, k in buckets]
    timed = {name: _time_table(torch, tensors, seeds, ent, reps) for name, ent in options.items()}
    best = min(timed, key=timed.get)
    rec["batch"] = {"chosen": best, "ms": round(timed[best], 4),
                    "default_ms": round(timed["uniform B=4096 lpp=0 512 thr"], 4),
                    "per_bucket_ms": round(timed["per-bucket"], 4), "options": len(timed)}
    chosen = {(e["elem_bytes"], e["log2_n"]): e for e in options[best]}
    rec["entries"] = [dict(e, **{k: chosen[(e["elem_bytes"], e["log2_n"])][k]
                                 for k in ("leaf_B", "levels_per_pass", "leaf_big")})
                      if (e["elem_bytes"], e["log2_n"]) in chosen else e for e in rec["entries"]]
    save(rec, path)
    install(rec)
    return rec
