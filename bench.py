"""Benchmark: MergeShuffle of one uint32 identity array, n = 2^30, seed 7, on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--n-log2 30] [--no-cpu-baseline]

A step is one complete shuffle (plan, leaf kernel, every merge pass and its
patch) of the resident 4 GiB array.  Prints one JSON line with the whole-job
throughput in Gelem/s, the roofline of the dominant kernel (the HBM merge
pass: 2 * n * 4 algorithmic bytes per launch over its average HIP-event
duration, against 8 TB/s) and the CPU oracle timed on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ms_kernels_data.hip", "ms_device.hpp", "ms_plan.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1508_03167_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(n_bytes_alg: float):
    """HBM bytes per merge-pass launch from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "merge_pass_n2^30_u32_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(n_log2: int):
    from oracle import oracle as O

    threads = max(1, min(os.cpu_count() or 1, 64))
    n = 1 << n_log2
    O.build(force=False)
    t = time.perf_counter()
    _, bits = O.permutation(n, 4096, 7, threads=threads)
    dt = time.perf_counter() - t
    return {"value": n / dt / 1e9, "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "sample": f"one MergeShuffle of a uint32 identity array, n=2^{n_log2}, seed 7, cutoff 4096 "
                      f"(same procedure as the GPU step at 1/{1 << (30 - n_log2)} the size), "
                      f"{dt:.2f} s, OpenMP over blocks and over merges of a level"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-log2", type=int, default=30)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=26)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1508_03167_amd as M

    n = 1 << args.n_log2
    dev = torch.device("cuda:0")
    x = torch.arange(n, dtype=torch.int32, device=dev)
    plan = M.plan(n, 4)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        M.shuffle_(x, args.seed)
    torch.cuda.synchronize()
    M.profile_read()
    M.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        M.shuffle_(x, args.seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    M.profile_enable(False)
    ms_cls, cnt_cls = M.profile_read()
    assert M.device_status() == 0
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e9

    pass_launches = max(cnt_cls["merge_pass"], 1)
    pass_ms = ms_cls["merge_pass"] / pass_launches
    alg_bytes = 2.0 * n * 4
    achieved = alg_bytes / (pass_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(alg_bytes),
            "kernel": "merge_pass_kernel<uint32_t,8192>", "avg_launch_ms": round(pass_ms, 4),
            "launches": cnt_cls["merge_pass"]}
    breakdown = {k: round(v / args.steps, 3) for k, v in ms_cls.items()}

    out = {
        "metric": "Gelem/s + HBM GB/s vs peak at n=2^30 u32; batched elem/s; p99 latency",
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"MergeShuffle of one uint32 identity array, n=2^{args.n_log2}, seed {args.seed}, "
                               f"cutoff 4096, resident in HBM",
                   "n": n, "levels": plan["levels"], "lds_levels": plan["lds_levels"],
                   "hbm_passes": plan["hbm_levels"], "parallelism": "single GPU"},
        "roofline": roof,
        "ms_per_step_by_kernel_class": breakdown,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_log2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
