"""Benchmark: MergeShuffle of one uint32 identity array, n = 2^30, seed 7, on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--n-log2 30] [--no-cpu-baseline]

A step is one complete shuffle of the resident 4 GiB array: the plan, the
leaf kernel (Fisher-Yates of every leaf plus the merge levels that fit in
LDS) and the HBM merge passes (each runs three or four merge levels, their
insertion loops included).  The JSON line carries the whole-job throughput
(Gelem/s), the roofline of the kernel class that takes most of the step
(measured with HIP events around each launch on the library's stream), and
the CPU oracle timed on a bounded sample.

Roofline figures:
  * merge pass (HBM-bound): algorithmic bytes per launch = 2 * n * 4 (every
    element read once and written once, however many levels the pass runs),
    against 8 TB/s;
  * leaf kernel (ALU-bound): algorithmic integer ops per element = the
    Philox-4x32-10 work of the bits it draws (one 100-op block per 4 leaf
    draws and per 128 coin flips of each LDS level) plus about 10 ops per
    Fast Dice Roller draw, against 256 CUs x 64 lanes x 2.4 GHz.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ALU_PEAK_GOPS = 256 * 64 * 2.4  # int32 vector lane-ops per ns -> Gop/s: 39321.6
PHILOX_OPS = 100.0
FDR_OPS = 10.0


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ms_kernels_data.hip", "ms_kernels_group.hip", "ms_kernels_pass.hip", "ms_device.hpp", "ms_plan.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1508_03167_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def valu_issue_from_profiles(kernel_class: str):
    """Fraction of the chip's VALU issue capacity the kernel used, from the
    committed instruction-counter summary, if it was taken on the current
    kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "merge_pass_and_leaf_n2^30_u32_instructions.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_source_hash() or kernel_class not in d:
        return None
    return round(d[kernel_class]["valu_issue_frac"], 3)


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_log2: int, single_log2: int = 25):
    """The oracle on this host's cores: one MergeShuffle of a uint32 identity
    array of 2^n_log2 elements (half the GPU step's size, so that the run takes
    about 10 s on 16 cores) with OpenMP over the blocks and over the merges of
    each level, and a single-thread leg on 2^single_log2 elements (about the
    same time on one core)."""
    from oracle import oracle as O

    threads = max(1, min(os.cpu_count() or 1, 64))
    O.build(force=False)
    n = 1 << n_log2
    t = time.perf_counter()
    O.permutation(n, 4096, 7, threads=threads)
    dt = time.perf_counter() - t
    n1 = 1 << single_log2
    t = time.perf_counter()
    O.permutation(n1, 4096, 7, threads=1)
    dt1 = time.perf_counter() - t
    return {"value": round(n / dt / 1e9, 4), "unit": "Gelem/s", "cores": threads, "kind": "oracle",
            "cpu": _cpu_model(),
            "sample": f"one MergeShuffle of a uint32 identity array, n=2^{n_log2}, seed 7, cutoff 4096 "
                      f"(the GPU step's procedure at 1/{1 << max(0, 30 - n_log2)} of its size, so the run stays "
                      f"near 10 s), {dt:.2f} s, OpenMP over the blocks and over the merges of a level",
            "single_thread": {"value": round(n1 / dt1 / 1e9, 4), "unit": "Gelem/s", "cores": 1,
                              "sample": f"n=2^{single_log2}, seed 7, cutoff 4096, {dt1:.2f} s"}}


def bench_batched(M, torch, reps: int = 5, count: int = 4096, seed: int = 3, tune: bool = True):
    """4096 uint32 arrays of log-uniform sizes in [2^8, 2^20] (seed_a = 3 + a),
    resident in HBM: one eager batched call, the same call captured in a HIP
    graph and replayed, the graph with autotuned knobs (cutoff, levels per
    pass, leaf shape per size bucket), and one call per array."""
    from paper_1508_03167_amd import autotune, inputs

    sizes = inputs.batched_sizes(count, seed)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    total = int(offs[-1])
    buf = torch.arange(total, dtype=torch.int32, device="cuda:0")
    views = [buf[int(offs[i]):int(offs[i + 1])] for i in range(count)]
    seeds = [seed + a for a in range(count)]

    def wall(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def replay(cfgs):
        g = M.BatchGraph(views, seeds, cfgs=cfgs)
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
            assert g.status() == 0
            return e0.elapsed_time(e1) / reps / 1e3, g.scratch_bytes
        finally:
            g.destroy()

    tb = wall(lambda: M.shuffle_batched_(views, seed))
    tg, gbytes = replay(None)
    out = {"workload": f"{count} uint32 arrays, sizes floor(2^(8+12u)), seed {seed}+a",
           "arrays": count, "elements": total,
           "arrays_in_one_workgroup": int(sum(1 for v in sizes if M.plan(int(v))["hbm_levels"] == 0)),
           "batched_ms": round(tb * 1e3, 3), "batched_gelem_s": round(total / tb / 1e9, 3),
           "graph_replay_ms": round(tg * 1e3, 3), "graph_replay_gelem_s": round(total / tg / 1e9, 3),
           "graph_scratch_bytes": gbytes}
    if tune:
        path = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"ms_tune_{os.getpid()}.json")
        t0 = time.perf_counter()
        rec = autotune.tune_for_batch(views, seeds, path=path, budget=1 << 22, reps=3)
        tune_s = time.perf_counter() - t0
        try:
            tt, _ = replay([M.config(tuned=True)] * count)
            out["tuned_graph_replay_ms"] = round(tt * 1e3, 3)
            out["tuned_graph_replay_gelem_s"] = round(total / tt / 1e9, 3)
            out["tuned_cutoffs_used"] = sorted({M.leaf_B_for(int(v)) for v in sizes})
        finally:
            M.tune_set([])
        out["tuning"] = {"seconds": round(tune_s, 2), "batch": rec["batch"], "per_bucket": {
            f"2^{e['log2_n']}": [e["leaf_B"], e["levels_per_pass"], "1024 thr" if e["leaf_big"] else "512 thr"]
            for e in rec["entries"]}}
    tl = wall(lambda: [M.shuffle_(v, seed + i) for i, v in enumerate(views)])
    out.update({"loop_ms": round(tl * 1e3, 3), "loop_gelem_s": round(total / tl / 1e9, 3),
                "speedup_batched_over_loop": round(tl / tb, 3),
                "speedup_graph_over_loop": round(tl / tg, 3)})
    del buf, views
    return out


def bench_r1(M, torch, n_log2: int = 26, seed: int = 7, reps: int = 5):
    """The printed listing's in-place placement (every level a one-level HBM
    pass whose A slots are gathered through the swap chains) against the
    default path and the default placement run the same way, uint32 identity."""
    n = 1 << n_log2
    x = torch.empty(n, dtype=torch.int32, device="cuda:0")

    def timed(**kw):
        M.permutation(x, seed, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            M.permutation(x, seed, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t1 = timed(placement="R1")
    t2 = timed(hbm_only=True, one_level_passes=True)
    t0 = timed()
    del x
    return {"workload": f"MergeShuffle permutation of 0..2^{n_log2}-1, seed {seed}, cutoff 4096, "
                        f"listing placement (R1)",
            "n": n, "r1_ms": round(t1 * 1e3, 3), "r1_gelem_s": round(n / t1 / 1e9, 3),
            "stable_one_level_hbm_only_ms": round(t2 * 1e3, 3), "default_path_ms": round(t0 * 1e3, 3)}


def bench_balanced(M, torch, n_log2: int = 26, seed: int = 7, reps: int = 5):
    """BalancedShuffle (Section 2): every level a one-level HBM pass over the
    final side labels the plan writes, against the default merge run the
    same way (one-level passes, every level in HBM) and the default path."""
    n = 1 << n_log2
    x = torch.empty(n, dtype=torch.int32, device="cuda:0")

    def timed(**kw):
        M.permutation(x, seed, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            M.permutation(x, seed, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    tb = timed(placement="BAL")
    t2 = timed(hbm_only=True, one_level_passes=True)
    t0 = timed()
    del x
    return {"workload": f"MergeShuffle permutation of 0..2^{n_log2}-1, seed {seed}, cutoff 4096, "
                        f"BalancedShuffle merges",
            "n": n, "balanced_ms": round(tb * 1e3, 3), "balanced_gelem_s": round(n / tb / 1e9, 3),
            "stable_one_level_hbm_only_ms": round(t2 * 1e3, 3), "default_path_ms": round(t0 * 1e3, 3)}


def _timed_classes(M, torch, fn, reps: int):
    """Wall time per call of fn() and the library's per-class kernel times."""
    fn()
    torch.cuda.synchronize()
    M.profile_read()
    M.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    M.profile_enable(False)
    ms, cnt = M.profile_read()
    return dt, ms, cnt


def bench_records(M, torch, n_log2: int = 27, seed: int = 11, reps: int = 5):
    """16-byte records {uint64 key from a seeded stream, uint64 payload = index},
    shuffled whole (the same permutation as the uint32 index array)."""
    from paper_1508_03167_amd.inputs import records16

    n = 1 << n_log2
    rec = torch.from_numpy(records16(n, seed).view(np.int64)).to("cuda:0")
    dt, ms, cnt = _timed_classes(M, torch, lambda: M.shuffle_(rec, seed), reps)
    del rec
    launches = max(cnt["merge_pass"], 1)
    avg = ms["merge_pass"] / launches
    gbs = 2.0 * n * 16 / (avg / 1e3) / 1e9
    return {"workload": f"MergeShuffle of 2^{n_log2} 16-byte records (uint64 key from a seeded stream, "
                        f"uint64 payload = index), seed {seed}, cutoff 4096",
            "n": n, "record_bytes": 16, "ms": round(dt * 1e3, 3), "gelem_s": round(n / dt / 1e9, 3),
            "merge_pass_avg_ms": round(avg, 4), "merge_passes": cnt["merge_pass"] // reps,
            "merge_pass_gb_s": round(gbs, 1), "merge_pass_frac_of_8tbs": round(gbs / HBM_PEAK_GBS, 4),
            "ms_by_kernel_class": {k: round(v / reps, 3) for k, v in ms.items()}}


def bench_small(M, torch, n_log2: int = 20, seed: int = 1, reps: int = 200):
    """The small plain-permutation case: a uint32 identity array of 2^20
    elements (4 MiB, resident in the caches), one call after another."""
    n = 1 << n_log2
    x = torch.arange(n, dtype=torch.int32, device="cuda:0")
    dt, ms, cnt = _timed_classes(M, torch, lambda: M.shuffle_(x, seed), reps)
    del x
    return {"workload": f"MergeShuffle of one uint32 identity array, n=2^{n_log2}, seed {seed}, cutoff 4096",
            "n": n, "ms": round(dt * 1e3, 4), "gelem_s": round(n / dt / 1e9, 3),
            "launches_per_call": {k: round(v / reps, 2) for k, v in cnt.items()},
            "ms_by_kernel_class": {k: round(v / reps, 4) for k, v in ms.items()}}


def bench_served(M, torch, count: int = 20000, seed: int = 5, load: float = 0.7, budget_gib: int = 32,
                 inflight: int = 3, batch_elems: int = 1 << 21):
    """20k requests of log-uniform size in [2^10, 2^26] elements, uint32 or
    uint64 (random values), Poisson arrivals at `load` times the measured
    capacity, admitted against an HBM budget (payload + library scratch) and
    served by the continuous-batching server: the admitted requests go, in
    arrival order, into the next batched call on a free stream (up to
    `inflight` batches on the device; a batch closes before it would exceed
    `batch_elems` elements, so a large request goes alone, and one large
    request is on the device at a time, passed meanwhile by smaller ones).
    The same stream
    through the plain loop: one ms_shuffle call per request, one at a time,
    same admission.  Capacity is the throughput of the first 2000 requests all
    present at the start, after a warm-up on the first 300."""
    from paper_1508_03167_amd import inputs
    from paper_1508_03167_amd.serve import GpuExecutor, Request, serve_stream

    spec = inputs.served_requests(count, seed, rate_per_s=1.0)
    budget = budget_gib << 30
    mean_n = float(np.mean([d["n"] for d in spec]))

    def fill(pool):
        g = torch.Generator(device="cuda:0")
        g.manual_seed(seed)
        pool.random_(0, 256, generator=g)

    def requests(rate, k=count):
        return [Request(i, d["n"], d["elem_bytes"], d["seed"], d["arrival_s"] / rate if rate else 0.0)
                for i, d in enumerate(spec[:k])]

    def run(rate, k, batched, check=()):
        ex = GpuExecutor(budget, inflight if batched else 1, fill=fill, batched=batched, check=check)
        if batched:
            r = serve_stream(requests(rate, k), ex, budget, inflight, max_batch_elems=batch_elems,
                             max_large_inflight=1)
        else:
            r = serve_stream(requests(rate, k), ex, budget, max_inflight=1, max_batch=1)
        if check:
            ex.verify()
            r["results_checked_alone"] = len(ex.checked)
            r["results_equal_alone_and_in_mix"] = not ex.mismatches and len(ex.checked) == len(check)
        del ex
        torch.cuda.empty_cache()
        return r

    run(None, 300, True)
    cap = run(None, 2000, True)
    cap_plain = run(None, 2000, False)
    rate = load * cap["gelem_s"] * 1e9 / mean_n
    batched = run(rate, count, True, check=set(range(0, count, count // 16)))
    plain = run(rate, count, False)
    return {"workload": f"{count} requests, sizes floor(2^(10+16u)), uint32 or uint64 random values, "
                        f"Poisson arrivals at {load} x measured capacity, HBM budget {budget_gib} GiB, seed {seed}",
            "requests": count, "mean_elements": round(mean_n), "inflight_batches": inflight,
            "batch_elems_cap": batch_elems, "large_requests_in_flight": 1,
            "capacity_gelem_s": {"continuous_batching": cap["gelem_s"], "one_call_per_request": cap_plain["gelem_s"]},
            "arrival_rate_req_s": round(rate, 1),
            "continuous_batching": batched, "one_call_per_request": plain}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-log2", type=int, default=30)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-log2", type=int, default=29)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the batched, served, listing-placement, balanced, records and small workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 2^28 uint32 (1 GiB) for counter calibration")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        a = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_dispatch": 1 << 30}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (no multi-GPU path)"}))
        sys.exit(2)

    import torch

    import paper_1508_03167_amd as M

    n = 1 << args.n_log2
    x = torch.arange(n, dtype=torch.int32, device="cuda:0")
    plan = M.plan(n, 4)
    plan_tile = 8192 if n >= (1 << 26) and not os.environ.get("MS_PASS_TILE") else int(os.environ.get("MS_PASS_TILE", 3584))
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
    assert M.device_status() == 0, "plan pool overflow flagged"
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e9

    def pass_roof():
        launches = max(cnt_cls["merge_pass"], 1)
        avg = ms_cls["merge_pass"] / launches
        ach = 2.0 * n * 4 / (avg / 1e3) / 1e9
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": traffic_from_profiles("merge_pass_n2^30_u32"),
                "kernel": f"pass_kernel<uint32_t,{plan_tile},levels,{1024 if plan_tile == 8192 else 512}>",
                "avg_launch_ms": round(avg, 4),
                "launches": cnt_cls["merge_pass"],
                "levels_per_launch": round(plan["hbm_levels"] * args.steps / launches, 3),
                "alg_bytes_per_launch": 2 * n * 4,
                "valu_issue_frac_from_counters": valu_issue_from_profiles("merge_pass")}

    def leaf_roof():
        launches = max(cnt_cls["leaf"], 1)
        avg = ms_cls["leaf"] / launches
        ops_per_elem = PHILOX_OPS * (0.25 + plan["lds_levels"] / 128.0) + FDR_OPS
        ach = ops_per_elem * n / (avg / 1e3) / 1e9
        return {"bound": "alu", "achieved": round(ach, 1), "peak": ALU_PEAK_GOPS, "unit": "Gop/s",
                "frac": round(ach / ALU_PEAK_GOPS, 4), "traffic": traffic_from_profiles("leaf_n2^30_u32"),
                "kernel": "leaf_kernel<uint32_t,16384,512>", "avg_launch_ms": round(avg, 4),
                "launches": cnt_cls["leaf"], "alg_ops_per_launch": ops_per_elem * n,
                "alg_bytes_per_launch": 2 * n * 4,
                "valu_issue_frac_from_counters": valu_issue_from_profiles("leaf")}

    roofs = {"merge_pass": pass_roof(), "leaf": leaf_roof()}
    dominant = max(("merge_pass", "leaf"), key=lambda k: ms_cls[k])
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
                   "hbm_levels": plan["hbm_levels"], "hbm_passes": cnt_cls["merge_pass"] // args.steps,
                   "parallelism": "single GPU"},
        "roofline": dict(roofs[dominant], dominant_kernel_class=dominant),
        "roofline_other": roofs["leaf" if dominant == "merge_pass" else "merge_pass"],
        "ms_per_step_by_kernel_class": breakdown,
    }
    if not args.no_extra:
        del x
        torch.cuda.empty_cache()
        out["batched"] = bench_batched(M, torch)
        torch.cuda.empty_cache()
        out["served"] = bench_served(M, torch)
        torch.cuda.empty_cache()
        out["r1_placement"] = bench_r1(M, torch)
        torch.cuda.empty_cache()
        out["balanced"] = bench_balanced(M, torch)
        torch.cuda.empty_cache()
        out["records"] = bench_records(M, torch)
        torch.cuda.empty_cache()
        out["small"] = bench_small(M, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample_log2)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
