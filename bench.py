"""Benchmark: TTN-HEOM steps/sec on one MI355X (mixed precision) vs the FP64
GPU path, with the SOP-contraction kernel's roofline and the FP64 CPU oracle
timed on a bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints ONE JSON line (see the keys below).  Inputs are seeded and synthetic
(workloads.py); the state is resident in HBM before the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "TTN-HEOM steps/sec at trace-dist<=1e-6, mixed/batched vs FP64; % MFMA peak"
PEAK_FP32_MFMA = 157.3  # TFLOP/s, MI355X dense FP32 matrix
PEAK_FP64_MFMA = 78.6
COPY_PROBE_BYTES = 256 << 20
# HBM traffic of the contraction kernel on the default workload (512-instance
# batch, default tile size): rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch
# (KiB), each scaled by what the counter reads for the copy probe of known size.
# Reported only while the kernel sources are the ones the counters were taken on.
HBM_COUNTERS = {
    "sources_sha256": "ab1fc72e5c1b606706ca193afad92c0c4f1c41c153fc9d15182f0ab89c936926",
    "fetch_kib": 9483.8, "write_kib": 7214.4, "fetch_scale": 2.000, "write_scale": 1.000,
}
KERNEL_SOURCES = ("paper_2603_17711_amd/csrc/kernels.hip", "paper_2603_17711_amd/csrc/tenso_internal.h")


def measured_traffic():
    """HBM bytes per contraction-kernel launch, or None if the kernel changed."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != HBM_COUNTERS["sources_sha256"]:
        return None
    c = HBM_COUNTERS
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


WORKLOADS = ["batch512", "spin-boson-train", "exciton-7site", "ps2-structured-ternary",
             "tfd-mctdh", "vmf-mix",
             "surrogate"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch512", choices=WORKLOADS,
                    help="batch512 (default): 512 uneven instances, ps1, batched; "
                         "spin-boson-train, exciton-7site: single ps1 instances; "
                         "ps2-structured-ternary: ps2 on the structured-bath ternary tree; "
                         "tfd-mctdh: the thermofield ML-MCTDH listing (wavefunction TTN); "
                         "surrogate: the learned-surrogate pipeline")
    ap.add_argument("--instances", type=int, default=512, help="batch size for batch512")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the run, a plain 256 MiB streaming kernel (torch.neg) whose "
                         "HBM counters calibrate FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--timed-only", action="store_true",
                    help="batch512: only the warm-up and one timed call of the mixed batch (for "
                         "hardware-counter runs, where every other pass is too slow)")
    ap.add_argument("--autotune", action="store_true",
                    help="batch512: autotune the apply tile size before timing (default: "
                         "the batch default tile size)")
    return ap.parse_args()


def instance(name, n):
    import workloads
    if name == "spin-boson-train":
        return workloads.spin_boson_train(n_steps=n), "spin-boson K=3 N=10 train R=8 ps1 (dt 0.01)"
    return workloads.exciton_7site(n_steps=n), "7-site exciton K=28 N=8 binary R=16 ps1 (dt 0.1 fs)"


def timed_run(inst, precision, steps, warmup):
    import torch
    from paper_2603_17711_amd import api
    plan = api.build_instance(inst, precision=precision)
    if warmup:
        plan.step(warmup, inst.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(steps, inst.dt, t0=warmup * inst.dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return plan, t1 - t0


def kernel_roofline(inst, precision, steps):
    """Average duration and algorithmic work of the SOP-contraction kernel,
    from HIP events recorded on the launching stream."""
    import ctypes as C
    import torch
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import check, lib
    plan = api.build_instance(inst, precision=precision)
    plan.step(1, inst.dt)
    torch.cuda.synchronize()
    check(lib().tenso_profile(1))
    plan.step(steps, inst.dt)
    torch.cuda.synchronize()
    ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().tenso_profile_stats(C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    check(lib().tenso_profile(0))
    return ms.value, n.value, fl.value, by.value


def cpu_baseline(inst, n_sample):
    """The FP64 oracle on the host, single BLAS thread, n_sample steps."""
    from threadpoolctl import threadpool_limits
    from oracle.run import propagate
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        _, rhos, _, _ = propagate(inst, n_steps=n_sample, every=1)
        t1 = time.perf_counter()
    return n_sample / (t1 - t0), rhos


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def trace_distance(a, b):
    """D(a, b) = 1/2 sum of the singular values of a - b."""
    import numpy as np
    return 0.5 * float(np.sum(np.linalg.svd(np.asarray(a) - np.asarray(b), compute_uv=False)))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_instance_steps(args):
    """Oracle work unit of the all-core CPU baseline: one batch instance, k steps."""
    i, k = args
    import workloads
    from threadpoolctl import threadpool_limits
    from oracle.run import propagate
    inst = workloads.uneven_batch(n_steps=k)[i]
    with threadpool_limits(limits=1):
        propagate(inst, n_steps=k, every=k)
    return i


def batch_cpu_baseline(n_inst, k=2):
    """The FP64 oracle on the host: one thread on a small sample, then every
    core the process may use (one worker process per core, one BLAS thread
    each) on a larger one.  Instances are every 16th of the batch, so the
    sample spans the batch's size range."""
    from multiprocessing import get_context
    from threadpoolctl import threadpool_limits
    import workloads
    from oracle.run import propagate
    ids1 = list(range(0, n_inst, 64))            # 8 instances, 1 thread
    sample = workloads.uneven_batch(n_steps=k)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for i in ids1:
            propagate(sample[i], n_steps=k, every=k)
        t1 = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 15))
    ids = list(range(0, n_inst, 16))             # 32 instances over all cores
    # spawned workers start a fresh interpreter: they never touch the GPU
    with get_context("spawn").Pool(cores) as pool:
        t0 = time.perf_counter()
        list(pool.imap_unordered(_oracle_instance_steps, [(i, k) for i in ids]))
        tn = time.perf_counter() - t0
    return {
        "value": round(len(ids) * k / tn, 4), "unit": "instance-steps/s", "cores": cores,
        "kind": "oracle",
        "sample": f"instances 0, 16, 32, ... ({len(ids)} of {n_inst}) x {k} steps, FP64 NumPy "
                  f"oracle, {cores} worker processes with 1 BLAS thread each",
        "cpu_model": cpu_model(),
        "single_thread_value": round(len(ids1) * k / t1, 4),
        "single_thread_sample": f"instances 0, 64, ... ({len(ids1)}) x {k} steps, 1 thread",
    }


def batch_accuracy(insts, precision, every=5):
    """Trace distance of rho_S of every instance to the stored FP64 oracle
    trajectory (tests/golden/batch512_25.npz, written by a script that calls
    only the oracle): a fresh batch at `precision`, 25 steps, compared at every
    10th step and the final step.  None if the stored file does not match the
    workload."""
    import numpy as np
    import torch
    from paper_2603_17711_amd import api
    from tests.golden.make_golden import batch_rhos, load
    try:
        g = load("batch512_25.npz", insts)
    except (OSError, RuntimeError):
        return None
    n = int(g["steps"][-1])
    b = api.Batch([api.build_instance(i, precision=precision) for i in insts])
    recs = b.step_record(n, [i.dt for i in insts], every)
    flagged = int(b.status().sum())
    del b
    torch.cuda.empty_cache()
    worst, where = 0.0, None
    for j, st in enumerate(g["steps"]):
        if st % 10 and st != n:
            continue
        ref = batch_rhos(g, j)
        for i in range(len(insts)):
            d = trace_distance(recs[j][i], ref[i])
            if not d <= worst:
                worst, where = d, (i, int(st))
    return {"value": worst, "steps": n, "instance": where[0], "at_step": where[1],
            "flagged": flagged,
            "sample": f"every instance ({len(insts)}) at every 10th step and the final step "
                      f"of {n}, against the stored FP64 oracle trajectories"}


def batch_main(a):
    """512 uneven instances advanced together (one launch per phase)."""
    import numpy as np
    import torch
    import workloads
    from paper_2603_17711_amd import api

    insts = workloads.uneven_batch(n_inst=a.instances, n_steps=a.steps + a.warmup)
    dts = [i.dt for i in insts]

    tile_work = {"w": None}

    from paper_2603_17711_amd._lib import TensoError

    def advance(b, n):
        # an instance that goes non-finite or grows 1e6-fold is flagged by the
        # library (ENUMERIC after completing every step); it is excluded from
        # the headline below, not hidden
        try:
            b.step(n, dts)
        except TensoError as e:
            if e.code != "ENUMERIC":
                raise

    def run_batch(precision, steps, warmup, tune=False, repeats=1):
        plans = [api.build_instance(i, precision=precision) for i in insts]
        b = api.Batch(plans)
        if tune:  # untimed set-up: pick the apply tile size for this batch
            tile_work["w"] = b.autotune(dts, trial_steps=2)
        advance(b, warmup)
        times = []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            advance(b, steps)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        return plans, b, times

    log(f"mixed batch: {len(insts)} instances, {a.warmup} warm-up + 3 x {a.steps} timed steps")
    plans, batch, times = run_batch(api.FP32, a.steps, a.warmup, tune=a.autotune,
                                    repeats=1 if a.timed_only else 3)
    dt_mixed = times[0]
    flags = batch.status()
    n_ok = int(len(insts) - flags.sum())
    value = n_ok * a.steps / dt_mixed
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "instance-steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * dt_mixed / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions (fp32 MFMA), f64 master/QR", "data": "synthetic",
        "config": {"workload": f"batch of {len(insts)} uneven spin-boson-type instances "
                               "(M 2-8, K 2-8, N 6-12, R 8-32, binary trees, ps1)",
                   "instances": len(insts), "precision": "mixed",
                   "apply_tile_flops": tile_work["w"] or 64e6,
                   "tile_size": "autotuned" if tile_work["w"] else "default"},
        "repeats": {"values": [round(n_ok * a.steps / t, 2) for t in times],
                    "median": round(float(np.median([n_ok * a.steps / t for t in times])), 2),
                    "note": "value is the first of three back-to-back timed calls of "
                            f"{a.steps} steps on the same batch"},
    }
    if a.timed_only:
        out["note"] = "timed call only (no accuracy, FP64, roofline or CPU passes)"
        print(json.dumps(out))
        return
    rho_mixed = batch.rho()
    flagged = [int(i) for i in np.nonzero(flags)[0]]
    nonfinite = [i for i in flagged if not np.isfinite(rho_mixed[i]).all()]
    trace_off = [i for i, r in enumerate(rho_mixed)
                 if i not in flagged and abs(np.trace(r).real - 1.0) > 1e-3]
    out["diverged_instances"] = {
        "flagged": len(flagged), "non_finite": len(nonfinite),
        "trace_off_by_1e-3": len(trace_off), "indices": (flagged + trace_off)[:32],
        "note": "flagged instances (non-finite, or norm grown 1e6-fold; the library's "
                "ENUMERIC) are excluded from value"}
    del batch, plans
    torch.cuda.empty_cache()
    log("accuracy pass (FP32) against the stored oracle trajectories")
    acc = batch_accuracy(insts, api.FP32)
    if acc is not None:
        out["trace_distance_vs_oracle"] = acc
        if acc["value"] > 1e-6:
            out["accuracy_note"] = "trace distance above the 1e-6 fixed-rank bar"
    log("FP32 batch with three real products per complex product, and its accuracy pass")
    st3 = max(1, a.steps // 2)
    plans3, b3, t3 = run_batch(api.FP32_3M, st3, 1)
    out["fp32_3m_batched_value"] = round(len(insts) * st3 / t3[0], 2)
    del b3, plans3
    torch.cuda.empty_cache()
    acc3 = batch_accuracy(insts, api.FP32_3M)
    if acc3 is not None:
        out["fp32_3m_trace_distance_vs_oracle"] = acc3["value"]
    if not a.no_fp64:
        log("FP64 batch, its accuracy pass and the plain FP64 sample")
        st64 = max(1, a.steps // 4)
        plans64, b64, t64 = run_batch(api.FP64, st64, 1)
        v64 = len(insts) * st64 / t64[0]
        out["fp64_batched_value"] = round(v64, 2)
        out["speedup_vs_fp64_batched"] = round(value / v64, 3)
        del b64, plans64
        torch.cuda.empty_cache()
        acc64 = batch_accuracy(insts, api.FP64)
        if acc64 is not None:
            out["fp64_trace_distance_vs_oracle"] = acc64["value"]
        # plain FP64 GPU path: one instance per call, eager launches (no graph),
        # sequential, on every 16th instance (the sample spans the size range)
        ids, k = list(range(0, len(insts), 16)), 2
        t_plain = 0.0
        for i in ids:
            p = api.build_instance(insts[i], precision=api.FP64)
            p.set_graph(False)
            p.step(1, insts[i].dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p.step(k, insts[i].dt)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
        v_plain = len(ids) * k / t_plain
        out["fp64_plain_value"] = round(v_plain, 2)
        out["fp64_plain_sample"] = (f"every 16th instance ({len(ids)}) x {k} steps, one instance "
                                    "per call, eager launches")
        out["speedup_vs_fp64_plain"] = round(value / v_plain, 2)
        out["speedup_note"] = ("equal accuracy: the FP32 and FP64 batches are both within the "
                               "1e-6 bar of the oracle (trace distances above)")
    log("contraction-kernel roofline pass")
    # contraction-kernel roofline inside the batched step
    import ctypes as C
    from paper_2603_17711_amd._lib import check, lib
    plans = [api.build_instance(i, precision=api.FP32) for i in insts]
    if tile_work["w"]:
        for p in plans:
            p.set_tile_work(tile_work["w"])
    b = api.Batch(plans)
    advance(b, 1)
    torch.cuda.synchronize()
    prof_steps = max(1, min(a.steps, 5))
    check(lib().tenso_profile(1))
    advance(b, prof_steps)
    torch.cuda.synchronize()
    ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().tenso_profile_stats(C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    check(lib().tenso_profile(0))
    avg_ms = ms.value / max(1, n.value)
    achieved = fl.value / max(1, n.value) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = {
        "kernel": "k_apply<float> (SOP contraction, MFMA 16x16x4 f32)",
        "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP32_MFMA,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 6),
        "traffic": None if tile_work["w"] else measured_traffic(),
        "avg_launch_us": round(1e3 * avg_ms, 3), "launches": int(n.value),
        "algorithmic_flops_per_launch": fl.value / max(1, n.value),
        "algorithmic_bytes_per_launch": by.value / max(1, n.value),
        "apply_share_of_step": round(ms.value / prof_steps / (1e3 * dt_mixed / a.steps), 4),
    }
    del b, plans
    if not a.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = batch_cpu_baseline(a.instances)
    print(json.dumps(out))


def copy_probe():
    """Known-size streaming kernel: reads and writes COPY_PROBE_BYTES each."""
    import torch
    x = torch.ones(COPY_PROBE_BYTES // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.neg(x, out=y)
    torch.cuda.synchronize()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    run_main(a)
    if a.copy_probe:
        copy_probe()


def ps2_main(a):
    """Adaptive-rank (ps2) propagation of the structured-bath ternary tree at rank
    cap 8 with eps 1e-6 (the ranks grow from 2 and eps decides them), one
    instance."""
    import ctypes as C
    import numpy as np
    import torch
    import workloads
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import check, lib
    cap = 8
    inst = workloads.structured_bath_ternary(n_steps=a.steps + a.warmup)
    wname = f"structured bath K=24 N=10 ternary ps2 (eps 1e-6, rank cap {cap}, dt 0.01)"

    def run(precision, steps, warmup, profile=False):
        plan = api.build_instance(inst, precision=precision, rank=cap)
        plan.step_adaptive(warmup, inst.dt, inst.eps, cap)
        torch.cuda.synchronize()
        if profile:
            check(lib().tenso_profile(1))
        t0 = time.perf_counter()
        plan.step_adaptive(steps, inst.dt, inst.eps, cap, t0=warmup * inst.dt)
        torch.cuda.synchronize()
        return plan, time.perf_counter() - t0

    log(f"ps2 mixed: {a.warmup} warm-up + {a.steps} timed steps at cap {cap}")
    plan, dt_mixed = run(api.FP32, a.steps, a.warmup)
    value = a.steps / dt_mixed
    ranks = plan.rank_log()
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * dt_mixed / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions (fp32 MFMA), f64 master/QR/SVD", "data": "synthetic",
        "config": {"workload": wname, "instances": 1, "precision": "mixed",
                   "max_rank_reached": int(max(ranks)), "ranks_last_step": ranks},
    }
    if not a.no_fp64:
        log("ps2 FP64 path over the same steps")
        # the same steps as the mixed run: the cost of a ps2 step grows with the ranks
        _, dt64 = run(api.FP64, a.steps, a.warmup)
        out["fp64_gpu_value"] = round(a.steps / dt64, 3)
        out["speedup_vs_fp64_gpu"] = round(value / (a.steps / dt64), 3)
    log("contraction-kernel roofline pass")
    prof_steps = max(1, min(a.steps, 5))
    _, _ = run(api.FP32, prof_steps, 1, profile=True)
    ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().tenso_profile_stats(C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    check(lib().tenso_profile(0))
    avg_ms = ms.value / max(1, n.value)
    achieved = fl.value / max(1, n.value) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = {
        "kernel": "k_apply<float> (SOP contraction, MFMA 16x16x4 f32)",
        "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP32_MFMA,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 6), "traffic": None,
        "avg_launch_us": round(1e3 * avg_ms, 3), "launches": int(n.value),
        "algorithmic_flops_per_launch": fl.value / max(1, n.value),
        "algorithmic_bytes_per_launch": by.value / max(1, n.value),
    }
    # accuracy: a fresh run against the stored oracle trajectory (10 steps)
    try:
        from tests.golden.make_golden import load
        g = load("ps2_ternary_cap8_10.npz", [workloads.structured_bath_ternary(n_steps=10)])
    except (OSError, RuntimeError):
        g = None
    if g is not None:
        log("accuracy pass against the stored oracle trajectory")
        cinst = workloads.structured_bath_ternary(n_steps=10)
        p2 = api.build_instance(cinst, precision=api.FP32, rank=cap)
        dmax = 0.0
        for k in range(10):
            p2.step_adaptive(1, cinst.dt, cinst.eps, cap, t0=k * cinst.dt)
            dmax = max(dmax, trace_distance(p2.rho(), g["rho"][k + 1]))
        out["trace_distance_vs_oracle"] = {
            "value": dmax, "steps": 10,
            "sample": "every step of 10, against the stored FP64 oracle trajectory (adaptive bar 1e-5)"}
    if not a.no_cpu:
        log("CPU oracle baseline")
        from threadpoolctl import threadpool_limits
        from oracle.run import propagate
        n_sample = 2
        cinst = workloads.structured_bath_ternary(n_steps=n_sample)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            propagate(cinst, n_steps=n_sample, every=n_sample, max_rank=cap)
            tc = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n_sample / tc, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {n_sample} ps2 steps of the same workload (ranks lowest there), "
                      "FP64 NumPy oracle, 1 BLAS thread", "cpu_model": cpu_model()}
    print(json.dumps(out))


def surrogate_main(a):
    """The surrogate pipeline (driven spin-boson trajectories) at a bounded size: TTN-HEOM trajectories
    on training seeds, BF16 MLP training, monitored rollout on held-out seeds,
    TTN fallback for tripped trajectories, judged against TTN-HEOM."""
    from paper_2603_17711_amd import surrogate
    n_train, n_held, n_steps, epochs = 1536, 64, 1000, 60
    res = surrogate.experiment(n_train, n_held, n_steps=n_steps, epochs=epochs, log=lambda *x: None)
    value = n_held * n_steps / res["surrogate_s"]
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "trajectory-steps/s (surrogate)",
        "n_gpus": 1, "steps": n_steps, "warmup": 0,
        "ms_per_step": round(1e3 * res["surrogate_s"] / n_steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MLP (fp32 accumulate); c64/f64 TTN fallback", "data": "synthetic",
        "config": {"workload": f"driven spin-boson surrogate: {n_train} training and {n_held} "
                               f"held-out trajectories x {n_steps} steps, {epochs} epochs",
                   "instances": n_held, "precision": "mixed"},
        "ttn_batched_value": round(n_held * n_steps / res["ttn_heldout_s"], 2),
        "gain_vs_ttn_batched": round(res["gain"], 3),
        "monitor_trips": res["monitor_trips"],
        "spot_checked": res["spot_checked"], "spot_trips": res["spot_trips"],
        "max_feature_error_vs_ttn": res["max_feature_error"],
        "median_feature_error_vs_ttn": res["median_feature_error"],
        "train_s": round(res["train_s"], 3), "train_mse_first_last": res["train_mse_first_last"],
        "roofline": None,
    }
    print(json.dumps(out))


def tfd_main(a):
    """The thermofield ML-MCTDH listing (Sec. III A 5): 50 star modes of Fock
    dimension 8 on a binary tree of rank 16, a wavefunction under -iH, ps1 with
    1 fs steps; one instance."""
    import ctypes as C
    import torch
    import workloads
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import check, lib
    from paper_2603_17711_amd.mctdh import build_tfd
    inst = workloads.tfd_spin_boson()

    def timed(precision, steps, warmup):
        plan = build_tfd(inst, precision=precision)
        plan.step(warmup, inst.dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(steps, inst.dt, t0=warmup * inst.dt)
        torch.cuda.synchronize()
        return plan, time.perf_counter() - t0

    log("thermofield: timed FP32 run")
    _, dt_mixed = timed(api.FP32, a.steps, a.warmup)
    value = a.steps / dt_mixed
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * dt_mixed / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions (fp32 MFMA), f64 master/QR", "data": "synthetic",
        "config": {"workload": inst.name + ", -iH on a wavefunction, ps1, 1 fs steps",
                   "instances": 1, "precision": "mixed"},
    }
    if not a.no_fp64:
        _, dt64 = timed(api.FP64, max(1, a.steps // 2), 2)
        out["fp64_gpu_value"] = round(max(1, a.steps // 2) / dt64, 3)
    # accuracy: 100 steps against the stored oracle trajectory
    from tests.golden.make_golden import load
    g = load("tfd_spin_boson_100.npz", [inst])
    plan = build_tfd(inst, precision=api.FP32)
    dmax = trace_distance(plan.rho_pure(), g["rho"][0])
    for k in range(1, 11):
        plan.step(10, inst.dt, t0=10 * (k - 1) * inst.dt)
        dmax = max(dmax, trace_distance(plan.rho_pure(), g["rho"][k]))
    out["trace_distance_vs_oracle"] = {"value": dmax, "steps": 100,
                                       "sample": "every 10th step against the stored oracle"}
    prof_steps = max(1, min(a.steps, 10))
    plan = build_tfd(inst, precision=api.FP32)
    plan.step(1, inst.dt)
    torch.cuda.synchronize()
    check(lib().tenso_profile(1))
    plan.step(prof_steps, inst.dt)
    torch.cuda.synchronize()
    ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().tenso_profile_stats(C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    check(lib().tenso_profile(0))
    avg_ms = ms.value / max(1, n.value)
    achieved = fl.value / max(1, n.value) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = {
        "kernel": "k_apply<float> (SOP contraction, MFMA 16x16x4 f32)",
        "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP32_MFMA,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 6), "traffic": None,
        "avg_launch_us": round(1e3 * avg_ms, 3), "launches": int(n.value),
        "algorithmic_flops_per_launch": fl.value / max(1, n.value),
        "algorithmic_bytes_per_launch": by.value / max(1, n.value),
    }
    if not a.no_cpu:
        from threadpoolctl import threadpool_limits
        from oracle.tfd import propagate_tfd
        n_sample = 5
        log("thermofield: CPU oracle baseline")
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            propagate_tfd(inst, n_steps=n_sample, every=n_sample)
            t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n_sample / t_cpu, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} steps of the same workload, FP64 NumPy oracle, 1 BLAS thread",
        }
    print(json.dumps(out))


def vmf_main(a):
    """The spin-boson train under the mixed strategy (Sec. VI, Sec. VII E): ps2
    (eps 1e-8) from rank 2 until a bond reaches rank 8, then direct (vmf)
    integration with adaptive dopri5, all FP64; value = output steps per second
    of the vmf phase (dt = 0.01 per step)."""
    import ctypes as C
    import torch
    import workloads
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import check, lib
    inst = workloads.spin_boson_train_mix()
    dt, eps, cap = inst.dt, inst.eps, inst.rank

    def to_vmf(extra):
        plan = api.build_instance(inst, precision=api.FP64)
        s, sw = 0, -1
        while sw < 0:
            sw = plan.step_mix(1, dt, eps, cap, t0=s * dt)
            s += 1
        if extra:
            plan.step_mix(extra, dt, eps, cap, t0=s * dt)
        return plan, s + extra, sw

    log("vmf: ps2 phase, then timed vmf steps")
    plan, s0, sw = to_vmf(a.warmup)
    acc0, rej0, _ = plan.vmf_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step_mix(a.steps, dt, eps, cap, t0=s0 * dt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    acc1, rej1, h = plan.vmf_stats()
    out = {
        "metric": METRIC, "value": round(a.steps / el, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * el / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 (contractions on FP64 MFMA)", "data": "synthetic",
        "config": {"workload": inst.name + " (dopri5 rtol 1e-5, atol 1e-7; shift 1e-7)",
                   "instances": 1, "precision": "fp64", "ps2_steps_before_switch": sw,
                   "substeps_per_step": round((acc1 + rej1 - acc0 - rej0) / a.steps, 3)},
    }
    # accuracy: 100 steps against the stored oracle trajectory
    from tests.golden.make_golden import load
    g = load("mix_spin_boson_train_100.npz", [inst])
    plan = api.build_instance(inst, precision=api.FP64)
    dmax = trace_distance(plan.rho(), g["rho"][0])
    for k in range(1, 11):
        sw2 = plan.step_mix(10, dt, eps, cap, t0=10 * (k - 1) * dt)
        dmax = max(dmax, trace_distance(plan.rho(), g["rho"][k]))
    acc, rej, _ = plan.vmf_stats()
    out["trace_distance_vs_oracle"] = {
        "value": dmax, "steps": 100, "switch": [sw2, int(g["switch"])],
        "substeps": [[acc, rej], [int(g["accepted"]), int(g["rejected"])]],
        "sample": "every 10th step against the stored oracle trajectory (switch step and "
                  "accepted / rejected substeps: library, oracle)"}
    # contraction kernel inside the vmf derivative
    prof = max(1, min(a.steps, 10))
    plan, s0, _ = to_vmf(1)
    torch.cuda.synchronize()
    check(lib().tenso_profile(1))
    plan.step_mix(prof, dt, eps, cap, t0=s0 * dt)
    torch.cuda.synchronize()
    ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check(lib().tenso_profile_stats(C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    check(lib().tenso_profile(0))
    avg_ms = ms.value / max(1, n.value)
    achieved = fl.value / max(1, n.value) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = {
        "kernel": "k_apply<double> (SOP contraction of every node, MFMA 16x16x4 f64)",
        "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP64_MFMA,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_MFMA, 6), "traffic": None,
        "avg_launch_us": round(1e3 * avg_ms, 3), "launches": int(n.value),
        "algorithmic_flops_per_launch": fl.value / max(1, n.value),
        "algorithmic_bytes_per_launch": by.value / max(1, n.value),
    }
    if not a.no_cpu:
        import copy
        from threadpoolctl import threadpool_limits
        from oracle.integrators import Propagator
        from oracle.run import build
        from oracle.ttn import initial_state
        from oracle.vmf import VmfPropagator
        log("vmf: CPU oracle baseline")
        terms, tree = build(inst)
        tree = copy.deepcopy(tree)
        with threadpool_limits(limits=1):
            P = Propagator(tree, terms, initial_state(tree, inst.rho0))
            k = 0
            while max(tree.rank[1:]) < cap:
                P.step_ps2(k * dt, dt, eps, cap)
                k += 1
            V = VmfPropagator(tree, terms, P.C)
            n_sample = 20
            t0 = time.perf_counter()
            for j in range(n_sample):
                V.step((k + j) * dt, dt)
            t_cpu = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": round(n_sample / t_cpu, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} vmf steps after the switch, FP64 NumPy oracle, 1 BLAS thread",
        }
    print(json.dumps(out))


def run_main(a):
    import numpy as np
    import torch
    torch.cuda.set_device(0)
    from paper_2603_17711_amd import api
    if a.workload == "batch512":
        return batch_main(a)
    if a.workload == "ps2-structured-ternary":
        return ps2_main(a)
    if a.workload == "surrogate":
        return surrogate_main(a)
    if a.workload == "vmf-mix":
        return vmf_main(a)
    if a.workload == "tfd-mctdh":
        return tfd_main(a)

    inst, wname = instance(a.workload, a.steps + a.warmup)
    plan, dt_mixed = timed_run(inst, api.FP32, a.steps, a.warmup)
    value = a.steps / dt_mixed
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(1e3 * dt_mixed / a.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 contractions (fp32 MFMA), f64 master/QR", "data": "synthetic",
        "config": {"workload": wname, "instances": 1, "precision": "mixed"},
    }
    if not a.no_fp64:
        _, dt64 = timed_run(inst, api.FP64, max(1, a.steps // 2), 2)
        v64 = max(1, a.steps // 2) / dt64
        out["fp64_gpu_value"] = round(v64, 3)
        out["speedup_vs_fp64_gpu"] = round(value / v64, 3)
    prof_steps = max(1, min(a.steps, 20))
    ms, n, fl, by = kernel_roofline(inst, api.FP32, prof_steps)
    avg_ms = ms / max(1, n)
    achieved = fl / max(1, n) / (avg_ms * 1e-3) / 1e12
    out["roofline"] = {
        "kernel": "k_apply<float> (SOP contraction, MFMA 16x16x4 f32)",
        "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_FP32_MFMA,
        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA, 6), "traffic": None,
        "avg_launch_us": round(1e3 * avg_ms, 3), "launches": int(n),
        "algorithmic_flops_per_launch": fl / max(1, n),
        "algorithmic_bytes_per_launch": by / max(1, n),
        "apply_share_of_step": round(ms / prof_steps / (1e3 * dt_mixed / a.steps), 4),
    }
    if not a.no_cpu:
        n_sample = 3 if a.workload == "exciton-7site" else 400
        cinst, _ = instance(a.workload, n_sample)
        v_cpu, rhos_cpu = cpu_baseline(cinst, n_sample)
        out["cpu_baseline"] = {
            "value": round(v_cpu, 4), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_sample} steps of the same workload, FP64 NumPy oracle, 1 BLAS thread",
        }
        # accuracy of the mixed path on the sample horizon
        p2 = api.build_instance(cinst, precision=api.FP32)
        dmax = 0.0
        for k in range(1, n_sample + 1):
            p2.step(1, cinst.dt, t0=(k - 1) * cinst.dt)
            if k % 10 == 0 or k == n_sample:
                dmax = max(dmax, trace_distance(p2.rho(), rhos_cpu[k]))
        out["trace_distance_vs_oracle"] = {"value": dmax, "steps": n_sample}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
