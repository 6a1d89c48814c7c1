"""Benchmark of the discrete-HMM bank on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the recognition path over one batch: the length-sorted
plan, the batched MFMA forward over every (sequence, model) pair, and the
arg-max over models (hmm_classify), on the 64-model bank (N=32 states, M=256
symbols) and 65,536 ragged sequences (log-uniform lengths in [16, 2048]) with
inputs resident in HBM.  The metric is state-steps/s = N^2 * sum(T) * models /
time.  Printed as one JSON line, with:
  roofline      the batched forward kernel's own HIP-event time against the
                FP32 MFMA peak (2 algorithmic FLOPs per state-step);
  cpu_baseline  the FP64 oracle on the host cores, on a stratified sample of the
                same workload, in the same unit;
  plain         the plain per-pair kernel on the same workload (batched / plain speedup);
  fwd_bwd       forward + adjoint (expected counts) on the gradient workload
                (8 models, N=64, M=512, 8192 sequences, T in [100, 1000]),
                6 algorithmic FLOPs per state-step, with alpha checkpointed
                every ceil(sqrt(T)) steps as that configuration states
                (`storage`); `every_step` times the same call with the scaled
                alpha of every step stored between the passes;
  large_states  the N=256 bank (16 models, M=1024, 16,384 sequences, T in
                [256, 4096], own model): forward, and forward + adjoint with
                every step stored when the device has room (38 GB of
                workspace) and the checkpoint storage timed beside it, on the
                cooperative kernels, and Viterbi decoding on the workgroup
                decoder;
  latency       the small workloads, whose time is the serial chain of steps
                (c1: one sequence of 64 steps; c2: 4096 sequences x 12 models,
                T up to 400, with labels): microseconds per call, eager and as a
                replayed HIP graph;
  graph         the recognition step captured once as a HIP graph and replayed;
  viterbi       Viterbi decoding of the c3 sequences, each with its owner model
                (max-plus on the vector ALUs: 2 operations per state-step, over
                the decoder and traceback kernels, against the FP32 vector issue
                rate without packing, 39.3 Tops/s);
  em            one Baum-Welch iteration on c4 (forward + adjoint + M-step);
  tuning        per leg, the kernel family and workgroups-per-CU cap the
                autotuner installed before the leg was timed, with the default
                choice's time and the tuned time.

Every leg is autotuned before it is timed (paper_1310_3322_amd.tune: each
candidate is checked against the default choice's outputs); --tune-cache FILE
installs the choices stored there instead of tuning again and stores new ones,
--no-tune keeps the built-in heuristics.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HMM state-steps/s (N²·ΣT·models) fwd and fwd+bwd, batched vs plain, FP32"
FP32_PEAK_TFLOPS = 157.3
# vector ALU issue rate for single (unpacked) FP32 operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_TOPS = 39.3
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# The kernel the recognition workload (N=32, all pairs) runs in each forward
# family, and the files its code comes from: counters taken on a kernel are
# valid while these files and the compile flags in build.py are unchanged.
_COMMON = ["paper_1310_3322_amd/csrc/common.cuh", "paper_1310_3322_amd/csrc/kernels.h", "paper_1310_3322_amd/build.py"]
FAMILY_KERNELS = {
    "tile32": ("k_fwd_mfma32<1, true>", "32-sequence-tile batched forward",
               ["paper_1310_3322_amd/csrc/fwd_mfma32.hip"] + _COMMON),
    "tile16": ("k_fwd_mfma<2, true, false>", "16-sequence-tile batched forward",
               ["paper_1310_3322_amd/csrc/fwd_mfma.hip"] + _COMMON),
}
# The kernels whose HBM traffic profiles/traffic.json records, by workload: the
# kernel as rocprofv3 names it and the files its code comes from.
_FWD_COOP = ["paper_1310_3322_amd/csrc/fwd_coop.hip", "paper_1310_3322_amd/csrc/coop_step.cuh"] + _COMMON
_ADJ_COOP = ["paper_1310_3322_amd/csrc/adj_coop.hip", "paper_1310_3322_amd/csrc/coop_step.cuh"] + _COMMON
TRAFFIC_KERNELS = {
    "c3_classify": ("k_fwd_mfma32<1, true>", FAMILY_KERNELS["tile32"][2]),
    "c4_grad_forward": ("k_fwd_coop<4, 1, true>", _FWD_COOP),
    "c4_grad_adjoint": ("k_adj_pipe<4>", _ADJ_COOP),
    "c5_forward": ("k_fwd_coop<16, 2, false>", _FWD_COOP),
    "c5_grad_forward": ("k_fwd_coop<16, 2, true>", _FWD_COOP),
    "c5_grad_adjoint": ("k_adj_coop<16, 2, false, true, true>", _ADJ_COOP),
    "c5_grad_counts": ("k_grows_reduce", _ADJ_COOP),
}
# The bench leg whose tuned choice (kernel family, workgroups-per-CU cap, flags)
# launched each recorded kernel: a figure holds only for the choice it was taken on.
TRAFFIC_LEGS = {"c3_classify": "c3_classify", "c4_grad_forward": "c4_grad", "c4_grad_adjoint": "c4_grad",
                "c5_forward": "c5_forward", "c5_grad_forward": "c5_grad", "c5_grad_adjoint": "c5_grad",
                "c5_grad_counts": "c5_grad"}
DEFAULT_CHOICE = {"kernel": "auto", "wg_per_cu": 0, "flags": 0}


def leg_choice(tuning: dict, leg: str) -> dict:
    """The choice a leg ran with: its tuned one, else the library's heuristics."""
    c = (tuning or {}).get(leg, {}).get("choice")
    return {k: c.get(k, 0) for k in DEFAULT_CHOICE} if c else dict(DEFAULT_CHOICE)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_source_hash(family: str = "tile32") -> str:
    return source_hash(FAMILY_KERNELS[family][2])


def measured_traffic(workload: str, choice: dict, family: str = None, path: str = TRAFFIC_FILE):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    holds a record taken on the workload's kernel (for c3: the family's kernel)
    with the current source and the same tuned choice; else None."""
    try:
        with open(path) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    if family is not None:
        if family not in FAMILY_KERNELS:
            return None
        kernel, files = FAMILY_KERNELS[family][0], FAMILY_KERNELS[family][2]
    elif workload in TRAFFIC_KERNELS:
        kernel, files = TRAFFIC_KERNELS[workload]
    else:
        return None
    h = source_hash(files)
    recs = data.get(workload)
    for rec in recs if isinstance(recs, list) else []:
        if isinstance(rec, dict) and rec.get("kernel") == kernel and rec.get("kernel_source_hash") == h and rec.get("choice") == choice:
            return rec.get("bytes_per_launch")
    return None


def traffic_summary(fetch_csv: str, write_csv: str, bench_out: str, out: str = TRAFFIC_FILE):
    """Records in profiles/traffic.json from two rocprofv3 --pmc runs of the same
    command (FETCH_SIZE, then WRITE_SIZE; counter_collection.csv of each, values
    in KiB per dispatch) that include --copy-calibration: the counters of the
    512 MiB device copies give the scale from counter to bytes; per kernel the
    average over its dispatches, scaled.  `bench_out` is the output of one of
    those runs (its JSON line names the tuned choice each leg ran with, which
    the record keeps).  Per workload the file holds one record per choice:
    a new record replaces the one of the same choice, and records taken on
    other source are dropped."""
    import csv

    tuning = {}
    with open(bench_out) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{"):
                tuning = json.loads(line).get("tuning", {})

    def per_kernel(path, counter):
        acc = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                a = acc.setdefault(r["Kernel_Name"], [])
                a.append(float(r["Counter_Value"]) * 1024.0)
        return acc

    fetch, write = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    copy_bytes = 512 << 20

    def calib(acc):  # the copies of 512 MiB: dispatches of the copy kernel that moved over 256 MiB
        vals = [v for name, vs in acc.items() if "copyBuffer" in name for v in vs if v > (256 << 20) * 0.4]
        if not vals:
            raise SystemExit("no 512 MiB copy dispatches in the counters (run the bench with --copy-calibration)")
        return float(np.mean(vals)), copy_bytes / float(np.mean(vals))

    fraw, fscale = calib(fetch)
    wraw, wscale = calib(write)

    def find(acc, kernel):
        hits = [vs for name, vs in acc.items() if ("::" + kernel + "(") in name]
        return hits[0] if len(hits) == 1 else None

    try:
        with open(out) as fh:
            old = json.load(fh)
    except (OSError, ValueError):
        old = {}
    data, new = {}, {}
    for wl, (kernel, files) in TRAFFIC_KERNELS.items():
        h = source_hash(files)
        choice = leg_choice(tuning, TRAFFIC_LEGS[wl])
        kept = [r for r in (old.get(wl) if isinstance(old.get(wl), list) else [])
                if r.get("kernel") == kernel and r.get("kernel_source_hash") == h]
        fv, wv = find(fetch, kernel), find(write, kernel)
        if fv is None or wv is None:
            if kept:
                data[wl] = kept
            continue
        fb, wb = float(np.mean(fv)) * fscale, float(np.mean(wv)) * wscale
        new[wl] = {"kernel": kernel, "kernel_source_hash": h, "choice": choice,
                   "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "bytes_per_launch": fb + wb,
                   "fetch_scale": fscale, "write_scale": wscale,
                   "calibration": f"__amd_rocclr_copyBuffer of 512 MiB: FETCH_SIZE {fraw / 1024:.1f} KiB, "
                                  f"WRITE_SIZE {wraw / 1024:.1f} KiB per dispatch",
                   "launches": min(len(fv), len(wv))}
        data[wl] = [r for r in kept if r.get("choice") != choice] + [new[wl]]
    with open(out, "w") as fh:
        json.dump(data, fh, indent=1)
        fh.write("\n")
    print(json.dumps({k: round(v["bytes_per_launch"] / 1e9, 4) for k, v in new.items()}))


def traffic_fields(kernels, tuning):
    """{name: (traffic workload, kernel ms)} -> HBM bytes per launch from the committed counter
    summary (None when it was taken on other code or another tuned choice) and the rate they
    give at that kernel time."""
    out = {}
    for name, (wl, ms) in kernels.items():
        b = measured_traffic(wl, leg_choice(tuning, TRAFFIC_LEGS[wl]))
        out[name] = {"kernel": TRAFFIC_KERNELS[wl][0], "hbm_bytes_per_launch": b,
                     "hbm_gbs": round(b / (ms / 1e3) / 1e9, 1) if b and ms > 0 else None}
    return out


def to_dev(w, torch, own):
    from paper_1310_3322_amd import hmm

    def d(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    return hmm.Problem(d(w.pi), d(w.A), d(w.B), d(w.symbols), d(w.offsets), d(w.lengths),
                       d(w.owner) if own else None, max_len=w.max_len, total_symbols=w.total_symbols)


def grad_rows(p, w, torch) -> int:
    """Scaled-alpha rows the gradient legs store: every step of the workload when that
    workspace fits the device's free memory with 2 GiB to spare, else none (checkpoints)."""
    free, _ = torch.cuda.mem_get_info()
    return w.total_symbols if p.grad_workspace_size(w.total_symbols) + (2 << 30) <= free else 0


def time_grad_storage(p, rows, reps, torch):
    """ms per gradient call and per forward / adjoint kernel with `rows` stored steps."""
    from paper_1310_3322_amd import hmm

    ws = p.grad_workspace(rows)
    ll, cnt, _ = hmm.forward_backward_grad(p, ws=ws)
    torch.cuda.synchronize()
    hmm.profile_enable(True)
    sec = time_steps(lambda: hmm.forward_backward_grad(p, loglik=ll, counts=cnt, ws=ws), reps, 0, torch)
    f_ms, f_n = hmm.profile_read(hmm.PROF_FWD_BATCHED)
    a_ms, a_n = hmm.profile_read(hmm.PROF_ADJ_BATCHED)
    hmm.profile_enable(False)
    return {"ms_per_step": sec * 1e3, "fwd_kernel_ms": f_ms / max(f_n, 1), "adj_kernel_ms": a_ms / max(a_n, 1),
            "workspace_bytes": ws.numel()}


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / max(steps, 1)


def graph_stats(fn, reps, torch, batch=1):
    """`batch` consecutive calls of fn captured once as a HIP graph and replayed: 3 warm-up
    replays, then `reps` replays each bracketed by its own events on the stream; milliseconds
    per call (median, min, mean of the replays, divided by `batch`)."""
    fn()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(batch):
            fn()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        g.replay()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev]) / batch
    # the same replays back to back (throughput: the launches overlap as eager calls do)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    b2b = (time.perf_counter() - t0) / reps / batch * 1e3
    return {"median_ms": float(np.median(t)), "min_ms": float(np.min(t)), "mean_ms": float(np.mean(t)),
            "back_to_back_ms": b2b, "replays": reps, "calls_per_graph": batch}


def graph_floor_us(torch, reps=200):
    """Back-to-back cost of replaying a graph of one trivial kernel against launching that
    kernel eagerly: the runtime's own cost per graph launch, in microseconds."""
    x = torch.zeros(64, device="cuda")
    f = lambda: x.add_(1.0)
    g = torch.cuda.CUDAGraph()
    f()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        f()

    def b2b(fn):
        for _ in range(10):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6
    return {"graph_of_one_kernel_us": b2b(g.replay), "eager_kernel_us": b2b(f)}


def eager_stats(fn, reps, torch):
    """Milliseconds per eager call on the stream (median, min, mean of `reps` calls, each
    bracketed by its own events, after 3 warm-up calls)."""
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median_ms": float(np.median(t)), "min_ms": float(np.min(t)), "mean_ms": float(np.mean(t)),
            "calls": reps}


def h2d_copy(w, torch):
    """The host-to-device term of a call (the CPU-GPU transfer of the paper's cost model,
    Eq. 1): the bank and the batch copied from pinned host memory to HBM, timed with
    events on the stream (median of 5 copies)."""
    host = [torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
            for a in (w.pi, w.A, w.B, w.symbols, w.offsets, w.lengths)]
    devs = [torch.empty_like(h, device="cuda") for h in host]
    nbytes = sum(h.numel() * h.element_size() for h in host)
    times = []
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for h, d in zip(host, devs):
            d.copy_(h, non_blocking=True)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times[1:]))
    return {"bytes": int(nbytes), "ms": ms, "GB_per_s": nbytes / (ms / 1e3) / 1e9}


def cpu_oracle_counts(w, target_s: float = 5.0):
    """FP64 oracle forward + backward (expected counts) on every stride-th sequence in length order."""
    from oracle import oracle as O
    order = np.argsort(-w.lengths, kind="stable")
    probe = w.subset(order[::256])
    t0 = time.perf_counter()
    O.counts(probe.pi, probe.A, probe.B, probe.symbols, probe.offsets, probe.lengths, probe.owner)
    dt = max(time.perf_counter() - t0, 1e-3)
    stride = int(np.clip(np.ceil(w.units() / (probe.units() / dt * target_s)), 1, 256))
    sample = w.subset(order[::stride])
    t0 = time.perf_counter()
    O.counts(sample.pi, sample.A, sample.B, sample.symbols, sample.offsets, sample.lengths, sample.owner)
    dt = time.perf_counter() - t0
    return {"value": sample.units() / dt, "unit": "state-steps/s", "cores": O.max_threads(), "kind": "oracle",
            "sample": f"one sequence in {stride} in length order ({sample.S} of {w.S}), own model, "
                      f"{sample.units():.3e} state-steps in {dt:.1f} s, FP64 forward + backward counts"}


def cpu_baseline(w, target_s: float = 15.0):
    """FP64 oracle on a stratified sample: every stride-th sequence in length order, all models."""
    from oracle import oracle as O
    order = np.argsort(-w.lengths, kind="stable")
    threads = O.max_threads()
    # calibrate on a small sample, then size the sample to about target_s seconds
    probe = w.subset(order[::1024])
    t0 = time.perf_counter()
    O.forward(probe.pi, probe.A, probe.B, probe.symbols, probe.offsets, probe.lengths, None)
    dt = max(time.perf_counter() - t0, 1e-3)
    rate = probe.units() / dt
    stride = int(np.clip(np.ceil(w.units() / (rate * target_s)), 1, 1024))
    sample = w.subset(order[::stride])
    t0 = time.perf_counter()
    O.forward(sample.pi, sample.A, sample.B, sample.symbols, sample.offsets, sample.lengths, None)
    dt = time.perf_counter() - t0
    return {"value": sample.units() / dt, "unit": "state-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"one sequence in {stride} in length order ({sample.S} of {w.S}) x all {w.K} models, "
                      f"{sample.units():.3e} state-steps in {dt:.1f} s, FP64, OpenMP over pairs"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip every leg but the recognition step")
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs after the recognition step: plain, grad (c4 forward + adjoint), "
                         "large (c5 forward and forward + adjoint), large_viterbi (c5 Viterbi), latency (c1, c2), "
                         "viterbi (c3 Viterbi), em, graph, h2d; default all")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run 4 device copies of 512 MiB (reference kernel for HBM counter scaling)")
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in kernel heuristics (no autotuning)")
    ap.add_argument("--no-storage-compare", action="store_true",
                    help="skip the gradient legs' second timing with checkpoints (profiled runs: the kernels of "
                         "both storages have the same names)")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON tuning cache: install the choices stored there instead of tuning, store new ones")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "BENCH_JSON"), default=None,
                    help="write profiles/traffic.json from the counter_collection.csv files of a FETCH_SIZE "
                         "and a WRITE_SIZE rocprofv3 run of this bench (with --copy-calibration and the "
                         "--tune-cache of the bench run whose output line BENCH_JSON holds) and exit")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    legs = {"plain", "grad", "large", "large_viterbi", "latency", "viterbi", "em", "graph", "h2d"}
    chosen = set() if args.no_extra else (legs if args.legs == "all" else set(args.legs.split(",")))
    if chosen - legs:
        print(f"unknown legs: {sorted(chosen - legs)}", file=sys.stderr)
        sys.exit(2)

    def want(leg):
        return leg in chosen

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (sequences would be "
              "sharded over GPUs, each running the same launch on its share).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1310_3322_amd import hmm, tune, workloads

    torch.cuda.set_device(0)
    hmm.load_library()
    hmm.select_kernel(hmm.KERNEL_AUTO)
    tuning, tuned_now = {}, []
    if args.tune_cache and os.path.exists(args.tune_cache) and not args.no_tune:
        log(f"installed {tune.load_cache(args.tune_cache)} tuning entries from {args.tune_cache}")

    def autotune(name, p, op, **kw):
        """Tunes the calls of `op` on p's shape before they are timed (or takes the cached choice)."""
        if args.no_tune:
            return
        b = p.batch_without_models() if op == hmm.OP_CLASSIFY else p.batch
        got = hmm.tune_get(hmm.tune_key(p.bank, b, op)) if args.tune_cache else None
        if got is not None:
            tuning[name] = {"choice": {"kernel": tune.KERNEL_NAMES[got[0]], "wg_per_cu": got[1], "flags": got[2]},
                            "source": "cache"}
            return
        log(f"autotuning {name}")
        r = tune.tune(p, op, **kw)
        tuned_now.append(r)
        tuning[name] = {"choice": r["choice"], "tuned_ms": round(r["ms"], 4), "default_ms": round(r["default_ms"], 4),
                        "accepted": sum(1 for c in r["candidates"] if c["ok"]),
                        "unsupported": sum(1 for c in r["candidates"] if c["reason"] == "unsupported"),
                        "rejected": [c for c in r["candidates"] if not c["ok"] and c["reason"] != "unsupported"]}

    log("generating the recognition workload (64 models, N=32, M=256, 65536 sequences)")
    w = workloads.make_workload("c3")
    units = w.units()
    p = to_dev(w, torch, own=False)
    b = p.batch_without_models()
    autotune("c3_classify", p, hmm.OP_CLASSIFY)
    family = tune.KERNEL_NAMES[hmm.call_kernel(p.bank, b, hmm.OP_CLASSIFY)]
    ws = p.workspace(hmm.OP_CLASSIFY, b)
    labels = torch.empty(w.S, dtype=torch.int32, device="cuda")
    ll = torch.empty((w.S, w.K), dtype=torch.float32, device="cuda")

    def step():
        hmm.classify(p, labels=labels, loglik=ll, ws=ws)

    log(f"timing {args.steps} steps after {args.warmup} warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hmm.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    kern_ms, launches = hmm.profile_read(hmm.PROF_FWD_BATCHED)
    hmm.profile_enable(False)
    kern_s = kern_ms / 1e3 / max(launches, 1)
    flops = 2.0 * units
    achieved = flops / kern_s / 1e12
    traffic = measured_traffic("c3_classify", leg_choice(tuning, "c3_classify"), family)
    kname = " ".join(FAMILY_KERNELS[family][:2]) if family in FAMILY_KERNELS else family
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": kname, "kernel_ms": round(kern_s * 1e3, 4),
                "launches": launches}
    result = {"metric": METRIC, "value": units / sec, "unit": "state-steps/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": "c3 recognition: 64 HMMs N=32 M=256 Dirichlet(0.5), 65536 sequences, "
                                     "log-uniform T in [16,2048], all pairs + arg-max (hmm_classify)",
                         "models": w.K, "states": w.N, "symbols": w.M, "sequences": w.S,
                         "sum_T": int(w.lengths.sum()), "state_steps_per_step": units},
              "roofline": roofline}

    if want("plain"):
        log("plain per-pair kernel on the same workload")
        hmm.select_kernel(hmm.KERNEL_PLAIN)
        psec = time_steps(step, 2, 1, torch)
        hmm.select_kernel(hmm.KERNEL_AUTO)
        result["plain"] = {"value": units / psec, "ms_per_step": psec * 1e3,
                           "speedup_batched_over_plain": psec / sec}
    w4 = workloads.make_workload("c4") if (want("grad") or want("em")) else None
    if want("grad"):
        log("forward + adjoint on the gradient workload (8 models, N=64, M=512, 8192 sequences)")
        p4 = to_dev(w4, torch, own=True)
        # the gradient configuration keeps alpha every ceil(sqrt(T)) steps; every step stored
        # is timed beside it
        rows4 = 0
        autotune("c4_grad", p4, hmm.OP_GRAD, grad_rows=rows4)
        ws4 = p4.grad_workspace(rows4)
        ll4 = torch.empty(w4.S, dtype=torch.float32, device="cuda")
        cnt = (torch.empty((w4.K, w4.N), device="cuda"), torch.empty((w4.K, w4.N, w4.N), device="cuda"),
               torch.empty((w4.K, w4.N, w4.M), device="cuda"))

        def gstep():
            hmm.forward_backward_grad(p4, phase=0, loglik=ll4, counts=cnt, ws=ws4)

        for _ in range(2):
            gstep()
        torch.cuda.synchronize()
        hmm.profile_enable(True)
        gsteps = 10
        t0 = time.perf_counter()
        for _ in range(gsteps):
            gstep()
        torch.cuda.synchronize()
        gsec = (time.perf_counter() - t0) / gsteps
        f_ms, f_n = hmm.profile_read(hmm.PROF_FWD_BATCHED)
        a_ms, a_n = hmm.profile_read(hmm.PROF_ADJ_BATCHED)
        hmm.profile_enable(False)
        u4 = w4.units()
        result["fwd_bwd"] = {"workload": "c4 gradient: 8 HMMs N=64 M=512, 8192 sequences, T in [100,1000], "
                                         "own model, fused forward + adjoint",
                             "value": u4 / gsec, "unit": "state-steps/s", "ms_per_step": gsec * 1e3,
                             "fwd_kernel_ms": f_ms / max(f_n, 1), "adj_kernel_ms": a_ms / max(a_n, 1),
                             "frac_fp32_peak": 6.0 * u4 / gsec / 1e12 / FP32_PEAK_TFLOPS,
                             "storage": "every step" if rows4 else "checkpoints", "workspace_bytes": ws4.numel(),
                             "traffic": traffic_fields({"forward": ("c4_grad_forward", f_ms / max(f_n, 1)),
                                                        "adjoint": ("c4_grad_adjoint", a_ms / max(a_n, 1))},
                                                       tuning)}
        if grad_rows(p4, w4, torch) and not args.no_storage_compare:
            result["fwd_bwd"]["every_step"] = time_grad_storage(p4, w4.total_symbols, 10, torch)
        if not args.no_cpu:
            log("CPU oracle forward + backward on a c4 sample")
            result["fwd_bwd"]["cpu_oracle"] = cpu_oracle_counts(w4)
        del p4, ws4, cnt

    if want("large") or want("large_viterbi"):
        log("the N=256 bank (16 models, M=1024, 16384 sequences)")
        w5 = workloads.make_workload("c5")
        p5 = to_dev(w5, torch, own=True)
        u5 = w5.units()
        ll5 = torch.empty(w5.S, dtype=torch.float32, device="cuda")
        large = {"workload": "c5: 16 HMMs N=256 M=1024 (A = Dirichlet(0.1) + band of 8), 16384 sequences, "
                             "T in [256,4096], own model, cooperative kernels"}
    if want("large"):
        log("c5 forward, then forward + adjoint")
        autotune("c5_forward", p5, hmm.OP_FORWARD, warmup=0, reps=2)
        ws5 = p5.workspace(hmm.OP_FORWARD)
        hmm.profile_enable(True)
        s5 = time_steps(lambda: hmm.forward_loglik(p5, out=ll5, ws=ws5), 3, 1, torch)
        k5_ms, k5_n = hmm.profile_read(hmm.PROF_FWD_BATCHED)
        hmm.profile_enable(False)
        del ws5
        large.update({"value": u5 / s5, "unit": "state-steps/s", "ms_per_step": s5 * 1e3,
                      "kernel_ms": k5_ms / max(k5_n, 1),
                      "frac_fp32_peak": 2.0 * u5 / (k5_ms / max(k5_n, 1) / 1e3) / 1e12 / FP32_PEAK_TFLOPS,
                      "traffic": traffic_fields({"forward": ("c5_forward", k5_ms / max(k5_n, 1))}, tuning)})
        rows5 = grad_rows(p5, w5, torch)
        autotune("c5_grad", p5, hmm.OP_GRAD, warmup=0, reps=2, grad_rows=rows5)
        ws5g = p5.grad_workspace(rows5)
        cnt5 = (torch.empty((w5.K, w5.N), device="cuda"), torch.empty((w5.K, w5.N, w5.N), device="cuda"),
                torch.empty((w5.K, w5.N, w5.M), device="cuda"))
        g5 = lambda: hmm.forward_backward_grad(p5, phase=0, loglik=ll5, counts=cnt5, ws=ws5g)
        g5()
        torch.cuda.synchronize()
        hmm.profile_enable(True)
        gs5 = time_steps(g5, 2, 0, torch)
        f5_ms, f5_n = hmm.profile_read(hmm.PROF_FWD_BATCHED)
        a5_ms, a5_n = hmm.profile_read(hmm.PROF_ADJ_BATCHED)
        hmm.profile_enable(False)
        large["fwd_bwd"] = {"value": u5 / gs5, "unit": "state-steps/s", "ms_per_step": gs5 * 1e3,
                            "fwd_kernel_ms": f5_ms / max(f5_n, 1), "adj_kernel_ms": a5_ms / max(a5_n, 1),
                            "frac_fp32_peak": 6.0 * u5 / gs5 / 1e12 / FP32_PEAK_TFLOPS,
                            "storage": "every step" if rows5 else "checkpoints", "workspace_bytes": ws5g.numel(),
                            "traffic": traffic_fields({"forward": ("c5_grad_forward", f5_ms / max(f5_n, 1)),
                                                       "adjoint": ("c5_grad_adjoint", a5_ms / max(a5_n, 1))},
                                                      tuning)}
        del ws5g, cnt5
        if rows5 and not args.no_storage_compare:
            log("c5 gradient with checkpoints (the bounded-memory storage)")
            large["fwd_bwd"]["checkpoints"] = time_grad_storage(p5, 0, 2, torch)
    if want("large_viterbi"):
        log("c5 Viterbi (workgroup decoder: 256 states)")
        wsv5 = p5.workspace(hmm.OP_VITERBI)
        scv5 = torch.empty(w5.S, dtype=torch.float32, device="cuda")
        pav5 = torch.empty(w5.total_symbols, dtype=torch.int32, device="cuda")
        fv5 = lambda: hmm.viterbi(p5, score=scv5, path=pav5, ws=wsv5)
        fv5()
        torch.cuda.synchronize()
        hmm.profile_enable(True)
        sv5 = time_steps(fv5, 2, 0, torch)
        kv5_ms, kv5_n = hmm.profile_read(hmm.PROF_VITERBI)
        hmm.profile_enable(False)
        kv5_s = kv5_ms / max(kv5_n, 1) / 1e3
        large["viterbi"] = {"value": u5 / sv5, "unit": "state-steps/s", "ms_per_step": sv5 * 1e3,
                            "kernels_ms": kv5_s * 1e3,  # decoder + traceback
                            "workspace_bytes": wsv5.numel(),
                            "roofline": {"bound": "alu", "achieved": round(2.0 * u5 / kv5_s / 1e12, 3),
                                         "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                                         "frac": round(2.0 * u5 / kv5_s / 1e12 / VALU_PEAK_TOPS, 4)}}
        # the same decode with room for every delta row (one round) for comparison
        del wsv5
        wsv5 = p5.viterbi_workspace(w5.total_symbols)
        fv5()
        torch.cuda.synchronize()
        large["viterbi"]["one_round"] = {"ms_per_step": time_steps(fv5, 2, 0, torch) * 1e3,
                                         "workspace_bytes": wsv5.numel()}
        del wsv5, scv5, pav5
    if want("large") or want("large_viterbi"):
        result["large_states"] = large
        del p5

    if want("latency"):
        log("latency-bound workloads c1 and c2")
        hmm.select_kernel(hmm.KERNEL_AUTO)
        lat = {}
        w1 = workloads.make_workload("c1")
        p1 = to_dev(w1, torch, own=True)
        autotune("c1_forward", p1, hmm.OP_FORWARD, warmup=5, reps=20)
        ws1 = p1.workspace(hmm.OP_FORWARD)
        ll1 = torch.empty(w1.S, dtype=torch.float32, device="cuda")
        f1 = lambda: hmm.forward_loglik(p1, out=ll1, ws=ws1)
        e1 = time_steps(f1, 50, 5, torch)
        es1, gs1 = eager_stats(f1, 50, torch), graph_stats(f1, 50, torch)
        gb1 = graph_stats(f1, 20, torch, batch=16)
        lat["c1"] = {"workload": "c1: 1 HMM N=8 M=16, one sequence T=64, forward (tuned choice: "
                                 f"{tune.KERNEL_NAMES[hmm.call_kernel(p1.bank, p1.batch, hmm.OP_FORWARD)]})",
                     "us_per_call": e1 * 1e6,
                     "us_per_call_stream_median": es1["median_ms"] * 1e3, "us_per_call_stream_min": es1["min_ms"] * 1e3,
                     "us_per_call_graph": gs1["median_ms"] * 1e3, "us_per_call_graph_min": gs1["min_ms"] * 1e3,
                     "us_per_call_graph_back_to_back": gs1["back_to_back_ms"] * 1e3,
                     "graph_replays": gs1["replays"],
                     "ns_per_step_graph": gs1["median_ms"] * 1e6 / int(w1.lengths.max()),
                     # 16 consecutive calls in one graph: the runtime's fixed cost per graph
                     # launch (graph_launch_floor) is paid once for 16 calls
                     "us_per_call_graph16": gb1["median_ms"] * 1e3, "us_per_call_graph16_min": gb1["min_ms"] * 1e3,
                     "us_per_call_graph16_back_to_back": gb1["back_to_back_ms"] * 1e3,
                     "graph16_replays": gb1["replays"]}
        lat["graph_launch_floor"] = graph_floor_us(torch)
        hmm.select_kernel(hmm.KERNEL_TILE16)
        lat["c1"]["us_per_call_tiles"] = time_steps(f1, 50, 5, torch) * 1e6
        hmm.select_kernel(hmm.KERNEL_AUTO)
        w1l = workloads.random_lengths_workload(np.random.default_rng(7), K=1, N=8, M=16,
                                                lengths=np.array([4096]), all_pairs=False)
        p1l = to_dev(w1l, torch, own=True)
        autotune("one_long_forward", p1l, hmm.OP_FORWARD, warmup=3, reps=10)
        ws1l = p1l.workspace(hmm.OP_FORWARD)
        ll1l = torch.empty(1, dtype=torch.float32, device="cuda")
        f1l = lambda: hmm.forward_loglik(p1l, out=ll1l, ws=ws1l)
        lat["one_long"] = {"workload": "one sequence T=4096, N=8 M=16 (c1 bank shape), forward (tuned choice: "
                                       f"{tune.KERNEL_NAMES[hmm.call_kernel(p1l.bank, p1l.batch, hmm.OP_FORWARD)]})",
                           "us_per_call": time_steps(f1l, 20, 3, torch) * 1e6}
        hmm.select_kernel(hmm.KERNEL_TILE16)
        lat["one_long"]["us_per_call_tiles"] = time_steps(f1l, 20, 3, torch) * 1e6
        hmm.select_kernel(hmm.KERNEL_AUTO)
        w2 = workloads.make_workload("c2")
        p2 = to_dev(w2, torch, own=False)
        b2 = p2.batch_without_models()
        autotune("c2_classify", p2, hmm.OP_CLASSIFY, warmup=3, reps=10)
        ws2 = p2.workspace(hmm.OP_CLASSIFY, b2)
        lab2 = torch.empty(w2.S, dtype=torch.int32, device="cuda")
        ll2 = torch.empty((w2.S, w2.K), dtype=torch.float32, device="cuda")
        f2 = lambda: hmm.classify(p2, labels=lab2, loglik=ll2, ws=ws2)
        e2 = time_steps(f2, 20, 3, torch)
        es2, gs2 = eager_stats(f2, 20, torch), graph_stats(f2, 20, torch)
        gb2 = graph_stats(f2, 20, torch, batch=16)
        g2 = gs2["median_ms"]
        lat["c2"] = {"workload": "c2: 12 HMMs N=16 M=64, 4096 sequences, T in [50,400], all pairs + labels",
                     "us_per_call": e2 * 1e6,
                     "us_per_call_stream_median": es2["median_ms"] * 1e3, "us_per_call_stream_min": es2["min_ms"] * 1e3,
                     "us_per_call_graph": g2 * 1e3, "us_per_call_graph_min": gs2["min_ms"] * 1e3,
                     "us_per_call_graph_back_to_back": gs2["back_to_back_ms"] * 1e3,
                     "graph_replays": gs2["replays"],
                     "ns_per_step_graph": g2 * 1e6 / int(w2.lengths.max()),
                     "state_steps_per_s_graph": w2.units() / (g2 / 1e3),
                     "us_per_call_graph16": gb2["median_ms"] * 1e3, "us_per_call_graph16_min": gb2["min_ms"] * 1e3,
                     "us_per_call_graph16_back_to_back": gb2["back_to_back_ms"] * 1e3,
                     "graph16_replays": gb2["replays"]}
        result["latency"] = lat

    if want("viterbi"):
        log("Viterbi decoding of the c3 sequences with their owner models")
        p3o = to_dev(w, torch, own=True)
        autotune("c3_viterbi", p3o, hmm.OP_VITERBI, warmup=0, reps=2)
        wsv = p3o.workspace(hmm.OP_VITERBI)
        scv = torch.empty(w.S, dtype=torch.float32, device="cuda")
        pav = torch.empty(w.total_symbols, dtype=torch.int32, device="cuda")
        fv = lambda: hmm.viterbi(p3o, score=scv, path=pav, ws=wsv)
        fv()
        torch.cuda.synchronize()
        hmm.profile_enable(True)
        sv = time_steps(fv, 5, 0, torch)
        kv_ms, kv_n = hmm.profile_read(hmm.PROF_VITERBI)
        hmm.profile_enable(False)
        uv = float(w.N) ** 2 * float(w.lengths.sum())
        kv_s = kv_ms / max(kv_n, 1) / 1e3
        result["viterbi"] = {"workload": "c3 bank, 65536 sequences each decoded with its owner model, "
                                         "score + path (N=32)",
                             "value": uv / sv, "unit": "state-steps/s", "ms_per_step": sv * 1e3,
                             "kernels_ms": kv_s * 1e3,  # decoder + traceback, HIP events around both
                             "workspace_bytes": wsv.numel(),
                             "roofline": {"bound": "alu", "achieved": round(2.0 * uv / kv_s / 1e12, 3),
                                          "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                                          "frac": round(2.0 * uv / kv_s / 1e12 / VALU_PEAK_TOPS, 4)}}
        del wsv
        wsv = p3o.viterbi_workspace(w.total_symbols)
        fv()
        torch.cuda.synchronize()
        result["viterbi"]["one_round"] = {"ms_per_step": time_steps(fv, 5, 0, torch) * 1e3,
                                          "workspace_bytes": wsv.numel()}
        del p3o, wsv, scv, pav

    if want("em"):
        log("one Baum-Welch iteration on c4")
        p4e = to_dev(w4, torch, own=True)
        hmm.baum_welch(p4e, 1)
        torch.cuda.synchronize()
        se = time_steps(lambda: hmm.baum_welch(p4e, 1), 5, 0, torch)
        result["em"] = {"workload": "c4: one EM iteration (forward + adjoint + M-step), parameters updated in place",
                        "value": w4.units() / se, "unit": "state-steps/s", "ms_per_iteration": se * 1e3}
        del p4e

    if want("graph"):
        gs = graph_stats(step, 20, torch)
        result["graph"] = {"ms_per_step": gs["median_ms"], "min_ms": gs["min_ms"], "mean_ms": gs["mean_ms"],
                           "back_to_back_ms": gs["back_to_back_ms"], "replays": gs["replays"],
                           "note": "the same recognition step captured once as a HIP graph: median, min and mean "
                                   "of 20 replays, each timed with its own events"}
    if want("h2d"):
        h2d = h2d_copy(w, torch)
        h2d["note"] = ("bank + symbols + offsets + lengths of the recognition workload, pinned host memory to HBM "
                       "(not part of `value`, whose inputs are resident in HBM)")
        h2d["state_steps_per_s_including_h2d"] = units / (sec + h2d["ms"] / 1e3)
        result["h2d"] = h2d

    if args.copy_calibration:
        log("copy calibration: 4 x 512 MiB device-to-device")
        src = torch.empty(128 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = src.numel() * 4

    result["provenance"] = {
        "inputs": "numpy default_rng(SeedSequence([1310, 3322, tag, 0])) per workload, regenerated each run; "
                  "tag = index in (brute, c1, paper, c2, c3, c4, c5)",
        "numpy": np.__version__, "torch": torch.__version__, "hip": getattr(torch.version, "hip", None),
        "device": torch.cuda.get_device_name(0), "host_cores": len(os.sched_getaffinity(0)),
        "library": os.path.relpath(hmm.LIB_PATH, ROOT)}
    if not args.no_tune:
        result["tuning"] = tuning
        if args.tune_cache and tuned_now:
            tune.save_cache(args.tune_cache, tuned_now)

    if not args.no_cpu:
        log("CPU oracle baseline on a stratified sample")
        result["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
