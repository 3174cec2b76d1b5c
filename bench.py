"""Benchmark: gates/s and effective HBM bandwidth of the state-vector gate engine on one MI355X.

Default workload: the 33-qubit complex128 brickwork circuit (128 GiB state, 20 layers of Haar-random
2x2 unitaries on every qubit + CZ on alternating neighbour pairs, 980 gates, seed 21, start
|0...0>). A step is one full run of the circuit from |0...0> through the framework's fastest plan;
the plain per-gate plan (one sweep per gate) is timed once beside it.

Prints ONE JSON line (rank 0). `value` is gates/s of the whole job (one GPU) with the state already
resident in HBM. `roofline` describes the dominant kernel of the timed plan, its average launch
duration measured with HIP events on the state's stream over the timed steps. `cpu_baseline` is the
FP64 CPU oracle timed on a bounded sample of the same circuit family on this host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
METRIC = "gates/s & effective HBM GB/s (% of peak) at 30–34 qubits; fused vs plain"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_quant_ph_0608239_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    e = rec.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(n_full: int, layers: int, seed: int, budget_s: float, n_sample: int) -> dict:
    """The oracle (unmodified) on the same brickwork family at n_sample qubits, gates in circuit order
    until the time budget is spent; gates/s scaled to n_full by the paper's O(2^L) work per gate."""
    import oracle
    import qsim_workloads as wl
    oracle.lib()
    text = wl.brickwork_circuit(n_sample, layers, seed)
    c = oracle.parse(text)
    a = oracle.basis_state(c.n, 0)
    t0 = time.perf_counter()
    done = 0
    for kw, args in c.ops:
        oracle.apply_op(a, c.n, kw, args)
        done += 1
        if time.perf_counter() - t0 > budget_s and done >= 8:
            break
    dt = time.perf_counter() - t0
    rate = done / dt
    scaled = rate * 2.0 ** (n_sample - n_full)
    threads = oracle.threads()
    return {"value": scaled, "unit": "gates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} gates of the {n_sample}-qubit complex128 brickwork circuit (seed {seed}) in "
                      f"{dt:.1f} s = {rate:.2f} gates/s at {n_sample} qubits, scaled by 2^({n_sample}-{n_full}) "
                      f"to {n_full} qubits (work per gate is O(2^n))"}


def sweep_mode(args) -> int:
    """Per-target timing of single gates (the per-qubit Hadamard timing of the paper's benchmark
    section, on one GPU) and of fused k-qubit gates at several qubit positions. One JSON line per
    measurement on stdout."""
    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    n, dtype = args.n, args.dtype
    amp = 16 if dtype == "c128" else 8
    full = 2.0 * amp * 2 ** n
    s = q.State(n, dtype)
    H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
    X = np.array([[0, 1], [1, 0]])
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timeit(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        best = 1e30
        for _ in range(reps):
            ev0.record()
            fn()
            ev1.record()
            torch.cuda.synchronize()
            best = min(best, ev0.elapsed_time(ev1))
        return best

    def emit(**kw):
        print(json.dumps(kw), flush=True)

    targets = list(range(n)) if args.targets == "all" else [int(x) for x in args.targets.split(",")]
    for t in targets:
        ms = timeit(lambda: s.apply_1q(t, H))
        emit(kind="H", n=n, dtype=dtype, target=t, ms=round(ms, 4), GBps=round(full / ms / 1e6, 1))
    for t in [0, 3, 10, n - 1]:
        c = (t + 1) % n
        ms = timeit(lambda: s.apply_ctrl(1 << c, t, X))
        emit(kind="CNOT", n=n, target=t, control=c, ms=round(ms, 4), GBps_alg=round(full / 2 / ms / 1e6, 1))
        ms = timeit(lambda: s.apply_phase(1 << c, t, 0.3))
        emit(kind="CPHASE", n=n, target=t, control=c, ms=round(ms, 4), GBps_alg=round(full / 4 / ms / 1e6, 1))
    rng = np.random.default_rng(0)
    for k in (3, 4, 5):
        Z = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
        U, _ = np.linalg.qr(Z)
        for name, qs in [("low", list(range(k))), ("high", list(range(n - k, n))),
                         ("mid", list(range(n // 2, n // 2 + k))), ("spread", [int(x) for x in np.linspace(0, n - 1, k)])]:
            ms = timeit(lambda: s.apply_fused(qs, U))
            fl = 8.0 * 2 ** (n + k)
            emit(kind=f"fused{k}", n=n, dtype=dtype, qubits=qs, where=name, ms=round(ms, 4),
                 GBps=round(full / ms / 1e6, 1), TFLOPs=round(fl / ms / 1e9, 2))
    return 0


def batch_mode(args) -> int:
    """Many independent circuits in one persistent launch: circuits/s, gates/s and per-circuit
    latency percentiles from device timestamps. One JSON line."""
    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    import qsim_workloads as wl
    texts = wl.batch_circuits(count=args.count, nmin=10, nmax=22, depth=50, seed=41)
    b = q.Batch(texts, args.dtype, lds_qubits=args.lds, lds_regs=args.lds_regs, use_graph=False)
    for _ in range(args.warmup):
        b.run()
    runs = [b.run() for _ in range(args.steps)]
    ms = float(np.mean([r["launch_ms"] for r in runs]))
    lat = b.latencies_us()
    out = {"metric": "circuits/s (batch of independent circuits, one persistent launch)", "value": round(args.count / ms * 1e3, 1),
           "unit": "circuits/s", "gates_per_s": round(b.total_gates / ms * 1e3, 1), "ms_per_launch": round(ms, 3),
           "latency_us": {"p50": round(float(np.percentile(lat, 50)), 1), "p99": round(float(np.percentile(lat, 99)), 1),
                          "max": round(float(lat.max()), 1)},
           "config": {"workload": f"batch-{args.count}-circuits-n10-22-depth50-{args.dtype}", "count": args.count,
                      "gates": b.total_gates, "seed": 41}, "dtype": "f64" if args.dtype == "c128" else "f32"}
    print(json.dumps(out), flush=True)
    return 0


def copycal_mode(args) -> int:
    """Calibration of the HBM byte counters: a fill (writes only) and a device-to-device copy (reads
    and writes) of a buffer of known size, so that FETCH_SIZE / WRITE_SIZE per dispatch can be
    scaled to bytes."""
    import torch
    nbytes = int(args.copy_gib * 2 ** 30)
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1.0)
    for _ in range(args.steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copycal", "fill_bytes_written": nbytes, "copy_bytes_read": nbytes,
                      "copy_bytes_written": nbytes, "copies": args.steps}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", default="bench", choices=["bench", "sweep", "batch", "copycal"])
    ap.add_argument("--copy-gib", type=float, default=4.0, help="buffer size of --mode copycal")
    ap.add_argument("--count", type=int, default=2048)
    ap.add_argument("--targets", default="all")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=33)
    ap.add_argument("--layers", type=int, default=20)
    ap.add_argument("--seed", type=int, default=21)
    ap.add_argument("--dtype", default="c128")
    ap.add_argument("--method", default="auto", choices=["auto", "fused", "staged", "plain"],
                    help="auto: the autotuner times the candidate plans on the state (outside the timed region)")
    ap.add_argument("--fuse-k", type=int, default=5)
    ap.add_argument("--lds", type=int, default=0, help="resident qubits per LDS block (staged plans)")
    ap.add_argument("--lds-regs", type=int, default=0, help="log2 amplitudes per thread (staged plans)")
    ap.add_argument("--plain-runs", type=int, default=1, help="timed runs of the plain per-gate plan (0 = skip)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-n", type=int, default=26)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.mode == "sweep":
        return sweep_mode(args)
    if args.mode == "batch":
        return batch_mode(args)
    if args.mode == "copycal":
        return copycal_mode(args)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (no sharding, no "
              "collectives); run it with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    import qsim_workloads as wl
    from paper_quant_ph_0608239_amd._lib import KERNEL_NAMES

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n, dtype = args.n, args.dtype
    amp = 16 if dtype == "c128" else 8
    workload = f"brickwork-{n}q-{dtype}-{args.layers}layers"
    log(f"workload {workload}: generating circuit")
    text = wl.brickwork_circuit(n, args.layers, args.seed)
    circ = q.parse_circuit(text)
    G = len(circ.gates)
    log(f"{G} gates; allocating {amp * 2 ** n / 2 ** 30:.0f} GiB state")
    state = q.State(n, dtype, device=dev)
    tuned = None
    if args.method == "auto":
        from paper_quant_ph_0608239_amd import tuning
        t0 = time.perf_counter()
        tuned = tuning.tune(circ, state, reps=1, include_plain=False, use_cache=False)
        log(f"autotune ({time.perf_counter() - t0:.1f} s): best {tuned['method']} k={tuned['fuse_k']} "
            f"lds={tuned['lds_qubits']}/{tuned['lds_regs']} {tuned['ms']:.1f} ms; tried "
            + ", ".join(f"{t['method']}:{t['fuse_k'] or ''}{t['lds_qubits'] or ''}/{t['lds_regs'] or ''}={t['ms']:.0f}"
                        for t in tuned["tried"]))
        plan = q.Plan(circ, dtype, method=tuned["method"], fuse_k=tuned["fuse_k"] or 5, lds_qubits=tuned["lds_qubits"],
                      lds_regs=tuned["lds_regs"])
    else:
        plan = q.Plan(circ, dtype, method=args.method, fuse_k=args.fuse_k, lds_qubits=args.lds, lds_regs=args.lds_regs)
    log(f"plan {args.method}: {plan.info}")

    def step(timed: bool):
        state.set_basis(0)
        if timed:
            return plan.execute_timed(state)
        plan.execute(state)
        return None

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch_ms, kinds, fks = [], None, None
    for i in range(args.steps):
        ms, kinds, fks = step(True)
        launch_ms.append(ms)
        log(f"step {i + 1}/{args.steps}: {ms.sum():.1f} ms in {len(ms)} launches")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    gates_per_s = G / (wall / args.steps)
    plan_bytes = plan.info["alg_bytes"]
    eff_gbps = plan_bytes / (wall / args.steps) / 1e9

    # dominant kernel of the timed plan: the class (and fused width) with the most total time
    L = np.stack(launch_ms)  # steps x launches
    avg_per_launch = L.mean(axis=0)
    classes = {}
    for i, (kd, fk) in enumerate(zip(kinds, fks)):
        key = (int(kd), int(fk))
        classes.setdefault(key, []).append(i)
    dom_key = max(classes, key=lambda k: avg_per_launch[classes[k]].sum())
    dom_idx = classes[dom_key]
    dom_avg_ms = float(avg_per_launch[dom_idx].mean())
    dom_name = KERNEL_NAMES[dom_key[0]] + (f"_k{dom_key[1]}" if dom_key[1] else "")
    if KERNEL_NAMES[dom_key[0]] == "staged":
        dom_name += f"_m{plan.info['lds_qubits']}r{plan.info['lds_regs']}"
    full_sweep_bytes = 2.0 * amp * 2 ** n
    if dom_key[0] in (4, 5, 6):
        dom_bytes = full_sweep_bytes
        dom_flops = 8.0 * 2 ** (n + dom_key[1]) if dom_key[1] else 0.0
    else:
        dom_bytes = full_sweep_bytes  # a 2x2 sweep reads and writes every amplitude
        dom_flops = 0.0
    achieved = dom_bytes / (dom_avg_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": load_traffic(workload, dom_name),
            "kernel": dom_name, "launches": len(dom_idx), "avg_launch_ms": round(dom_avg_ms, 3),
            "alg_bytes_per_launch": dom_bytes}
    if dom_flops:
        peak_tf = FP64_PEAK_TFLOPS if dtype == "c128" else FP32_PEAK_TFLOPS
        tf = dom_flops / (dom_avg_ms / 1e3) / 1e12
        roof["mfma_tflops"] = round(tf, 2)
        roof["mfma_frac"] = round(tf / peak_tf, 4)
        roof["alg_flops_per_launch"] = dom_flops

    out = {
        "metric": METRIC, "value": round(gates_per_s, 3), "unit": "gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if dtype == "c128" else "f32", "data": "synthetic",
        "config": {"workload": workload, "n_qubits": n, "state": dtype, "layers": args.layers, "gates": G,
                   "seed": args.seed, "method": ["plain", "fused", "staged"][int(plan.info["method"])],
                   "fuse_k": int(plan.info["fuse_k"]) or None, "lds_qubits": int(plan.info["lds_qubits"]) or None,
                   "launches_per_step": int(plan.info["launches"]),
                   "autotune": None if tuned is None else {
                       "choice": {k: tuned[k] for k in ("method", "fuse_k", "lds_qubits", "lds_regs")},
                       "tried_ms": {f"{t['method']}{'-k' + str(t['fuse_k']) if t['method'] == 'fused' else ''}"
                                    f"{'-m' + str(t['lds_qubits']) + 'r' + str(t['lds_regs']) if t['method'] == 'staged' else ''}":
                                    round(t["ms"], 1) for t in tuned["tried"]}}},
        "eff_GBps": round(eff_gbps, 1), "hbm_frac": round(eff_gbps / HBM_PEAK_GBPS, 4),
        "roofline": roof,
    }

    # the plain per-gate plan, timed beside it
    if args.plain_runs > 0:
        pplan = q.Plan(circ, dtype, method="plain")
        pms = []
        pk = None
        for r in range(args.plain_runs):
            state.set_basis(0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, pk, _ = pplan.execute_timed(state)
            torch.cuda.synchronize()
            pms.append((time.perf_counter() - t1, ms))
            log(f"plain run {r + 1}/{args.plain_runs}: {pms[-1][0]:.2f} s")
        pwall = float(np.mean([w for w, _ in pms]))
        pl = np.mean(np.stack([m for _, m in pms]), axis=0)
        gen = [i for i, kd in enumerate(pk) if kd == 0]
        gen_ms = float(pl[gen].mean()) if gen else None
        out["plain"] = {
            "gates_per_s": round(G / pwall, 3), "s_per_run": round(pwall, 3),
            "eff_GBps": round(pplan.info["alg_bytes"] / pwall / 1e9, 1),
            "hbm_frac": round(pplan.info["alg_bytes"] / pwall / 1e9 / HBM_PEAK_GBPS, 4),
            "general_sweep_avg_ms": round(gen_ms, 3) if gen_ms else None,
            "general_sweep_GBps": round(full_sweep_bytes / (gen_ms / 1e3) / 1e9, 1) if gen_ms else None,
        }
        out["speedup_vs_plain"] = round(gates_per_s / (G / pwall), 2)

    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(n, args.layers, args.seed, args.cpu_budget, min(args.cpu_n, n))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
