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
FP64_PEAK_TFLOPS = 78.6       # dense FP64 MFMA
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 MFMA
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s, the same for FP64 and
# for FP32 as compiled here (no packed FP32 instructions)
VALU_PEAK_TFLOPS = 78.6
METRIC = "gates/s & effective HBM GB/s (% of peak) at 30–34 qubits; fused vs plain"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = {"staged": ("staged.hip", "staged_device.h", "qsim_internal.h"),
                  "fused": ("fused.hip", "qsim_internal.h"),
                  "sweep": ("sweep.hip", "qsim_internal.h")}


def kernel_source_hash(kernel: str) -> str:
    """Hash of the source files that hold a kernel class's device code (staged_*, fused_*, else the
    sweeps)."""
    fam = "staged" if kernel.startswith("staged") else "fused" if kernel.startswith("fused") else "sweep"
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_quant_ph_0608239_amd", "csrc")
    for f in KERNEL_SOURCES[fam]:
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
    if not e or e.get("source_hash") != kernel_source_hash(kernel):
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


# elapsed times of the paper's runs (App. B tables), seconds: context only, other machines
PAPER_T_E = {
    "H-33": {"IBM Blue Gene/L N=512": 79, "IBM Regatta p690+ N=64": 492, "Hitachi SR11000/J1 N=64": 148},
    "H-34": {"IBM Blue Gene/L N=1024": 85, "IBM Regatta p690+ N=128": 526, "Hitachi SR11000/J1 N=128": 164},
    "3-11QBA": {"IBM Blue Gene/L N=512": 649, "IBM Regatta p690+ N=64": 2568, "Hitachi SR11000/J1 N=128": 586,
                "SGI Altix 3700 N=64": 4112},
    "2-17QBA": {"IBM Blue Gene/L N=1024": 934, "IBM Regatta p690+ N=128": 4019, "Hitachi SR11000/J1 N=128": 1653},
    "Shor-33-1961": {"SGI Altix 3700 N=64": 630, "IBM Regatta p690+ N=64": 810},
    "Shor-33-2047": {"SGI Altix 3700 N=64": 630, "IBM Regatta p690+ N=64": 810},
}


def paper_mode(args) -> int:
    """The paper's own workloads at full size (Sec. V; App. B): Hadamard on every qubit, the QFT
    register adders 3-11QBA (33 qubits, complex128) and 2-17QBA (34 qubits, complex64), and Shor's
    algorithm at L = 33 (the two Table Shortab cases). Each run is timed from the initial state to
    the measured qubit expectation values <Q_i>, as the paper's elapsed times are, and its result is
    checked: <Q_i> = 1/2 after the Hadamards, the printed sum with probability ~1 for the adders, and
    the printed <Q_i> table for Shor. One JSON line per workload."""
    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    import qsim_workloads as wl

    table = {}
    with open(os.path.join(ROOT, "tests", "golden", "shor_table.txt")) as f:
        for ln in f:
            if ln.strip() and not ln.startswith("#"):
                t = ln.split()
                table[tuple(int(v) for v in t[:4])] = np.array([float(v) for v in t[5:]])

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res

    def emit(name, n, dtype, n_o, gates, secs, ok, detail):
        print(json.dumps({"workload": name, "n_qubits": n, "state": dtype, "paper_N_O": n_o, "gates": gates,
                          "seconds": round(secs, 4), "paper_ops_per_s": round(n_o / secs, 2), "check_passed": ok,
                          "check": detail, "paper_t_E_s": PAPER_T_E.get(name)}), flush=True)

    for n, dtype in ((33, "c128"), (34, "c64")):
        s = q.State(n, dtype)
        # Hadamard on every qubit, then <Q_i>
        c = q.parse_circuit(wl.circuit_text(n, [f"H {k}" for k in range(n)]))
        p = q.Plan(c, dtype, method="auto")
        s.set_basis(0)
        p.execute(s)
        s.marginals()
        secs, m = timed(lambda: (s.set_basis(0), p.execute(s), s.marginals())[2])
        dev = float(np.max(np.abs(m - 0.5)))
        emit(f"H-{n}", n, dtype, n, n, secs, dev < (1e-12 if dtype == "c128" else 1e-5), {"max_abs_Q_minus_half": dev})
        p.close()
        # the register adder of this size
        values, m_bits = ((292, 585, 1170), 11) if n == 33 else ((26214, 104857), 17)
        text, lay = wl.qft_adder_circuit(list(values), m_bits)
        c = q.parse_circuit(text)
        p = q.Plan(c, dtype, method="auto")
        s.set_basis(0)
        p.execute(s)
        secs, mq = timed(lambda: (s.set_basis(0), p.execute(s), s.marginals())[2])
        want = 0
        for i, v in enumerate(values[:-1]):
            want |= v << (i * m_bits)
        want |= lay["sum"] << ((len(values) - 1) * m_bits)
        bits = np.array([(want >> i) & 1 for i in range(n)], dtype=np.float64)
        dev = float(np.max(np.abs(mq - bits)))
        name = f"{len(values)}-{m_bits}QBA"
        emit(name, n, dtype, wl.count_gates(text), len(c.gates), secs, dev < (1e-10 if dtype == "c128" else 1e-4),
             {"sum": lay["sum"], "max_abs_Q_minus_sum_bits": dev})
        p.close()
        if n == 33:
            for G, y in ((1961, 1698), (2047, 617)):
                X = 22
                pre, mx, post = wl.shor_parts(n, X, G, y)
                p1 = q.Plan(q.parse_circuit(pre), dtype, method="auto")
                p2 = q.Plan(q.parse_circuit(post), dtype, method="auto")

                def shor():
                    s.set_basis(0)
                    p1.execute(s)
                    s.apply_modexp(*mx)
                    p2.execute(s)
                    return s.marginals()

                shor()
                secs, mq = timed(shor)
                dev = float(np.max(np.abs(mq[:X] - table[(n, X, G, y)])))
                n_o = len(q.parse_circuit(pre).gates) + 1 + len(q.parse_circuit(post).gates)
                emit(f"Shor-33-{G}", n, dtype, n_o, n_o, secs, dev <= 5e-4 + 1e-12, {"max_abs_Q_minus_table": dev})
                p1.close()
                p2.close()
        s.close()
        del s
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
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
    ap.add_argument("--mode", default="bench", choices=["bench", "sweep", "batch", "paper", "copycal"])
    ap.add_argument("--copy-gib", type=float, default=4.0, help="buffer size of --mode copycal")
    ap.add_argument("--count", type=int, default=2048)
    ap.add_argument("--targets", default="all")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=33)
    ap.add_argument("--layers", type=int, default=20)
    ap.add_argument("--seed", type=int, default=None, help="circuit seed (default 21 for complex128, 31 for complex64)")
    ap.add_argument("--dtype", default="c128")
    ap.add_argument("--method", default="auto", choices=["auto", "fused", "staged", "plain"],
                    help="auto: the autotuner times the candidate plans on the state (outside the timed region)")
    ap.add_argument("--fuse-k", type=int, default=5)
    ap.add_argument("--lds", type=int, default=0, help="resident qubits per LDS block (staged plans)")
    ap.add_argument("--lds-regs", type=int, default=0, help="log2 amplitudes per thread (staged plans)")
    ap.add_argument("--plain-runs", type=int, default=1, help="timed runs of the plain per-gate plan (0 = skip)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--cpu-n", type=int, default=27)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--renorm-every", type=int, default=None,
                    help="layers between FP64 renormalisations (default 10 for complex64, 0 = none for complex128)")
    args = ap.parse_args()
    if args.mode == "sweep":
        return sweep_mode(args)
    if args.mode == "batch":
        return batch_mode(args)
    if args.mode == "copycal":
        return copycal_mode(args)
    if args.mode == "paper":
        return paper_mode(args)

    if args.seed is None:
        args.seed = 31 if args.dtype == "c64" else 21
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (no sharding, no "
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
    renorm = args.renorm_every if args.renorm_every is not None else (10 if dtype == "c64" else 0)
    workload = f"brickwork-{n}q-{dtype}-{args.layers}layers" + (f"-renorm{renorm}" if renorm else "")
    log(f"workload {workload}: generating circuit")
    # one circuit per group of `renorm` layers (the whole circuit when renorm = 0); the draws of all
    # layers are made in the same order, so the groups concatenate to the full circuit
    groups = [(a, min(args.layers, a + renorm)) for a in range(0, args.layers, renorm)] if renorm else [(0, args.layers)]
    circs = [q.parse_circuit(wl.brickwork_circuit(n, args.layers, args.seed, layer_range=g)) for g in groups]
    G = sum(len(c.gates) for c in circs)
    log(f"{G} gates in {len(circs)} group(s); allocating {amp * 2 ** n / 2 ** 30:.0f} GiB state")
    state = q.State(n, dtype, device=dev)
    tuned = None
    if args.method == "auto":
        from paper_quant_ph_0608239_amd import tuning
        t0 = time.perf_counter()
        tuned = tuning.tune(circs[0], state, reps=1, include_plain=False, use_cache=False)
        log(f"autotune ({time.perf_counter() - t0:.1f} s): best {tuned['method']} k={tuned['fuse_k']} "
            f"lds={tuned['lds_qubits']}/{tuned['lds_regs']} {tuned['ms']:.1f} ms; tried "
            + ", ".join(f"{t['method']}:{t['fuse_k'] or ''}{t['lds_qubits'] or ''}/{t['lds_regs'] or ''}={t['ms']:.0f}"
                        for t in tuned["tried"]))
        popts = dict(method=tuned["method"], fuse_k=tuned["fuse_k"] or 5, lds_qubits=tuned["lds_qubits"],
                     lds_regs=tuned["lds_regs"])
    else:
        popts = dict(method=args.method, fuse_k=args.fuse_k, lds_qubits=args.lds, lds_regs=args.lds_regs)
    plans = [q.Plan(c, dtype, **popts) for c in circs]
    info = dict(plans[0].info)
    for k in ("gates", "launches", "passes", "alg_bytes", "alg_flops"):
        info[k] = sum(p.info[k] for p in plans)
    log(f"plan {popts}: {info}")
    norms = []

    def step(timed: bool):
        state.set_basis(0)
        ms, kd, fk = [], [], []
        for p in plans:
            if timed:
                a, b, c = p.execute_timed(state)
                ms.append(a)
                kd.append(b)
                fk.append(c)
            else:
                p.execute(state)
            if renorm:
                norms.append(state.renormalize())
        return (np.concatenate(ms), np.concatenate(kd), np.concatenate(fk)) if timed else None

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    norms.clear()
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
    plan_bytes = info["alg_bytes"]
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
        dom_name += f"_m{info['lds_qubits']}r{info['lds_regs']}"
    full_sweep_bytes = 2.0 * amp * 2 ** n
    kname = KERNEL_NAMES[dom_key[0]]
    dom_bytes = full_sweep_bytes  # fused blocks, staged passes and general sweeps read and write every amplitude
    if kname in ("fused_mfma", "fused_valu"):
        dom_flops = 8.0 * 2 ** (n + dom_key[1])
        mfma = kname == "fused_mfma"
        alu_peak = (FP64_PEAK_TFLOPS if dtype == "c128" else FP32_MFMA_PEAK_TFLOPS) if mfma else VALU_PEAK_TFLOPS
    elif kname == "staged":
        dom_flops = info["alg_flops"] / max(1, info["passes"])  # per pass, averaged over the passes
        mfma, alu_peak = False, VALU_PEAK_TFLOPS
    else:
        dom_flops, mfma, alu_peak = 0.0, False, VALU_PEAK_TFLOPS
    secs = dom_avg_ms / 1e3
    hbm_gbps = dom_bytes / secs / 1e9
    alu_tf = dom_flops / secs / 1e12
    t_hbm = dom_bytes / (HBM_PEAK_GBPS * 1e9)
    t_alu = dom_flops / (alu_peak * 1e12)
    traffic = load_traffic(workload, dom_name)
    if t_alu > t_hbm:
        roof = {"bound": "mfma" if mfma else "alu", "achieved": round(alu_tf, 2), "peak": alu_peak, "unit": "TFLOP/s",
                "frac": round(alu_tf / alu_peak, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(hbm_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(hbm_gbps / HBM_PEAK_GBPS, 4), "traffic": traffic}
    roof.update({"kernel": dom_name, "launches": len(dom_idx), "avg_launch_ms": round(dom_avg_ms, 3),
                 "alg_bytes_per_launch": dom_bytes, "alg_flops_per_launch": dom_flops,
                 "hbm_GBps": round(hbm_gbps, 1), "hbm_frac": round(hbm_gbps / HBM_PEAK_GBPS, 4)})
    if dom_flops:
        roof.update({"alu_TFLOPs": round(alu_tf, 2), "alu_peak": alu_peak, "alu_frac": round(alu_tf / alu_peak, 4),
                     "floor_ms": {"hbm": round(t_hbm * 1e3, 2), "alu": round(t_alu * 1e3, 2)}})

    out = {
        "metric": METRIC, "value": round(gates_per_s, 3), "unit": "gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if dtype == "c128" else "f32", "data": "synthetic",
        "config": {"workload": workload, "n_qubits": n, "state": dtype, "layers": args.layers, "gates": G,
                   "seed": args.seed, "method": ["plain", "fused", "staged"][int(info["method"])],
                   "fuse_k": int(info["fuse_k"]) or None, "lds_qubits": int(info["lds_qubits"]) or None,
                   "lds_regs": int(info["lds_regs"]) or None, "launches_per_step": int(info["launches"]),
                   "renormalise_every_layers": renorm or None,
                   "autotune": None if tuned is None else {
                       "choice": {k: tuned[k] for k in ("method", "fuse_k", "lds_qubits", "lds_regs")},
                       "tried_ms": {f"{t['method']}{'-k' + str(t['fuse_k']) if t['method'] == 'fused' else ''}"
                                    f"{'-m' + str(t['lds_qubits']) + 'r' + str(t['lds_regs']) if t['method'] == 'staged' else ''}":
                                    round(t["ms"], 1) for t in tuned["tried"]}}},
        "eff_GBps": round(eff_gbps, 1), "hbm_frac": round(eff_gbps / HBM_PEAK_GBPS, 4),
        "roofline": roof,
    }
    if renorm:
        # FP64 norms just before each renormalisation, last timed step
        last = norms[-len(plans):]
        out["norm_before_renormalisation"] = last
        out["max_norm_drift"] = max(abs(x - 1.0) for x in last)

    # the plain per-gate plan, timed beside it
    if args.plain_runs > 0:
        pplans = [q.Plan(c, dtype, method="plain") for c in circs]
        pbytes = sum(p.info["alg_bytes"] for p in pplans)
        pms = []
        pk = None
        for r in range(args.plain_runs):
            state.set_basis(0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            parts = []
            for p in pplans:
                parts.append(p.execute_timed(state))
                if renorm:
                    state.renormalize()
            torch.cuda.synchronize()
            ms = np.concatenate([m for m, _, _ in parts])
            pk = np.concatenate([k for _, k, _ in parts])
            pms.append((time.perf_counter() - t1, ms))
            log(f"plain run {r + 1}/{args.plain_runs}: {pms[-1][0]:.2f} s")
        pwall = float(np.mean([w for w, _ in pms]))
        pl = np.mean(np.stack([m for _, m in pms]), axis=0)
        gen = [i for i, kd in enumerate(pk) if kd == 0]
        gen_ms = float(pl[gen].mean()) if gen else None
        out["plain"] = {
            "gates_per_s": round(G / pwall, 3), "s_per_run": round(pwall, 3),
            "eff_GBps": round(pbytes / pwall / 1e9, 1),
            "hbm_frac": round(pbytes / pwall / 1e9 / HBM_PEAK_GBPS, 4),
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
