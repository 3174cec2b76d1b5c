"""Benchmark: gates/s and effective HBM bandwidth of the state-vector gate engine on one MI355X.

Default workload: the 33-qubit complex128 brickwork circuit (128 GiB state, 20 layers of Haar-random
2x2 unitaries on every qubit + CZ on alternating neighbour pairs, 980 gates, seed 21, start
|0...0>). A step is one full run of the circuit from |0...0> through the framework's fastest plan
(the initial state is generated inside the first pass); the plain per-gate plan (one sweep per gate)
and the fused plan (5-qubit dense blocks on the FP64 matrix cores) are each timed whole beside it.

Prints ONE JSON line (rank 0). `value` is gates/s of the whole job (one GPU) with the state already
resident in HBM. `roofline` describes the dominant kernel of the timed plan, its average launch
duration measured with HIP events on the state's stream over the timed steps. `cpu_baseline` is the
FP64 CPU oracle run on whole circuits of the same family at sizes it finishes in seconds (28 qubits
on all host threads, 20 qubits on one), measured, with the GPU timed on the same 28-qubit circuit.
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
# vector ALU, published: FP64 78.6 TFLOP/s = 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz;
# FP32 157.3 TFLOP/s, which needs packed (two-wide) FP32 instructions
FP64_VALU_PEAK_TFLOPS = 78.6
FP32_VALU_PEAK_TFLOPS = 157.3
# the FP32 rate without packed instructions (the code here is compiled without them)
FP32_UNPACKED_PEAK_TFLOPS = 78.6
METRIC = "gates/s & effective HBM GB/s (% of peak) at 30–34 qubits; fused vs plain"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


KERNEL_SOURCES = {"staged": ("staged.hip", "staged_device.h", "staged_kernels.h", "staged_k128.hip", "staged_k128w.hip",
                             "staged_k64.hip", "staged_k64w.hip", "qsim_internal.h"),
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


def _oracle_run_json(n: int, layers: int, seed: int):
    """Whole-circuit oracle run of the brickwork family in this process (its OpenMP threads as the
    environment sets them); wall time around the gate loop only."""
    import oracle
    import qsim_workloads as wl
    oracle.lib()
    text = wl.brickwork_circuit(n, layers, seed)
    psi, secs, gates = oracle.timed_run(text)
    return {"n": n, "gates": gates, "seconds": secs, "threads": oracle.threads()}, psi


def cpu_baseline(args, popts: dict, dtype: str) -> dict:
    """The oracle, unmodified, on whole circuits of the benchmark's family at sizes it finishes in
    seconds: on every host thread at args.cpu_n qubits (the GPU plan is timed on the same circuit in
    the same run and checked against the oracle's state), and on one thread at args.cpu_n1 qubits.
    Rates are the measured ones, with no scaling to other sizes."""
    import subprocess

    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    import qsim_workloads as wl
    n, layers, seed = args.cpu_n, args.layers, args.seed
    full, psi = _oracle_run_json(n, layers, seed)
    circ = q.parse_circuit(wl.brickwork_circuit(n, layers, seed))
    plain = q.Plan(circ, "c128", method="plain")
    alg_bytes = plain.info["alg_bytes"]  # the per-gate sweeps the oracle performs, in bytes moved
    plain.close()
    # the same circuit on the GPU, through the benchmark's plan options (complex128 at this size)
    gpu = {}
    s = q.State(n, "c128")
    opts = dict(popts)
    if opts["method"] == "staged" and dtype != "c128":
        opts.update(lds_qubits=0, lds_regs=0)
    p = q.Plan(circ, "c128", **opts)
    p.execute_from_zero(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        p.execute_from_zero(s)
    torch.cuda.synchronize()
    gsecs = (time.perf_counter() - t0) / reps
    d = float(np.max(np.abs(s.download() - psi)))
    gpu = {"method": opts["method"], "seconds": round(gsecs, 5), "gates_per_s": round(full["gates"] / gsecs, 1),
           "max_abs_diff_vs_oracle": d}
    p.close()
    s.close()
    del s, psi
    # one thread, in a child process (OpenMP reads its thread count at start-up)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, %r); import bench; r, _ = bench._oracle_run_json(%d, %d, %d); "
            "print(json.dumps(r))" % (ROOT, args.cpu_n1, layers, seed))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, check=True)
    one = json.loads(r.stdout.strip().splitlines()[-1])
    c1 = q.parse_circuit(wl.brickwork_circuit(args.cpu_n1, layers, seed))
    p1 = q.Plan(c1, "c128", method="plain")
    bytes1 = p1.info["alg_bytes"]
    p1.close()
    rate = full["gates"] / full["seconds"]
    return {"value": round(rate, 3), "unit": "gates/s", "cores": full["threads"], "kind": "oracle",
            "sample": f"the whole {n}-qubit complex128 brickwork circuit of the same family (20 layers, seed {seed}, "
                      f"{full['gates']} gates) from |0...0>, measured: {full['seconds']:.2f} s on {full['threads']} "
                      f"threads; no scaling to other sizes",
            "n_qubits": n, "seconds": round(full["seconds"], 3), "GBps": round(alg_bytes / full["seconds"] / 1e9, 2),
            "gpu_same_circuit": gpu, "gpu_speedup_same_circuit": round(full["seconds"] / gsecs, 1),
            "one_thread": {"n_qubits": args.cpu_n1, "gates": one["gates"], "seconds": round(one["seconds"], 3),
                           "gates_per_s": round(one["gates"] / one["seconds"], 3),
                           "GBps": round(bytes1 / one["seconds"] / 1e9, 3), "threads": one["threads"]}}


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
    """Many independent circuits (2048 seeded circuits, n uniform in 10..22, 50 random gates each) run
    from |0...0> as one HIP graph on a stream of their own: circuits/s, gates/s and per-circuit latency
    percentiles from device timestamps. The batch's LDS block shape is autotuned first (each candidate
    built, run and timed, outside the timed region) unless --lds is given. One JSON line."""
    import numpy as np
    import torch

    import paper_quant_ph_0608239_amd as q
    import qsim_workloads as wl
    from paper_quant_ph_0608239_amd import tuning
    texts = wl.batch_circuits(count=args.count, nmin=10, nmax=22, depth=50, seed=41)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        tuned = None
        if args.lds:
            shape = (args.lds, args.lds_regs or 4)
        else:
            t0 = time.perf_counter()
            tuned = tuning.tune_batch(texts, args.dtype, reps=2)
            shape = (tuned["lds_qubits"], tuned["lds_regs"])
            log(f"batch autotune ({time.perf_counter() - t0:.1f} s): m={shape[0]} r={shape[1]}; tried " +
                ", ".join(f"m{t['lds_qubits']}r{t['lds_regs']}={t['ms']:.2f}" for t in tuned["tried"]))
        b = q.Batch(texts, args.dtype, lds_qubits=shape[0], lds_regs=shape[1], use_graph=True)
        for _ in range(max(1, args.warmup)):
            b.run()
        runs = [b.run() for _ in range(args.steps)]
    ms = float(np.mean([r["launch_ms"] for r in runs]))
    lat = b.latencies_us()
    out = {"metric": "circuits/s (batch of independent circuits, one graph launch)", "value": round(args.count / ms * 1e3, 1),
           "unit": "circuits/s", "gates_per_s": round(b.total_gates / ms * 1e3, 1), "ms_per_run": round(ms, 3),
           "latency_us": {"p50": round(float(np.percentile(lat, 50)), 1), "p99": round(float(np.percentile(lat, 99)), 1),
                          "max": round(float(lat.max()), 1)},
           "config": {"workload": f"batch-{args.count}-circuits-n10-22-depth50-{args.dtype}", "count": args.count,
                      "gates": b.total_gates, "seed": 41, "lds_qubits": shape[0], "lds_regs": shape[1],
                      "split_circuits": b.info["split_circuits"], "launch_steps": b.info["steps"],
                      "kernel_launches": b.info["launches"], "graph": True,
                      "autotune": None if tuned is None else {
                          "choice": {"lds_qubits": shape[0], "lds_regs": shape[1]},
                          "tried_ms": {f"m{t['lds_qubits']}r{t['lds_regs']}": round(t["ms"], 3) for t in tuned["tried"]}}},
           "dtype": "f64" if args.dtype == "c128" else "f32"}
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
    ap.add_argument("--fused-runs", type=int, default=1, help="timed runs of the fused k = 5 plan (0 = skip)")
    ap.add_argument("--cpu-n", type=int, default=28, help="qubits of the oracle run on all host threads")
    ap.add_argument("--cpu-n1", type=int, default=20, help="qubits of the one-thread oracle run")
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
    # one circuit; with renormalisation a RENORM point after every `renorm` layers (the plan folds each
    # into the passes around it)
    points = tuple(range(renorm, args.layers + 1, renorm)) if renorm else ()
    circs = [q.parse_circuit(wl.brickwork_circuit(n, args.layers, args.seed, renorm_after=points))]
    G = sum(1 for c in circs for g in c.gates if g.op != q._lib.OPS["RENORM"])
    log(f"{G} gates, {len(points)} renormalisation point(s); allocating {amp * 2 ** n / 2 ** 30:.0f} GiB state")
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
    for k in ("gates", "launches", "passes", "alg_bytes", "alg_flops", "issued_flops"):
        info[k] = sum(p.info[k] for p in plans)
    info["gates"] = G
    log(f"plan {popts}: {info}")

    def run(pl, timed: bool):
        """One run of the circuit from |0...0> (a staged plan generates the initial state inside its
        first pass), renormalising in FP64 at its RENORM points."""
        ms, kd, fk = [], [], []
        for i, p in enumerate(pl):
            if timed:
                a, b, c = p.execute_timed(state, from_zero=(i == 0))
                ms.append(a)
                kd.append(b)
                fk.append(c)
            elif i == 0:
                p.execute_from_zero(state)
            else:
                p.execute(state)
        return (np.concatenate(ms), np.concatenate(kd), np.concatenate(fk)) if timed else None

    for i in range(args.warmup):
        run(plans, False)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    launch_ms, kinds, fks = [], None, None
    for i in range(args.steps):
        ms, kinds, fks = run(plans, True)
        launch_ms.append(ms)
        log(f"step {i + 1}/{args.steps}: {ms.sum():.1f} ms in {len(ms)} launches")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    gates_per_s = G / (wall / args.steps)
    run_bytes = info["alg_bytes"] - (amp * 2 ** n if int(info["method"]) == 2 else 0)  # the first pass reads nothing
    eff_gbps = run_bytes / (wall / args.steps) / 1e9
    roof = roofline(np.stack(launch_ms), kinds, fks, info, n, dtype, workload, zero_first=True)

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
        # FP64 squared norms found at the renormalisation points in the last timed step
        last = [float(x) for p in plans for x in p.norms()]
        out["norm_before_renormalisation"] = last
        out["max_norm_drift"] = max(abs(x - 1.0) for x in last)
        out["config"]["renormalisation"] = ("folded into the staged passes around each point; a scaling sweep after the "
                                            "last" if info["method"] == 2 else "a norm sweep and a scaling sweep per point")

    # the plain per-gate plan (one sweep per gate) and the fused k = 5 plan (dense 32 x 32 blocks on
    # the matrix cores), each timed whole beside the headline plan
    full_sweep_bytes = 2.0 * amp * 2 ** n
    for leg, legopts, runs in (("plain", dict(method="plain"), args.plain_runs),
                               ("fused", dict(method="fused", fuse_k=5), args.fused_runs)):
        if runs <= 0 or (leg == popts["method"] and leg != "fused"):
            continue
        lplans = [q.Plan(c, dtype, **legopts) for c in circs]
        lbytes = sum(p.info["alg_bytes"] for p in lplans)
        walls, lms, lk, lf = [], [], None, None
        for r in range(runs):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ms, lk, lf = run(lplans, True)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t1)
            lms.append(ms)
            log(f"{leg} run {r + 1}/{runs}: {walls[-1]:.2f} s in {len(ms)} launches")
        lwall = float(np.mean(walls))
        linfo = dict(lplans[0].info)
        for k in ("gates", "launches", "passes", "alg_bytes", "alg_flops", "issued_flops"):
            linfo[k] = sum(p.info[k] for p in lplans)
        entry = {"gates_per_s": round(G / lwall, 3), "s_per_run": round(lwall, 3), "launches": int(linfo["launches"]),
                 "eff_GBps": round(lbytes / lwall / 1e9, 1), "hbm_frac": round(lbytes / lwall / 1e9 / HBM_PEAK_GBPS, 4),
                 "roofline": roofline(np.stack(lms), lk, lf, linfo, n, dtype, workload)}
        if leg == "plain":
            L = np.mean(np.stack(lms), axis=0)
            gen = [i for i, kd in enumerate(lk) if kd == 0]
            gen_ms = float(L[gen].mean()) if gen else None
            entry["general_sweep_avg_ms"] = round(gen_ms, 3) if gen_ms else None
            entry["general_sweep_GBps"] = round(full_sweep_bytes / (gen_ms / 1e3) / 1e9, 1) if gen_ms else None
        out[leg] = entry
        out[f"speedup_vs_{leg}"] = round(gates_per_s / (G / lwall), 2)
        for p in lplans:
            p.close()

    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(args, popts, dtype)
    print(json.dumps(out), flush=True)
    return 0


def roofline(L, kinds, fks, info, n, dtype, workload, zero_first=False) -> dict:
    """The dominant kernel of a plan (the class, and fused width, with the most total time over the
    timed runs) against the bound that limits it. L: runs x launches of HIP-event durations (ms).
    Algorithmic work per launch: a staged pass or fused block reads and writes all 2^n amplitudes
    once (with zero_first, the first staged pass of the run generates |0...0> and only writes); a
    fused k-qubit block does 8 * 2^(n+k) flops on the matrix cores; a staged pass does the plan's 2x2
    flops (14 per amplitude per dense 2x2) divided over its passes."""
    import numpy as np

    from paper_quant_ph_0608239_amd._lib import KERNEL_NAMES
    amp = 16 if dtype == "c128" else 8
    avg = L.mean(axis=0)
    classes = {}
    for i, (kd, fk) in enumerate(zip(kinds, fks)):
        classes.setdefault((int(kd), int(fk)), []).append(i)
    key = max(classes, key=lambda k: avg[classes[k]].sum())
    idx = classes[key]
    dom_ms = float(avg[idx].mean())
    kname = KERNEL_NAMES[key[0]]
    name = kname + (f"_k{key[1]}" if key[1] else "")
    if kname == "staged":
        name += f"_m{info['lds_qubits']}r{info['lds_regs']}"
    dom_bytes = 2.0 * amp * 2 ** n
    if zero_first and kname == "staged" and 0 in idx:
        # a run from |0...0>: the first pass generates the state and reads nothing
        dom_bytes = amp * 2 ** n * (2.0 * len(idx) - 1.0) / len(idx)
    issued = None
    if kname in ("fused_mfma", "fused_valu"):
        flops = 8.0 * 2 ** (n + key[1])
        mfma = kname == "fused_mfma"
        peak = (FP64_PEAK_TFLOPS if dtype == "c128" else FP32_MFMA_PEAK_TFLOPS) if mfma else \
            (FP64_VALU_PEAK_TFLOPS if dtype == "c128" else FP32_VALU_PEAK_TFLOPS)
    elif kname == "staged":
        flops = info["alg_flops"] / len(idx)  # over the staged passes (not the renormalisation sweeps)
        mfma = False
        peak = FP64_VALU_PEAK_TFLOPS if dtype == "c128" else FP32_VALU_PEAK_TFLOPS
        # the flops the kernels actually issue (the plan's count: 2x2s with a real first column and
        # two-qubit blocks issue fewer than the algorithmic 14 per amplitude per 2x2); complex64 code has
        # no packed FP32 instructions, so it can issue at most half the published FP32 vector rate
        issued = {"flops_per_launch": info["issued_flops"] / len(idx), "frac_of_peak": None,
                  "peak_as_compiled": FP64_VALU_PEAK_TFLOPS if dtype == "c128" else FP32_UNPACKED_PEAK_TFLOPS}
    else:
        flops, mfma, peak = 0.0, False, FP64_VALU_PEAK_TFLOPS
    secs = dom_ms / 1e3
    gbps = dom_bytes / secs / 1e9
    tf = flops / secs / 1e12
    t_hbm = dom_bytes / (HBM_PEAK_GBPS * 1e9)
    t_alu = flops / (peak * 1e12)
    traffic = load_traffic(workload, name)
    if t_alu > t_hbm:
        roof = {"bound": "mfma" if mfma else "alu", "achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tf / peak, 4), "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": traffic}
    roof.update({"kernel": name, "launches": len(idx), "avg_launch_ms": round(dom_ms, 3),
                 "alg_bytes_per_launch": dom_bytes, "alg_flops_per_launch": flops,
                 "hbm_GBps": round(gbps, 1), "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4)})
    if flops:
        roof.update({"alu_TFLOPs": round(tf, 2), "alu_peak": peak, "alu_frac": round(tf / peak, 4),
                     "floor_ms": {"hbm": round(t_hbm * 1e3, 2), "alu": round(t_alu * 1e3, 2)}})
    if issued:
        itf = issued["flops_per_launch"] / secs / 1e12
        issued["TFLOPs"] = round(itf, 2)
        issued["frac_of_peak"] = round(itf / peak, 4)
        issued["frac_as_compiled"] = round(itf / issued["peak_as_compiled"], 4)
        roof["issued"] = issued
    return roof


if __name__ == "__main__":
    sys.exit(main())
