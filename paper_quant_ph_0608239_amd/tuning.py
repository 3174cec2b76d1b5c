"""Autotuning of the plan method and its parameters (fusion width k, LDS block size, amplitudes
per thread), with an on-disk JSON cache.

The timing itself runs in libqsim (qsim_plan_tune): every candidate plan is executed on a scratch
state of the same size with HIP events around it. This module keys and stores the results.
Cache file: $QSIM_TUNE_CACHE, else ~/.cache/qsim_tune.json.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import os

from . import _lib
from ._lib import check, lib

_METHOD_NAMES = {0: "plain", 1: "fused", 2: "staged"}


def cache_path() -> str:
    return os.environ.get("QSIM_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "qsim_tune.json"))


def circuit_key(circuit, dtype: int) -> str:
    """State size, dtype and a hash of the gate list (op, qubits, controls; not the angle values,
    which do not change the schedule)."""
    h = hashlib.sha256()
    for g in circuit.gates:
        h.update(bytes(f"{g.op},{g.target},{g.target2},{g.controls};", "ascii"))
    return f"n{circuit.n}-d{dtype}-{h.hexdigest()[:16]}"


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def opts_to_dict(o) -> dict:
    return {"method": _METHOD_NAMES.get(o.method, str(o.method)), "fuse_k": o.fuse_k, "lds_qubits": o.lds_qubits,
            "lds_regs": o.lds_regs}


def tune(circuit, scratch, reps: int = 1, include_plain: bool = False, use_cache: bool = True) -> dict:
    """Best plan options for `circuit` on states like `scratch` (whose contents are overwritten).
    Returns {"method", "fuse_k", "lds_qubits", "lds_regs", "ms", "tried": [...], "cached": bool}."""
    key = circuit_key(circuit, scratch.dtype)
    db = _load() if use_cache else {}
    if use_cache and key in db:
        r = dict(db[key])
        r["cached"] = True
        return r
    best = _lib.PlanOpts()
    best_ms = ctypes.c_double()
    maxt = 16
    tried = (_lib.PlanOpts * maxt)()
    tried_ms = (ctypes.c_double * maxt)()
    nt = ctypes.c_int()
    check(lib().qsim_plan_tune(circuit.n, scratch.dtype, circuit.gate_array(), len(circuit.gates), scratch.handle,
                               int(reps), int(include_plain), ctypes.byref(best), ctypes.byref(best_ms), tried, tried_ms,
                               maxt, ctypes.byref(nt)))
    r = opts_to_dict(best)
    r["ms"] = best_ms.value
    r["tried"] = [dict(opts_to_dict(tried[i]), ms=tried_ms[i]) for i in range(min(nt.value, maxt))]
    if use_cache:
        db[key] = r
        _store(db)
    r = dict(r)
    r["cached"] = False
    return r


# LDS block shapes (resident qubits, log2 amplitudes per thread) that a batch can use, per dtype
BATCH_SHAPES = {1: [(12, 4), (11, 4), (11, 3)], 0: [(12, 4), (11, 4), (13, 5)]}


def tune_batch(circuits, dtype, reps: int = 2, use_cache: bool = False) -> dict:
    """The fastest LDS block shape for a batch of circuits: each candidate batch is built, run once
    (warm-up) and timed over `reps` runs (HIP events around each run) on the current stream. Returns
    {"lds_qubits", "lds_regs", "ms", "tried": [...]}; cached by the circuits' gate lists if use_cache."""
    import numpy as np

    from . import Batch, dtype_code, parse_circuit
    cs = [parse_circuit(c) if isinstance(c, str) else c for c in circuits]
    code = dtype_code(dtype)
    h = hashlib.sha256()
    for c in cs:
        h.update(bytes(f"{c.n}:{circuit_key(c, code)};", "ascii"))
    key = f"batch-d{code}-{h.hexdigest()[:16]}"
    db = _load() if use_cache else {}
    if use_cache and key in db:
        return dict(db[key], cached=True)
    tried = []
    for m, r in BATCH_SHAPES[code]:
        b = Batch(cs, code, lds_qubits=m, lds_regs=r)
        try:
            b.run()
            ms = float(np.mean([b.run()["launch_ms"] for _ in range(reps)]))
        finally:
            b.close()
        tried.append({"lds_qubits": m, "lds_regs": r, "ms": ms})
    best = min(tried, key=lambda t: t["ms"])
    out = {"lds_qubits": best["lds_qubits"], "lds_regs": best["lds_regs"], "ms": best["ms"], "tried": tried}
    if use_cache:
        db[key] = out
        _store(db)
    return dict(out, cached=False)
