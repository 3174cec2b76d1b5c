"""MI355X (gfx950) state-vector gate engine: Python binding of libqsim.so.

The binding only marshals arguments: every step of the gate path runs in the HIP kernels of
libqsim.so. PyTorch provides device memory (the amplitudes live in a torch tensor that the library
wraps) and the HIP stream the work is issued on.

Qubit q is bit q of the amplitude index; amplitudes are stored interleaved (re, im).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from ._lib import (PLAN_AUTO, PLAN_FUSED, PLAN_PLAIN, PLAN_STAGED, QSIM_C64, QSIM_C128, STAGED_FULL, STAGED_HALF,
                   STAGED_WAVE, Gate, QsimError, check, lib)
from .circuit import Circuit, parse_circuit

__all__ = ["State", "Plan", "Batch", "Circuit", "parse_circuit", "QsimError", "lib", "dtype_code",
           "PLAN_PLAIN", "PLAN_FUSED", "PLAN_STAGED", "PLAN_AUTO", "QSIM_C64", "QSIM_C128",
           "STAGED_FULL", "STAGED_HALF", "STAGED_WAVE", "KERNEL_STAGED", "KERNEL_FUSED_MFMA",
           "KERNEL_RENORM"]

KERNEL_STAGED = 6
KERNEL_FUSED_MFMA = 5
KERNEL_RENORM = 7


def dtype_code(dtype) -> int:
    if dtype in (QSIM_C64, QSIM_C128):
        return int(dtype)
    d = str(dtype).lower()
    if d in ("c64", "complex64"):
        return QSIM_C64
    if d in ("c128", "complex128"):
        return QSIM_C128
    raise ValueError(f"unknown dtype {dtype!r}")


def _u8(U) -> ctypes.Array:
    u = np.asarray(U, dtype=np.complex128).reshape(2, 2)
    flat = u.reshape(-1).view(np.float64)
    return (ctypes.c_double * 8)(*flat.tolist())


def _stream_ptr(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class State:
    """A state of n qubits in device memory owned by a torch tensor (interleaved re/im)."""

    def __init__(self, n: int, dtype="c128", device="cuda:0"):
        import torch
        self.n = int(n)
        self.dtype = dtype_code(dtype)
        self.device = torch.device(device)
        rt = torch.float64 if self.dtype == QSIM_C128 else torch.float32
        with torch.cuda.device(self.device):
            self.tensor = torch.empty(2 ** (self.n + 1), dtype=rt, device=self.device)
            h = ctypes.c_void_p()
            check(lib().qsim_wrap(ctypes.c_void_p(self.tensor.data_ptr()), self.n, self.dtype,
                                  _stream_ptr(self.device), ctypes.byref(h)))
        self.handle = h
        self.set_basis(0)

    # -- lifetime
    def close(self):
        if getattr(self, "handle", None):
            lib().qsim_free(self.handle)
            self.handle = None
        self.tensor = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def amp_bytes(self) -> int:
        return 16 if self.dtype == QSIM_C128 else 8

    @property
    def nbytes(self) -> int:
        return self.amp_bytes << self.n

    # -- contents
    def set_basis(self, x: int = 0):
        check(lib().qsim_set_basis(self.handle, int(x)))

    def upload(self, psi: np.ndarray):
        cd = np.complex128 if self.dtype == QSIM_C128 else np.complex64
        a = np.ascontiguousarray(np.asarray(psi, dtype=cd))
        if a.size != 2 ** self.n:
            raise ValueError("state size mismatch")
        check(lib().qsim_upload(self.handle, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))

    def download(self) -> np.ndarray:
        cd = np.complex128 if self.dtype == QSIM_C128 else np.complex64
        out = np.empty(2 ** self.n, dtype=cd)
        check(lib().qsim_download(self.handle, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def sync(self):
        check(lib().qsim_sync(self.handle))

    # -- gates
    def apply_1q(self, target: int, U):
        check(lib().qsim_apply_1q(self.handle, int(target), _u8(U)))

    def apply_ctrl(self, controls, target: int, U):
        check(lib().qsim_apply_ctrl(self.handle, _mask(controls), int(target), _u8(U)))

    def apply_phase(self, controls, target: int, theta: float):
        check(lib().qsim_apply_phase(self.handle, _mask(controls), int(target), float(theta)))

    def apply_swap(self, q0: int, q1: int, controls=0):
        check(lib().qsim_apply_swap(self.handle, _mask(controls), int(q0), int(q1)))

    def apply_fused(self, qubits, U):
        q = [int(x) for x in qubits]
        k = len(q)
        Ua = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).reshape(2 ** k, 2 ** k)
        flat = Ua.reshape(-1).view(np.float64)
        check(lib().qsim_apply_fused(self.handle, k, (ctypes.c_int * k)(*q),
                                     flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def apply_modexp(self, x_first: int, x_qubits: int, f_first: int, f_qubits: int, y: int, G: int):
        """|x>|z> -> |x>|z XOR (y^x mod G)> (Shor's conditional operation; asynchronous)."""
        check(lib().qsim_apply_modexp(self.handle, int(x_first), int(x_qubits), int(f_first), int(f_qubits),
                                      int(y), int(G)))

    # -- reductions
    def norm(self) -> float:
        v = ctypes.c_double()
        check(lib().qsim_norm(self.handle, ctypes.byref(v)))
        return v.value

    def probs(self, device: bool = False):
        if device:
            import torch
            out = torch.empty(2 ** self.n, dtype=torch.float64, device=self.device)
            check(lib().qsim_probs(self.handle, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        out = np.empty(2 ** self.n, dtype=np.float64)
        check(lib().qsim_probs(self.handle, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def marginals(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        check(lib().qsim_marginals(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def renormalize(self) -> float:
        v = ctypes.c_double()
        check(lib().qsim_renormalize(self.handle, ctypes.byref(v)))
        return v.value

    def sample(self, uniforms) -> np.ndarray:
        u = np.ascontiguousarray(np.asarray(uniforms, dtype=np.float64))
        out = np.empty(u.size, dtype=np.uint64)
        check(lib().qsim_sample(self.handle, u.size, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
        return out

    def run(self, circuit, method="plain", **kw):
        """Lower the circuit to a plan and execute it on this state (asynchronous)."""
        c = parse_circuit(circuit) if isinstance(circuit, str) else circuit
        p = Plan(c, self.dtype, method=method, **kw)
        p.execute(self)
        return p


def _mask(controls) -> int:
    if isinstance(controls, (list, tuple, set)):
        m = 0
        for c in controls:
            m |= 1 << int(c)
        return m
    return int(controls)


_METHODS = {"plain": PLAN_PLAIN, "fused": PLAN_FUSED, "staged": PLAN_STAGED, "auto": PLAN_AUTO}


class Plan:
    """A circuit lowered once to kernel launches (plain sweeps, fused k-qubit gates or LDS passes)."""

    def __init__(self, circuit: Circuit, dtype="c128", method="plain", fuse_k: int = 5, lds_qubits: int = 0,
                 use_graph: bool = False, lds_regs: int = 0):
        self.n = circuit.n
        self.dtype = dtype_code(dtype)
        opts = _lib.PlanOpts(_METHODS[method] if isinstance(method, str) else int(method), int(fuse_k),
                             int(lds_qubits), int(bool(use_graph)), int(lds_regs))
        arr = circuit.gate_array()
        h = ctypes.c_void_p()
        check(lib().qsim_plan_create(self.n, self.dtype, arr, len(circuit.gates), ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h
        info = _lib.PlanInfo()
        check(lib().qsim_plan_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _lib.PlanInfo._fields_}

    def execute(self, state: State):
        check(lib().qsim_plan_execute(self.handle, state.handle))

    def execute_from_zero(self, state: State):
        """Run the circuit from |0...0> (the state's contents are ignored; a staged plan generates the
        initial state in its first pass)."""
        check(lib().qsim_plan_execute_from_zero(self.handle, state.handle))

    def norms(self) -> np.ndarray:
        """FP64 squared norms found at the circuit's RENORM points by the latest execution (waits for it)."""
        R = int(self.info["renorms"])
        out = np.zeros(max(R, 1), dtype=np.float64)
        check(lib().qsim_plan_get_norms(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), R))
        return out[:R]

    def launches(self):
        """(kind, variant) numpy arrays, one entry per launch, without running the plan: the kernel
        class of each launch, and its fused width or staged form (STAGED_FULL / HALF / WAVE)."""
        L = int(self.info["launches"])
        kind = np.zeros(max(L, 1), dtype=np.int32)
        var = np.zeros(max(L, 1), dtype=np.int32)
        check(lib().qsim_plan_launches(self.handle, kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       var.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return kind[:L], var[:L]

    def execute_timed(self, state: State, from_zero: bool = False):
        """Execute (from |0...0> if from_zero) with HIP events around every launch (synchronises).
        Returns (ms, kind, fused_k) numpy arrays, one entry per launch."""
        L = int(self.info["launches"])
        ms = np.zeros(max(L, 1), dtype=np.float64)
        kind = np.zeros(max(L, 1), dtype=np.int32)
        fk = np.zeros(max(L, 1), dtype=np.int32)
        check(lib().qsim_plan_execute_timed(self.handle, state.handle, int(bool(from_zero)),
                                            ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            kind.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            fk.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return ms[:L], kind[:L], fk[:L]

    def close(self):
        if getattr(self, "handle", None):
            lib().qsim_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent small circuits run from |0...0> in one persistent launch."""

    def __init__(self, circuits: list, dtype="c64", device="cuda:0", lds_qubits: int = 0, lds_regs: int = 0,
                 use_graph: bool = False):
        import torch
        cs = [parse_circuit(c) if isinstance(c, str) else c for c in circuits]
        self.count = len(cs)
        self.nqubits = [c.n for c in cs]
        self.dtype = dtype_code(dtype)
        offs = [0]
        gates = []
        for c in cs:
            gates.extend(c.gates)
            offs.append(len(gates))
        self.total_gates = len(gates)  # gates over all circuits
        garr = (Gate * max(1, len(gates)))(*gates)
        nq = (ctypes.c_int * self.count)(*self.nqubits)
        of = (ctypes.c_int64 * (self.count + 1))(*offs)
        h = ctypes.c_void_p()
        opts = _lib.PlanOpts(PLAN_STAGED, 0, int(lds_qubits), int(bool(use_graph)), int(lds_regs))
        with torch.cuda.device(torch.device(device)):
            check(lib().qsim_batch_create(self.count, nq, of, garr, self.dtype, ctypes.byref(opts),
                                          _stream_ptr(torch.device(device)), ctypes.byref(h)))
        self.handle = h
        info = _lib.BatchInfo()
        check(lib().qsim_batch_get_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in _lib.BatchInfo._fields_}

    def run(self) -> dict:
        st = _lib.BatchStats()
        check(lib().qsim_batch_run(self.handle, ctypes.byref(st)))
        return {"launch_ms": st.launch_ms, "circuits": st.circuits, "gates": st.gates}

    def latencies_us(self) -> np.ndarray:
        out = np.empty(self.count, dtype=np.float64)
        check(lib().qsim_batch_latencies(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def download(self, c: int) -> np.ndarray:
        cd = np.complex128 if self.dtype == QSIM_C128 else np.complex64
        out = np.empty(2 ** self.nqubits[c], dtype=cd)
        check(lib().qsim_batch_download(self.handle, int(c), out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def close(self):
        if getattr(self, "handle", None):
            lib().qsim_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
