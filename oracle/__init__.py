"""Plain FP64 CPU oracle for the state-vector gate engine.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package. The GPU product path never imports, links or calls it, and this package
imports nothing from the product package.

The update rules live in ``qsim_oracle.c`` (plain loops over the index, one per equation of the
paper's Sec. III.A). This file parses the circuit text (its own parser), turns each gate name into
the rule the paper gives for it and calls that rule gate by gate, in file order, with no fusion,
no reordering, and no renormalisation except where the circuit asks for one.

Gate readings (the paper's notation on the left):
  H                      Eq. Hadamard / NUM2                 -> or_hadamard
  X, X-bar (RX90, RX90DG) Eq. Xoperation / NUM3 (pi/2 x-rotation) -> or_xrot
  Y, Y-bar (RY90, RY90DG) Eq. Yoperation / NUM4 (pi/2 y-rotation) -> or_yrot
  R(phi) (R, RK, RKDG)   Eq. singlephase / NUM5             -> or_phase
  controlled R (CPHASE, CRK, CRKDG)  Eq. COMM5              -> or_phase with a control mask
  CNOT                   Eq. CNOT2 / NUM6                    -> or_cnot
  controlled V (CV)      Eq. COMM4 / NUM7                    -> or_cv
  Toffoli (TOFFOLI)      Eq. Toffoli / NUM8                  -> or_cnot with two controls
  Pauli X, Y, Z, S, T, RZ, CZ, explicit U: 2x2 matrices applied with the common form of NUM2-NUM8
  (or_unitary); Pauli X uses the flip rule of NUM6 without a control.
  RENORM                 Eq. STAT1: every amplitude divided by the square root of sum |a_i|^2
                         (or_norm, FP64); a state whose sum is 0 is left as it is
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qsim_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no fused multiply-add contraction, no fast-math, OpenMP."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i32, u64, f64 = ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        sigs = {
            "or_hadamard": [dp, i32, i32],
            "or_xrot": [dp, i32, i32, i32],
            "or_yrot": [dp, i32, i32, i32],
            "or_phase": [dp, i32, i32, u64, f64],
            "or_cnot": [dp, i32, u64, i32],
            "or_cv": [dp, i32, u64, i32, f64],
            "or_unitary": [dp, i32, i32, u64, dp],
            "or_swap": [dp, i32, i32, i32],
            "or_dense": [dp, i32, i32, ctypes.POINTER(ctypes.c_int), dp],
            "or_probs": [dp, i32, dp],
            "or_norm": [dp, i32],
            "or_marginals": [dp, i32, dp],
            "or_threads": [],
            "or_modexp": [dp, i32, i32, i32, i32, i32, u64, u64],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = f64 if name == "or_norm" else (i32 if name == "or_threads" else None)
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops use on this host."""
    return int(lib().or_threads())


def _dp(x: np.ndarray):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _u8(u: np.ndarray) -> np.ndarray:
    """2x2 complex -> 8 doubles {u00r, u00i, u01r, u01i, u10r, u10i, u11r, u11i}."""
    u = np.asarray(u, dtype=np.complex128).reshape(2, 2)
    return np.ascontiguousarray(u.reshape(-1).view(np.float64))


_SQ = 1.0 / math.sqrt(2.0)
# Exact 2x2 matrices of the standard gates (row-major, a' = U a).
_MATS = {
    "Y": np.array([[0, -1j], [1j, 0]]),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
    "S": np.array([[1, 0], [0, 1j]]),
    "SDG": np.array([[1, 0], [0, -1j]]),
    "T": np.array([[1, 0], [0, complex(_SQ, _SQ)]]),
    "TDG": np.array([[1, 0], [0, complex(_SQ, -_SQ)]]),
}


def rk_angle(k: int) -> float:
    """2 pi / 2^k in FP64 (an exact power-of-two scaling of fl(2 pi))."""
    return math.ldexp(2.0 * math.pi, -k)


class Circuit:
    """Parsed circuit: n, initial basis state, list of (keyword, args) in file order."""

    def __init__(self, n: int, init: int, ops: list):
        self.n, self.init, self.ops = n, init, ops


def parse(text: str) -> Circuit:
    n = None
    init = 0
    ops = []
    for raw in text.splitlines():
        s = raw.split("!")[0].split("#")[0].strip()
        if not s:
            continue
        tok = s.split()
        kw = tok[0].upper()
        if kw == "QUBITS":
            n = int(tok[1])
        elif kw == "INITIAL":
            init = int(tok[2])
        else:
            ops.append((kw, tok[1:]))
    if n is None:
        raise ValueError("circuit has no QUBITS line")
    return Circuit(n, init, ops)


def apply_op(a: np.ndarray, n: int, kw: str, args: list[str]) -> None:
    """Apply one gate line to the interleaved FP64 state a (float64 array of length 2^(n+1))."""
    L = lib()
    p = _dp(a)
    iv = lambda k: int(args[k])
    fv = lambda k: float.fromhex(args[k]) if args[k].lower().startswith(("0x", "-0x")) else float(args[k])
    if kw == "H":
        L.or_hadamard(p, n, iv(0))
    elif kw in ("RX90", "RX90DG"):
        L.or_xrot(p, n, iv(0), int(kw.endswith("DG")))
    elif kw in ("RY90", "RY90DG"):
        L.or_yrot(p, n, iv(0), int(kw.endswith("DG")))
    elif kw == "X":
        L.or_cnot(p, n, 0, iv(0))
    elif kw in _MATS:
        L.or_unitary(p, n, iv(0), 0, _dp(_u8(_MATS[kw])))
    elif kw == "R":
        L.or_phase(p, n, iv(0), 0, fv(1))
    elif kw in ("RK", "RKDG"):
        sgn = -1.0 if kw == "RKDG" else 1.0
        L.or_phase(p, n, iv(0), 0, sgn * rk_angle(iv(1)))
    elif kw == "RZ":
        th = fv(1)
        u = np.array([[complex(math.cos(th / 2), -math.sin(th / 2)), 0],
                      [0, complex(math.cos(th / 2), math.sin(th / 2))]])
        L.or_unitary(p, n, iv(0), 0, _dp(_u8(u)))
    elif kw == "U":
        vals = [fv(1 + k) for k in range(8)]
        L.or_unitary(p, n, iv(0), 0, _dp(np.array(vals, dtype=np.float64)))
    elif kw == "CNOT":
        L.or_cnot(p, n, 1 << iv(0), iv(1))
    elif kw == "TOFFOLI":
        L.or_cnot(p, n, (1 << iv(0)) | (1 << iv(1)), iv(2))
    elif kw == "CZ":
        L.or_unitary(p, n, iv(1), 1 << iv(0), _dp(_u8(_MATS["Z"])))
    elif kw == "CPHASE":
        L.or_phase(p, n, iv(1), 1 << iv(0), fv(2))
    elif kw in ("CRK", "CRKDG"):
        sgn = -1.0 if kw == "CRKDG" else 1.0
        L.or_phase(p, n, iv(1), 1 << iv(0), sgn * rk_angle(iv(2)))
    elif kw == "CV":
        L.or_cv(p, n, 1 << iv(0), iv(1), fv(2))
    elif kw == "QSWAP":
        L.or_swap(p, n, iv(0), iv(1))
    elif kw == "RENORM":
        s = L.or_norm(p, n)
        if s > 0.0:
            a /= math.sqrt(s)
    elif kw == "MODEXP":
        xf, xq, ff, fq, y, G = (iv(k) for k in range(6))
        if not (G >= 2 and G <= 2 ** fq and xf + xq <= n and ff + fq <= n and (xf + xq <= ff or ff + fq <= xf)):
            raise ValueError("MODEXP: registers must be disjoint, inside the state, and G <= 2^fq")
        L.or_modexp(p, n, xf, xq, ff, fq, y, G)
    else:
        raise ValueError(f"unknown gate keyword {kw!r}")


def basis_state(n: int, x: int = 0) -> np.ndarray:
    a = np.zeros(2 ** (n + 1), dtype=np.float64)
    a[2 * x] = 1.0
    return a


def to_interleaved(psi: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64).copy()


def to_complex(a: np.ndarray) -> np.ndarray:
    return a.view(np.complex128)


def run_circuit(text: str, psi0: np.ndarray | None = None, ops_limit: int | None = None) -> np.ndarray:
    """Run the circuit from its INITIAL STATE (or from psi0 if given); returns complex128 amplitudes."""
    c = parse(text)
    a = basis_state(c.n, c.init) if psi0 is None else to_interleaved(psi0)
    if a.size != 2 ** (c.n + 1):
        raise ValueError("initial state has the wrong size")
    for i, (kw, args) in enumerate(c.ops):
        if ops_limit is not None and i >= ops_limit:
            break
        apply_op(a, c.n, kw, args)
    return to_complex(a)


def timed_run(text: str, psi0: np.ndarray | None = None, ops_limit: int | None = None) -> tuple[np.ndarray, float, int]:
    """run_circuit with a wall-clock time around the gate loop only; returns (state, seconds, gates)."""
    c = parse(text)
    a = basis_state(c.n, c.init) if psi0 is None else to_interleaved(psi0)
    ops = c.ops if ops_limit is None else c.ops[:ops_limit]
    t0 = time.perf_counter()
    for kw, args in ops:
        apply_op(a, c.n, kw, args)
    dt = time.perf_counter() - t0
    return to_complex(a), dt, len(ops)


def apply_dense(psi: np.ndarray, qubits: list[int], U: np.ndarray) -> np.ndarray:
    """Dense k-qubit gate (matrix index bit s <-> qubits[s]) on a copy of psi."""
    n = int(round(math.log2(psi.size)))
    a = to_interleaved(psi)
    k = len(qubits)
    q = (ctypes.c_int * k)(*qubits)
    Ui = np.ascontiguousarray(np.asarray(U, dtype=np.complex128)).view(np.float64)
    lib().or_dense(_dp(a), n, k, q, _dp(Ui))
    return to_complex(a)


def probs(psi: np.ndarray) -> np.ndarray:
    n = int(round(math.log2(psi.size)))
    a = to_interleaved(psi)
    p = np.empty(psi.size, dtype=np.float64)
    lib().or_probs(_dp(a), n, _dp(p))
    return p


def norm(psi: np.ndarray) -> float:
    n = int(round(math.log2(psi.size)))
    a = to_interleaved(psi)
    return lib().or_norm(_dp(a), n)


def marginals(psi: np.ndarray) -> np.ndarray:
    n = int(round(math.log2(psi.size)))
    a = to_interleaved(psi)
    q = np.empty(n, dtype=np.float64)
    lib().or_marginals(_dp(a), n, _dp(q))
    return q


# ---- error metrics (host, FP64) ----
def max_abs_diff(psi: np.ndarray, ref: np.ndarray) -> float:
    """max_i |psi_i - ref_i| (complex modulus, no global-phase alignment)."""
    return float(np.max(np.abs(np.asarray(psi, np.complex128) - np.asarray(ref, np.complex128))))


def infidelity(psi: np.ndarray, ref: np.ndarray) -> float:
    """1 - |<ref|psi>|^2 / (<ref|ref><psi|psi>), sums pairwise (numpy)."""
    psi = np.asarray(psi, np.complex128)
    ref = np.asarray(ref, np.complex128)
    ov = np.sum(np.conj(ref) * psi)
    nr = np.sum(ref.real ** 2 + ref.imag ** 2)
    nps = np.sum(psi.real ** 2 + psi.imag ** 2)
    return float(1.0 - (ov.real ** 2 + ov.imag ** 2) / (nr * nps))


def qft_sample(psi: np.ndarray, ks) -> np.ndarray:
    """Selected outputs of the quantum Fourier transform of psi (the Fourier representation used in
    the paper's Shor analysis, Sec. V): out_k = 2^{-n/2} sum_x psi_x e^{+2 pi i x k / 2^n}, with the
    phase x k reduced modulo 2^n exactly in integer arithmetic; one O(2^n) sum per k."""
    psi = np.asarray(psi, np.complex128)
    N = psi.size
    x = np.arange(N, dtype=np.int64)
    out = []
    for k in ks:
        ph = (x * int(k)) % N
        out.append(np.sum(psi * np.exp(2j * np.pi * ph / N)) / math.sqrt(N))
    return np.array(out)


def multiplicative_order(y: int, G: int) -> int:
    """The period r of f(x) = y^x mod G (smallest r > 0 with y^r = 1 mod G), by stepping through the
    powers (Sec. V); y must be coprime to G."""
    if math.gcd(y, G) != 1:
        raise ValueError("y and G are not coprime")
    r, v = 1, y % G
    while v != 1:
        v = (v * y) % G
        r += 1
    return r


def shor_probabilities(X: int, r: int) -> np.ndarray:
    """p_k, k = 0 .. 2^X - 1: the probability to observe |k> in the x-register after the Fourier
    transform in Shor's algorithm (Sec. V), for a function of period r. From the Fourier
    representation, the x-values that share f(x0) are x0 + j r, and
        p_k = 2^{-2X} sum_{x0 < r} | sum_j e^{2 pi i k (x0 + j r) / 2^X} |^2 ,
    where x0 < c = 2^X - r s (s = floor(2^X / r)) has s + 1 terms and the other r - c residues have s.
    Each inner sum is a geometric series of ratio e^{2 pi i phi}, phi = (k r mod 2^X) / 2^X, whose
    squared modulus for t terms is sin^2(pi t phi) / sin^2(pi phi), or t^2 when phi = 0; the products
    k r and t (k r) are reduced modulo 2^X in exact integer arithmetic before the sines. This sum replaces the printed closed form Eq. Shor5, whose second term carries
    the wrong sign (with it the p_k do not sum to 1)."""
    N = 1 << X
    s = N // r
    c = N - r * s
    k = np.arange(N, dtype=np.int64)
    m = (k * r) % N  # phi = m / N

    def sin2(u):
        # sin^2(pi u / N) for integers u: periodic in u with period N and symmetric under u -> N - u,
        # so the sine is taken at an argument in [0, pi/2]
        u = u % N
        return np.sin(np.pi * np.minimum(u, N - u) / N) ** 2

    zero = m == 0
    safe = np.where(zero, 1.0, sin2(m))

    def geo(t):
        return np.where(zero, float(t) ** 2, sin2(t * m) / safe)

    return (c * geo(s + 1) + (r - c) * geo(s)) / float(N) ** 2


def shor_expectations(X: int, r: int) -> np.ndarray:
    """<Q_i> = sum_k p_k bit_i(k), i = 0 .. X-1 (Eq. Shor7)."""
    p = shor_probabilities(X, r)
    k = np.arange(1 << X, dtype=np.int64)
    return np.array([float(np.sum(p[((k >> i) & 1) == 1])) for i in range(X)])
