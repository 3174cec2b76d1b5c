"""Seeded synthetic inputs shared by the GPU path, the CPU oracle and the benchmark.

This module only *draws* and *writes down* inputs: circuits as text (one gate per line, in the
keyword-plus-values style of the paper's App. A input file) and initial state vectors. It contains
none of the simulator's arithmetic: no gate matrix is built from a gate name here, no amplitude
is updated, no angle is turned into a phase factor. Random numbers that a workload needs (Haar
2x2 unitaries, rotation angles, adder operands, Gaussian amplitudes) are drawn here and passed on
as inputs, written as C99 hex floats so that both consumers read bit-identical values.

Circuit text format (each consumer has its own parser)::

    QUBITS n
    INITIAL STATE x            optional basis state |x>, default 0
    ! comment  /  # comment
    H q | X q | Y q | Z q | S q | SDG q | T q | TDG q
    RX90 q | RX90DG q | RY90 q | RY90DG q     the paper's X = exp(i pi S^x/2), Y = exp(i pi S^y/2)
    R q phi                    phase shift diag(1, e^{i phi})
    RK q k | RKDG q k          R(+2 pi/2^k) | R(-2 pi/2^k)
    RZ q theta                 diag(e^{-i theta/2}, e^{+i theta/2})
    U q u00r u00i u01r u01i u10r u10i u11r u11i     explicit 2x2, row-major, a' = U a
    CNOT c t | CZ c t | CPHASE c t phi | CRK c t k | CRKDG c t k | CV c t phi
    TOFFOLI c1 c2 t
    QSWAP a b                  quantum swap of two qubits
    MODEXP xf xq ff fq y G     |x>|z> -> |x>|z XOR (y^x mod G)>, x = qubits xf..xf+xq-1, z = ff..ff+fq-1

Qubit q is bit q of the amplitude index (qubit 0 = least significant bit). For controlled gates
the control(s) come first and the target last.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "CONFIG0_KINDS", "random_gate_circuit", "config0_circuit", "brickwork_circuit",
    "qft_lines", "iqft_lines", "qft_circuit", "ripple_adder_circuit", "adder_operands",
    "qft_adder_circuit", "gaussian_state", "random_state", "batch_circuits", "hexf",
    "circuit_text", "count_gates", "shor_circuit_layout", "inverse_lines", "haar_2x2", "u_line",
    "SHOR_CASES", "shor_parts", "shor_circuit", "PAPER_ADDERS",
]


def hexf(x: float) -> str:
    """Exact text form of an FP64 value (C99 hex float; read back by strtod / float.fromhex)."""
    return float(x).hex()


def circuit_text(n: int, lines: list[str], initial_state: int = 0, header: list[str] | None = None) -> str:
    out = []
    for h in header or []:
        out.append("! " + h)
    out.append(f"QUBITS {n}")
    if initial_state:
        out.append(f"INITIAL STATE {initial_state}")
    out.extend(lines)
    return "\n".join(out) + "\n"


def count_gates(text: str) -> int:
    """Number of gate lines (every elementary gate counts as one operation)."""
    n = 0
    for ln in text.splitlines():
        s = ln.strip()
        if not s or s[0] in "!#":
            continue
        kw = s.split()[0]
        if kw in ("QUBITS", "INITIAL"):
            continue
        n += 1
    return n


# --------------------------------------------------------------------------------------------
# Random gates from the nine-name set {H, X, Y, Z, S, T, RZ(theta), CNOT, CPHASE(theta)}
# --------------------------------------------------------------------------------------------
CONFIG0_KINDS = ("H", "X", "Y", "Z", "S", "T", "RZ", "CNOT", "CPHASE")


def random_gate_circuit(n: int, ngates: int, rng: np.random.Generator) -> list[str]:
    """ngates gates; per gate the draws are, in order: kind (uniform over the nine names), the
    qubit(s) (a target uniform in [0, n); an ordered (control, target) pair uniform over the
    n(n-1) distinct pairs), then theta ~ U[0, 2 pi) for RZ and CPHASE."""
    if n < 2:
        raise ValueError("two-qubit gates need n >= 2")
    lines = []
    for _ in range(ngates):
        kind = CONFIG0_KINDS[int(rng.integers(0, len(CONFIG0_KINDS)))]
        if kind in ("CNOT", "CPHASE"):
            p = int(rng.integers(0, n * (n - 1)))
            c = p // (n - 1)
            t = p % (n - 1)
            if t >= c:
                t += 1
            if kind == "CNOT":
                lines.append(f"CNOT {c} {t}")
            else:
                theta = float(rng.uniform(0.0, 2.0 * np.pi))
                lines.append(f"CPHASE {c} {t} {hexf(theta)}")
        else:
            q = int(rng.integers(0, n))
            if kind == "RZ":
                theta = float(rng.uniform(0.0, 2.0 * np.pi))
                lines.append(f"RZ {q} {hexf(theta)}")
            else:
                lines.append(f"{kind} {q}")
    return lines


def config0_circuit(n: int = 16, ngates: int = 200, seed: int = 1) -> str:
    """Hadamard on every qubit, then ngates random gates (start |0...0>)."""
    rng = np.random.default_rng(seed)
    lines = [f"H {q}" for q in range(n)] + random_gate_circuit(n, ngates, rng)
    return circuit_text(n, lines, header=[f"random circuit n={n} gates={ngates} seed={seed} (H prefix)"])


# --------------------------------------------------------------------------------------------
# Brickwork: layers of Haar-random 2x2 unitaries on every qubit, then CZ on alternating pairs
# --------------------------------------------------------------------------------------------
def haar_2x2(rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed U(2) element by Mezzadri's recipe (QR of a complex Ginibre matrix with the
    phases of R's diagonal moved into Q). A random draw, passed on as an input."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


def u_line(q: int, u: np.ndarray) -> str:
    vals = []
    for r in range(2):
        for c in range(2):
            vals += [hexf(u[r, c].real), hexf(u[r, c].imag)]
    return f"U {q} " + " ".join(vals)


def brickwork_circuit(n: int, layers: int = 20, seed: int = 21, layer_range: tuple[int, int] | None = None,
                      renorm_after: tuple[int, ...] = ()) -> str:
    """Layer l = 0..layers-1: a Haar U on every qubit (qubit order 0..n-1), then CZ(q, q+1) for every
    q = l (mod 2) with q+1 < n. Start |0...0>. layer_range=(a, b) emits only layers a..b-1 (the random
    draws of all layers are made in the same order, so the pieces concatenate to the full circuit).
    renorm_after: a RENORM line after that many layers, once per entry (0: before the first layer)."""
    rng = np.random.default_rng(seed)
    a, b = layer_range if layer_range else (0, layers)
    lines = []
    lines += ["RENORM"] * sum(1 for k in renorm_after if k == 0)
    for layer in range(layers):
        us = [haar_2x2(rng) for _ in range(n)]
        if not a <= layer < b:
            continue
        for q in range(n):
            lines.append(u_line(q, us[q]))
        for q in range(layer % 2, n - 1, 2):
            lines.append(f"CZ {q} {q + 1}")
        lines += ["RENORM"] * sum(1 for k in renorm_after if k == layer + 1)
    tag = f" renorm_after={','.join(map(str, renorm_after))}" if renorm_after else ""
    return circuit_text(n, lines, header=[f"brickwork n={n} layers={layers} seed={seed} range={a}..{b - 1}{tag}"])


def inverse_lines(text: str) -> list[str]:
    """Gate lines of the exact inverse circuit: reversed order, every gate replaced by its inverse
    (explicit U by its conjugate transpose, self-inverse gates unchanged). For the families used
    here: U, CZ, H, X, Z, CNOT, TOFFOLI, QSWAP, CRK/CRKDG."""
    out = []
    for ln in reversed(text.splitlines()):
        t = ln.split()
        if not t or t[0] in ("QUBITS", "INITIAL", "!", "#") or t[0].startswith(("!", "#")):
            continue
        kw = t[0]
        if kw == "U":
            v = [float.fromhex(x) for x in t[2:10]]
            u = np.array([[complex(v[0], v[1]), complex(v[2], v[3])], [complex(v[4], v[5]), complex(v[6], v[7])]])
            out.append(u_line(int(t[1]), u.conj().T))
        elif kw in ("CZ", "H", "X", "Z", "CNOT", "TOFFOLI", "QSWAP"):
            out.append(ln)
        elif kw in ("CRK", "CRKDG"):
            out.append(("CRKDG " if kw == "CRK" else "CRK ") + " ".join(t[1:]))
        else:
            raise ValueError(f"no inverse rule for {kw}")
    return out


# --------------------------------------------------------------------------------------------
# Quantum Fourier transform (Hadamards and controlled phase shifts by 2 pi / 2^k)
# --------------------------------------------------------------------------------------------
def qft_lines(qubits: list[int], swaps: bool = True) -> list[str]:
    """|x> -> 2^{-m/2} sum_k e^{+2 pi i x k / 2^m} |k> on the register qubits[0..m-1] (qubits[0] = least
    significant bit). For j = m-1 down to 0: H on qubits[j], then controlled R(2 pi / 2^{j-l+1}) from
    qubits[l] onto qubits[j] for l = j-1 down to 0; then the bit-reversal swaps."""
    m = len(qubits)
    lines = []
    for j in range(m - 1, -1, -1):
        lines.append(f"H {qubits[j]}")
        for l in range(j - 1, -1, -1):
            lines.append(f"CRK {qubits[l]} {qubits[j]} {j - l + 1}")
    if swaps:
        for i in range(m // 2):
            lines.append(f"QSWAP {qubits[i]} {qubits[m - 1 - i]}")
    return lines


def iqft_lines(qubits: list[int], swaps: bool = True) -> list[str]:
    """Exact inverse of qft_lines: the gates in reverse order, each replaced by its inverse."""
    inv = []
    for ln in reversed(qft_lines(qubits, swaps)):
        kw, *rest = ln.split()
        if kw == "CRK":
            inv.append("CRKDG " + " ".join(rest))
        else:  # H and QSWAP are their own inverses
            inv.append(ln)
    return inv


def qft_circuit(n: int) -> str:
    return circuit_text(n, qft_lines(list(range(n))), header=[f"QFT on {n} qubits"])


# --------------------------------------------------------------------------------------------
# Ripple-carry adder from CNOT and Toffoli gates (Cuccaro, Draper, Kutin, Moulton, 2004)
# --------------------------------------------------------------------------------------------
def ripple_adder_circuit(m: int = 14) -> tuple[str, dict]:
    """Adds two m-bit registers in place: |a>|b>|0> -> |a>|(a+b) mod 2^m>|0>.

    Layout: a = qubits 0..m-1, b = qubits m..2m-1, qubit 2m = carry-in ancilla c (starts and ends 0),
    2m+1 qubits in all. Built from the MAJ and UMA blocks of the published construction: MAJ(c, b_i, a_i)
    leaves the carry in a_i, UMA undoes it and leaves the sum bit in b_i."""
    a = list(range(m))
    b = list(range(m, 2 * m))
    c = 2 * m
    lines = []

    def maj(x, y, z):  # x: incoming carry, y: b_i, z: a_i
        lines.append(f"CNOT {z} {y}")
        lines.append(f"CNOT {z} {x}")
        lines.append(f"TOFFOLI {x} {y} {z}")

    def uma(x, y, z):
        lines.append(f"TOFFOLI {x} {y} {z}")
        lines.append(f"CNOT {z} {x}")
        lines.append(f"CNOT {x} {y}")

    carry = [c] + a[:-1]
    for i in range(m):
        maj(carry[i], b[i], a[i])
    for i in range(m - 1, -1, -1):
        uma(carry[i], b[i], a[i])
    n = 2 * m + 1
    layout = {"a": a, "b": b, "ancilla": c, "n": n, "m": m}
    return circuit_text(n, lines, header=[f"ripple-carry adder m={m} (CNOT+TOFFOLI)"]), layout


def adder_operands(m: int = 14, count: int = 64, seed: int = 11) -> list[tuple[int, int]]:
    rng = np.random.default_rng(seed)
    ab = rng.integers(0, 2 ** m, size=(count, 2))
    return [(int(x), int(y)) for x, y in ab]


# --------------------------------------------------------------------------------------------
# The paper's register adder (QFT on the target register, controlled phases from the others)
# --------------------------------------------------------------------------------------------
_PREP_CYCLE = ("RX90", "RY90", "RX90DG", "RY90DG")


def qft_adder_circuit(values: list[int], m: int) -> tuple[str, dict]:
    """r registers of m qubits each (register i = qubits i*m .. i*m+m-1), loaded with values[i] by
    applying one of XX, YY, X'X', Y'Y' (the paper's pi/2 rotations twice; each takes |0> to |1> up to
    a phase) to each set bit, cycling through the four; then QFT on the last register, controlled
    phase shifts from every other register onto it, inverse QFT. The last register ends in
    (sum of values) mod 2^m. No bit-reversal swaps are used inside the adder; the QFT output is then
    bit-reversed on the register, which the controlled phases take into account."""
    r = len(values)
    n = r * m
    lines = []
    cyc = 0
    for i, v in enumerate(values):
        if not 0 <= v < 2 ** m:
            raise ValueError("register value out of range")
        for bit in range(m):
            if (v >> bit) & 1:
                g = _PREP_CYCLE[cyc % 4]
                cyc += 1
                q = i * m + bit
                lines += [f"{g} {q}", f"{g} {q}"]
    tgt = list(range((r - 1) * m, r * m))
    # QFT without swaps: after it, qubit tgt[j] carries the phase of Fourier bit (m-1-j)
    lines += qft_lines(tgt, swaps=False)
    # add register s: phase e^{2 pi i x_s k / 2^m}; Fourier index bit (m-1-j) sits on tgt[j];
    # contribution of control bit l of x_s and Fourier bit p = m-1-j: 2 pi 2^{l+p} / 2^m
    for s in range(r - 1):
        for j in range(m - 1, -1, -1):
            p = m - 1 - j
            for l in range(m):
                kexp = m - l - p          # angle 2 pi / 2^kexp
                if kexp >= 1:
                    lines.append(f"CRK {s * m + l} {tgt[j]} {kexp}")
    lines += iqft_lines(tgt, swaps=False)
    return circuit_text(n, lines, header=[f"{r}-{m} QFT register adder values={values}"]), {
        "n": n, "target": tgt, "sum": sum(values) % (2 ** m)}


# the register adders of the paper's runs: (values, m) with the printed operation counts N_O
# (Fig. adder; App. B tables)
PAPER_ADDERS = (((1365, 682), 11, None), ((292, 585, 1170), 11, 286), ((26214, 104857), 17, 493),
                ((7, 9, 19, 35, 65), 7, 194), ((781, 1054, 3296), 12, 342))


# --------------------------------------------------------------------------------------------
# Shor's period finding: register layout (Eq. Shor0); the modular exponentiation is input data
# --------------------------------------------------------------------------------------------
def shor_circuit_layout(L: int, X: int, G: int, y: int) -> dict:
    """x-register = qubits 0..X-1, f-register = qubits X..L-1 (F = L - X qubits, G < 2^F)."""
    F = L - X
    if G >= 2 ** F or not (G * G <= 2 ** X <= 2 * G * G):
        raise ValueError("register sizes violate G^2 <= 2^X <= 2 G^2 or G < 2^F")
    return {"L": L, "X": X, "F": F, "G": G, "y": y}


# (L, X, G, y) of the paper's Shor runs (Table Shortab)
SHOR_CASES = ((24, 16, 247, 194), (33, 22, 1961, 1698), (33, 22, 2047, 617), (36, 24, 4087, 1392),
              (36, 24, 4033, 1693))


def shor_parts(L: int, X: int, G: int, y: int) -> tuple[str, tuple, str]:
    """Shor's period finding in three parts: Hadamard on every x-register qubit; the modular
    exponentiation (xf, xq, ff, fq, y, G); the QFT of the x-register (with its bit-reversal swaps,
    so that bit i of the final x-register value is qubit i)."""
    lay = shor_circuit_layout(L, X, G, y)
    pre = circuit_text(L, [f"H {q}" for q in range(X)], header=[f"Shor L={L} X={X} G={G} y={y}: Hadamards"])
    post = circuit_text(L, qft_lines(list(range(X))), header=[f"Shor L={L} X={X}: QFT of the x-register"])
    return pre, (0, X, X, lay["F"], y, G), post


def shor_circuit(L: int, X: int, G: int, y: int) -> str:
    pre, (xf, xq, ff, fq, yy, GG), post = shor_parts(L, X, G, y)
    body = lambda t: [ln for ln in t.splitlines() if ln and not ln.startswith(("!", "QUBITS"))]
    return circuit_text(L, body(pre) + [f"MODEXP {xf} {xq} {ff} {fq} {yy} {GG}"] + body(post),
                        header=[f"Shor L={L} X={X} G={G} y={y}"])


# --------------------------------------------------------------------------------------------
# Initial states
# --------------------------------------------------------------------------------------------
def gaussian_state(n: int, seed: int = 12) -> np.ndarray:
    """re, im ~ N(0,1) i.i.d. (PCG64), scaled to unit norm in FP64 (numpy's pairwise sum)."""
    rng = np.random.default_rng(seed)
    psi = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    psi /= np.sqrt(np.sum(psi.real ** 2 + psi.imag ** 2))
    return psi


def random_state(n: int, seed: int) -> np.ndarray:
    return gaussian_state(n, seed)


# --------------------------------------------------------------------------------------------
# Many small independent circuits of uneven size
# --------------------------------------------------------------------------------------------
def batch_circuits(count: int = 2048, nmin: int = 10, nmax: int = 22, depth: int = 50,
                   seed: int = 41) -> list[str]:
    """count circuits; qubit counts uniform in [nmin, nmax]; depth gates each from the nine-name set,
    no Hadamard prefix, start |0...0>."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i, n in enumerate(ns):
        lines = random_gate_circuit(int(n), depth, rng)
        out.append(circuit_text(int(n), lines, header=[f"batch circuit {i} n={int(n)} depth={depth}"]))
    return out
