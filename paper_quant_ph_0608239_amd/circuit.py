"""Circuit text -> gate records of the C ABI (marshalling only).

The text format is one gate per line, a keyword followed by values, with `!`/`#` comments, in the
style of the paper's App. A input file: QUBITS n, INITIAL STATE x, then gate lines such as
`H 0`, `CNOT 0 1`, `CRK 2 5 3`, `U 4 <8 hex floats>`. Floats may be decimal or C99 hex.
Controlled gates list the control(s) first and the target last. `RK t k` / `CRK c t k` carry the
integer k of the phase shift 2 pi / 2^k; the library forms the angle.
"""
from __future__ import annotations

from ._lib import OPS, Gate

_ONE_QUBIT = {"H", "X", "Y", "Z", "S", "SDG", "T", "TDG", "RX90", "RX90DG", "RY90", "RY90DG"}


def _f(s: str) -> float:
    t = s.strip()
    if t.lower().startswith(("0x", "-0x", "+0x")):
        return float.fromhex(t)
    return float(t)


def _gate(op: str, target: int, controls: int = 0, theta: float = 0.0, target2: int = -1, u=None) -> Gate:
    g = Gate()
    g.op = OPS[op]
    g.target = target
    g.target2 = target2
    g.reserved = 0
    g.controls = controls
    g.theta = theta
    if u is not None:
        for i, v in enumerate(u):
            g.u[i] = v
    return g


class Circuit:
    def __init__(self, n: int, gates: list[Gate], init: int = 0, names: list[str] | None = None):
        self.n = n
        self.gates = gates
        self.init = init
        self.names = names or []

    def __len__(self):
        return len(self.gates)

    def gate_array(self):
        return (Gate * max(1, len(self.gates)))(*self.gates)


def parse_circuit(text: str) -> Circuit:
    n = None
    init = 0
    gates: list[Gate] = []
    names: list[str] = []
    for raw in text.splitlines():
        s = raw.split("!")[0].split("#")[0].strip()
        if not s:
            continue
        tok = s.split()
        kw = tok[0].upper()
        a = tok[1:]
        if kw == "QUBITS":
            n = int(a[0])
            continue
        if kw == "INITIAL":
            init = int(a[1])
            continue
        if kw in _ONE_QUBIT:
            g = _gate(kw, int(a[0]))
        elif kw == "R":
            g = _gate("PHASE", int(a[0]), theta=_f(a[1]))
        elif kw in ("RK", "RKDG"):
            g = _gate(kw, int(a[0]), target2=int(a[1]))
        elif kw == "RZ":
            g = _gate("RZ", int(a[0]), theta=_f(a[1]))
        elif kw == "U":
            g = _gate("MATRIX", int(a[0]), u=[_f(x) for x in a[1:9]])
        elif kw == "CNOT":
            g = _gate("X", int(a[1]), controls=1 << int(a[0]))
        elif kw == "CZ":
            g = _gate("Z", int(a[1]), controls=1 << int(a[0]))
        elif kw == "CPHASE":
            g = _gate("PHASE", int(a[1]), controls=1 << int(a[0]), theta=_f(a[2]))
        elif kw in ("CRK", "CRKDG"):
            g = _gate(kw[1:], int(a[1]), controls=1 << int(a[0]), target2=int(a[2]))
        elif kw == "CV":
            g = _gate("V", int(a[1]), controls=1 << int(a[0]), theta=_f(a[2]))
        elif kw == "TOFFOLI":
            g = _gate("X", int(a[2]), controls=(1 << int(a[0])) | (1 << int(a[1])))
        elif kw == "QSWAP":
            g = _gate("SWAP", int(a[0]), target2=int(a[1]))
        elif kw == "RENORM":
            g = _gate("RENORM", 0)
        else:
            raise ValueError(f"unknown gate keyword {kw!r}")
        gates.append(g)
        names.append(kw)
    if n is None:
        raise ValueError("circuit has no QUBITS line")
    return Circuit(n, gates, init, names)
