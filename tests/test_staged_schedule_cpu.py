"""CPU tests of the LDS-staged scheduler (no GPU): the host scheduler's tables, applied by a numpy model
of the staged kernels' semantics, must reproduce the oracle, and every half-buffer LDS round trip must
move each element to the slot the next layout reads. The scheduler runs inside libqsim (host code);
tests/sched_dump.cpp calls it and writes its tables."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import qsim_workloads as wl
from paper_quant_ph_0608239_amd.circuit import parse_circuit
from tests import staged_model as sm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_quant_ph_0608239_amd")
LIB = os.path.join(PKG, "libqsim.so")


@pytest.fixture(scope="module")
def dumper(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(LIB) or not os.path.exists(hipcc):
        pytest.skip("needs the built libqsim.so and hipcc")
    out = str(tmp_path_factory.mktemp("sched") / "sched_dump")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           os.path.join(ROOT, "tests", "sched_dump.cpp"), "-L", PKG, "-lqsim", "-Wl,-rpath," + PKG, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def tables(dumper, tmp_path, text, n, c128, m, le, width=None):
    """Tables of the plan scheduler (width None: the pass search plans use; 1: the greedy rule)."""
    gates = tmp_path / "g.bin"
    gates.write_bytes(bytes(parse_circuit(text).gate_array()))
    out = tmp_path / "s.bin"
    extra = [] if width is None else [str(width)]
    r = subprocess.run([dumper, str(gates), str(n), "1" if c128 else "0", str(m), str(le), str(out)] + extra,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    return sm.load_tables(str(out))


def mixed_circuit(n, count, seed):
    rng = np.random.default_rng(seed)
    lines = []
    for _ in range(count):
        k = rng.integers(0, 7)
        qs = rng.choice(n, 3, replace=False)
        if k == 0:
            lines.append(wl.u_line(int(qs[0]), wl.haar_2x2(rng)))
        elif k == 1:
            lines.append(f"CNOT {qs[0]} {qs[1]}")
        elif k == 2:
            lines.append(f"TOFFOLI {qs[0]} {qs[1]} {qs[2]}")
        elif k == 3:
            lines.append(f"CPHASE {qs[0]} {qs[1]} {float(rng.uniform(0, 6)).hex()}")
        elif k == 4:
            lines.append(f"RZ {qs[0]} {float(rng.uniform(0, 6)).hex()}")
        elif k == 5:
            lines.append(f"CZ {qs[0]} {qs[1]}")
        else:
            lines.append(f"QSWAP {qs[0]} {qs[1]}")
    return wl.circuit_text(n, lines)


def u_cz_circuit(n, count, seed):
    rng = np.random.default_rng(seed)
    lines = []
    for _ in range(count):
        qs = rng.choice(n, 2, replace=False)
        lines.append(wl.u_line(int(qs[0]), wl.haar_2x2(rng)) if rng.integers(0, 2) == 0 else f"CZ {qs[0]} {qs[1]}")
    return wl.circuit_text(n, lines)


CASES = {
    "brickwork": lambda: (wl.brickwork_circuit(13, 6, seed=21), 13),
    "config0": lambda: (wl.config0_circuit(13, 150, seed=3), 13),
    "qft_with_swaps": lambda: (wl.qft_circuit(12), 12),
    "u_cz": lambda: (u_cz_circuit(13, 200, seed=5), 13),
    "mixed": lambda: (mixed_circuit(12, 120, seed=7), 12),
}
VARIANTS = [(True, 10, 4), (True, 11, 4), (True, 12, 4), (True, 11, 3), (False, 11, 5), (False, 12, 5), (False, 12, 4)]


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("c128,m,le", VARIANTS)
def test_schedule_reproduces_oracle(dumper, tmp_path, oracle_mod, case, c128, m, le):
    text, n = CASES[case]()
    P, S, RD, O, B = tables(dumper, tmp_path, text, n, c128, m, le)
    psi0 = wl.gaussian_state(n, 3)
    ref = oracle_mod.run_circuit(text, psi0=psi0)
    got = sm.run_schedule(psi0, n, m, le, P, S, RD, O, B)
    assert np.max(np.abs(got - ref)) < 1e-12
    sm.check_half_exchanges(P, S, m, le, c128)
    if m - le >= 7:
        sm.check_wave_barriers(P, S, m, le)


SEARCH_CASES = {
    "brickwork16": lambda: (wl.brickwork_circuit(16, 10, seed=21), 16, True, 10, 4),
    "brickwork17": lambda: (wl.brickwork_circuit(17, 8, seed=21), 17, True, 10, 4),
    "qft15_with_swaps": lambda: (wl.qft_circuit(15), 15, True, 10, 4),
    "mixed15_c64": lambda: (mixed_circuit(15, 150, 7), 15, False, 11, 5),
}


@pytest.mark.parametrize("case", sorted(SEARCH_CASES))
def test_pass_search_saves_passes_and_reproduces_oracle(dumper, tmp_path, oracle_mod, case):
    """Where the greedy choice of resident sets leaves a ragged frontier (brickworks, a QFT with its
    swaps, random gates with controls and swaps), the plans' pass search finds a sequence with one pass
    fewer; that schedule still reproduces the oracle and keeps its LDS exchanges valid."""
    text, n, c128, m, le = SEARCH_CASES[case]()
    greedy = tables(dumper, tmp_path, text, n, c128, m, le, width=1)
    P, S, RD, O, B = tables(dumper, tmp_path, text, n, c128, m, le)
    assert len(P) == len(greedy[0]) - 1
    psi0 = wl.gaussian_state(n, 3)
    ref = oracle_mod.run_circuit(text, psi0=psi0)
    got = sm.run_schedule(psi0, n, m, le, P, S, RD, O, B)
    assert np.max(np.abs(got - ref)) < 1e-12
    sm.check_half_exchanges(P, S, m, le, c128)


def test_brickwork_passes_use_wave_splits(dumper, tmp_path):
    """At 12 resident qubits (complex128, 16 amplitudes per thread) the brickwork's passes take the
    half-size buffer with every split at a wave position."""
    text = wl.brickwork_circuit(16, 8, seed=21)
    P, S, RD, O, B = tables(dumper, tmp_path, text, 16, True, 12, 4)
    nhalf, nwave = sm.check_half_exchanges(P, S, 12, 4, True)
    assert nhalf == len(P) and nwave == len(P)
    assert sm.check_wave_barriers(P, S, 12, 4) == len(P)


def test_wave_barrier_model_catches_a_missing_barrier(dumper, tmp_path, monkeypatch):
    """The barrier check fails when one half of a round trip skips a barrier (planted in the model)."""
    text = wl.brickwork_circuit(16, 8, seed=21)
    P, S, RD, O, B = tables(dumper, tmp_path, text, 16, True, 12, 4)
    orig = sm._wave_trace

    def drop_one(ps, sts, w):
        ev = orig(ps, sts, w)
        if w == 0:
            ev.remove(('B',))
        return ev

    monkeypatch.setattr(sm, "_wave_trace", drop_one)
    with pytest.raises(AssertionError):
        sm.check_wave_barriers(P, S, 12, 4)


def test_wave_barrier_model_catches_an_early_write(dumper, tmp_path, monkeypatch):
    """The ordering check fails when the second half writes before its two waiting barriers (the
    barrier count stays equal; planted in the model)."""
    text = wl.brickwork_circuit(16, 8, seed=21)
    P, S, RD, O, B = tables(dumper, tmp_path, text, 16, True, 12, 4)
    orig = sm._wave_trace

    def early(ps, sts, w):
        ev = orig(ps, sts, w)
        for i in range(len(ev) - 2):
            if ev[i] == ('B',) and ev[i + 1] == ('B',) and ev[i + 2][0] == 'W':
                ev[i], ev[i + 2] = ev[i + 2], ev[i]
                break
        return ev

    monkeypatch.setattr(sm, "_wave_trace", early)
    with pytest.raises(AssertionError):
        sm.check_wave_barriers(P, S, 12, 4)
