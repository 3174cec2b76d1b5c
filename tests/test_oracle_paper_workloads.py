"""Pins of the oracle on the paper's own workloads (Sec. V): the QFT register adders of Fig. adder and
of the App. B tables, and Shor's period finding of Table Shortab.

What pins them: the printed sums and operation counts N_O (tests/golden/paper_adders.txt), the
printed periods and qubit expectation values <Q_i> (tests/golden/shor_table.txt), integer
arithmetic (Python's pow for y^x mod G), and brute-force Fourier sums for the Shor probabilities.
"""
import cmath
import math
import os

import numpy as np
import pytest

import qsim_workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def shor_rows():
    out = []
    for t in _rows("shor_table.txt"):
        L, X, G, y, r = (int(v) for v in t[:5])
        out.append((L, X, G, y, r, [float(v) for v in t[5:]]))
    return out


def adder_rows():
    out = []
    for t in _rows("paper_adders.txt"):
        m = int(t[0])
        n_o = None if t[1] == "-" else int(t[1])
        out.append((m, n_o, [int(v) for v in t[2:]]))
    return out


# ----------------------------------------------------------------------------------------------
# QFT register adders
# ----------------------------------------------------------------------------------------------
def test_adder_fixture_matches_generator_cases():
    assert [(m, no, tuple(v)) for m, no, v in adder_rows()] == [(m, no, v) for v, m, no in wl.PAPER_ADDERS]


@pytest.mark.parametrize("m,n_o,values", adder_rows())
def test_adder_operation_counts(m, n_o, values):
    """The generated network has the paper's number of quantum operations: two per set input bit
    (XX, YY, X'X' or Y'Y'), a QFT and an inverse QFT of m(m+1)/2 operations each, and m(m+1)/2
    controlled phase shifts per added register; for the 2-11 adder of Fig. adder that is 22
    preparation operations and 66 controlled phase shifts."""
    text, lay = wl.qft_adder_circuit(values, m)
    lines = [ln.split()[0] for ln in text.splitlines() if ln and ln[0] not in "!#" and not ln.startswith("QUBITS")]
    prep = sum(1 for kw in lines if kw in ("RX90", "RY90", "RX90DG", "RY90DG"))
    assert prep == 2 * sum(bin(v).count("1") for v in values)
    assert wl.count_gates(text) == prep + (len(values) + 1) * m * (m + 1) // 2
    if n_o is not None:
        assert wl.count_gates(text) == n_o
    else:
        assert prep == 22 and lines.count("CRK") - m * (m - 1) // 2 == 66
    assert lay["sum"] == sum(values) % 2 ** m


def _adder_final_register(oracle_mod, values, m):
    text, lay = wl.qft_adder_circuit(values, m)
    psi = oracle_mod.run_circuit(text)
    p = np.abs(psi) ** 2
    want = 0
    for i, v in enumerate(values[:-1]):
        want |= v << (i * m)
    want |= lay["sum"] << ((len(values) - 1) * m)
    return p, want


@pytest.mark.parametrize("r,m", [(2, 3), (3, 2)])
def test_small_adders_exhaustive(oracle_mod, r, m):
    """Every combination of register values: the last register ends in the sum mod 2^m, the other
    registers keep their values, with probability 1."""
    import itertools
    for values in itertools.product(range(2 ** m), repeat=r):
        p, want = _adder_final_register(oracle_mod, list(values), m)
        assert p[want] > 1 - 1e-13, values


def test_adder_fig_2x11_1365_plus_682(oracle_mod):
    """Fig. adder: 1365 + 682 in two 11-qubit registers gives 2047."""
    p, want = _adder_final_register(oracle_mod, [1365, 682], 11)
    assert want >> 11 == 2047
    assert p[want] > 1 - 1e-12


# ----------------------------------------------------------------------------------------------
# Shor's period finding
# ----------------------------------------------------------------------------------------------
def test_shor_fixture_matches_generator_cases():
    assert [(L, X, G, y) for L, X, G, y, _, _ in shor_rows()] == list(wl.SHOR_CASES)


@pytest.mark.parametrize("L,X,G,y,r,q", shor_rows())
def test_shor_table_periods_and_registers(oracle_mod, L, X, G, y, r, q):
    """The printed r is the order of y mod G (checked with Python's pow), y^(r/2) != +-1 mod G, the
    register sizes satisfy Eq. Shor0, and <Q_i> is printed for the X qubits of the x-register."""
    assert oracle_mod.multiplicative_order(y, G) == r
    assert pow(y, r, G) == 1 and all(pow(y, d, G) != 1 for d in range(1, r))
    assert r % 2 == 0 and pow(y, r // 2, G) not in (1, G - 1)
    assert G * G <= 2 ** X <= 2 * G * G and G < 2 ** (L - X)
    assert len(q) == X
    f1, f2 = math.gcd(pow(y, r // 2, G) - 1, G), math.gcd(pow(y, r // 2, G) + 1, G)
    assert f1 * f2 == G and 1 < f1 < G


@pytest.mark.parametrize("X,r", [(6, 5), (7, 6), (8, 10), (9, 12), (8, 3)])
def test_shor_probabilities_brute_force(oracle_mod, X, r):
    """p_k from the closed-form geometric sums equals the Fourier sum over the x-values of each
    residue class, evaluated term by term."""
    N = 2 ** X
    got = oracle_mod.shor_probabilities(X, r)
    want = np.zeros(N)
    for k in range(N):
        tot = 0.0
        for x0 in range(r):
            acc = sum(cmath.exp(2j * math.pi * k * x / N) for x in range(x0, N, r))
            tot += abs(acc) ** 2
        want[k] = tot / N ** 2
    assert np.max(np.abs(got - want)) < 1e-13
    assert abs(got.sum() - 1.0) < 1e-13


@pytest.mark.parametrize("L,X,G,y,r,q", shor_rows())
def test_shor_expectations_match_table(oracle_mod, L, X, G, y, r, q):
    """<Q_i> = sum_k p_k bit_i(k) (Eq. Shor7) reproduces every printed value to three decimals, with
    qubit i = bit i of k."""
    got = oracle_mod.shor_expectations(X, r)
    assert np.max(np.abs(got - np.array(q))) <= 5e-4 + 1e-12


def test_oracle_modexp_permutation(oracle_mod):
    """The oracle's conditional operation against y^x mod G from Python's pow, on a random state and
    with the f-register below the x-register; applying it twice restores the state."""
    n, xf, xq, ff, fq, y, G = 9, 4, 5, 0, 4, 7, 13
    psi = wl.gaussian_state(n, 5)
    line = f"MODEXP {xf} {xq} {ff} {fq} {y} {G}"
    got = oracle_mod.run_circuit(wl.circuit_text(n, [line]), psi0=psi)
    want = np.empty_like(psi)
    for i in range(2 ** n):
        x = (i >> xf) & (2 ** xq - 1)
        j = i ^ (pow(y, x, G) << ff)
        want[j] = psi[i]
    assert np.array_equal(got, want)
    back = oracle_mod.run_circuit(wl.circuit_text(n, [line]), psi0=got)
    assert np.array_equal(back, psi)


def test_oracle_shor_small_full_circuit(oracle_mod):
    """G = 15 = 3 x 5, y = 7 (period 4), X = 8, F = 4: the simulated x-register marginals equal the
    Fourier-sum prediction."""
    L, X, G, y = 12, 8, 15, 7
    psi = oracle_mod.run_circuit(wl.shor_circuit(L, X, G, y))
    q = oracle_mod.marginals(psi)[:X]
    r = oracle_mod.multiplicative_order(y, G)
    assert r == 4
    assert np.max(np.abs(q - oracle_mod.shor_expectations(X, r))) < 1e-13


def test_oracle_shor_L24_table(oracle_mod):
    """Table Shortab, first column (L = 24, X = 16, G = 247, y = 194): the full circuit on the oracle
    gives the printed <Q_i> and the Fourier-sum values."""
    L, X, G, y, r, q = shor_rows()[0]
    psi = oracle_mod.run_circuit(wl.shor_circuit(L, X, G, y))
    got = oracle_mod.marginals(psi)[:X]
    assert np.max(np.abs(got - oracle_mod.shor_expectations(X, r))) < 1e-12
    assert np.max(np.abs(got - np.array(q))) <= 5e-4 + 1e-12
