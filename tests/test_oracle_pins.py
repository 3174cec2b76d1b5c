"""Pins of the FP64 CPU oracle against what the paper and plain mathematics fix.

Each test checks the oracle against something other than itself: amplitude maps and register
identities printed in (or following directly from) the paper, textbook dense matrices built with
Kronecker products, closed-form identities between gates, the discrete Fourier transform, and
integer addition. A dropped term, a wrong sign, a wrong bit index or a transposed matrix in any
rule of the oracle fails at least one of them.
"""
import cmath
import functools
import itertools
import math
import os

import numpy as np
import pytest

import qsim_workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore")


def rand_state(n, seed):
    return wl.gaussian_state(n, seed)


def run(oracle_mod, n, lines, psi0):
    return oracle_mod.run_circuit(wl.circuit_text(n, lines), psi0=psi0)


# ----------------------------------------------------------------------------------------------
# Worked amplitude maps (Eqs. CNOT2, COMM5, COMM4, Toffoli)
# ----------------------------------------------------------------------------------------------
def _worked_maps():
    out = []
    with open(os.path.join(GOLD, "worked_maps.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            gate, n, outs = [s.strip() for s in ln.split("|")]
            out.append((gate, int(n), [s.strip() for s in outs.split(";")]))
    return out


def _eval_expr(expr, a, phi):
    e = cmath.exp(1j * phi)
    env = {"e": e, "p": (1 + e) / 2, "m": (1 - e) / 2}
    env.update({f"a{k}": a[k] for k in range(len(a))})
    return eval(expr, {"__builtins__": {}}, env)


@pytest.mark.parametrize("case", _worked_maps(), ids=lambda c: c[0].split()[0])
def test_worked_maps(oracle_mod, case):
    gate, n, outs = case
    phi = 0.7390851332151607
    psi = rand_state(n, 5)
    line = gate.replace("PHI", float(phi).hex())
    got = run(oracle_mod, n, [line], psi)
    want = np.array([_eval_expr(x, psi, phi) for x in outs])
    assert np.max(np.abs(got - want)) < 1e-15


@pytest.mark.parametrize("case", _worked_maps(), ids=lambda c: c[0].split()[0])
def test_worked_maps_embedded(oracle_mod, case):
    """The same maps with the gate qubits placed at random positions among spectator qubits."""
    gate, k, outs = case
    kw, *rest = gate.split()
    nq = k
    rng = np.random.default_rng(7)
    phi = 1.9
    for n in (4, 6):
        for _ in range(6):
            pos = [int(x) for x in rng.permutation(n)[:nq]]   # gate qubit s of the map -> pos[s]
            args = [str(pos[int(x)]) if x.isdigit() else float(phi).hex() for x in rest]
            psi = rand_state(n, int(rng.integers(1 << 30)))
            got = run(oracle_mod, n, [" ".join([kw] + args)], psi)
            want = np.empty_like(psi)
            others = [q for q in range(n) if q not in pos]
            for rest_bits in range(2 ** (n - nq)):
                base = 0
                for s, q in enumerate(others):
                    if (rest_bits >> s) & 1:
                        base |= 1 << q
                idx = []
                for local in range(2 ** nq):
                    x = base
                    for s in range(nq):
                        if (local >> s) & 1:
                            x |= 1 << pos[s]
                    idx.append(x)
                a = [psi[x] for x in idx]
                for local in range(2 ** nq):
                    want[idx[local]] = _eval_expr(outs[local], a, phi)
            assert np.max(np.abs(got - want)) < 1e-15


# ----------------------------------------------------------------------------------------------
# Register preparation identities (Sec. V; Eqs. Xoperation, Yoperation)
# ----------------------------------------------------------------------------------------------
def test_register_preparation(oracle_mod):
    with open(os.path.join(GOLD, "register_preparation.txt")) as f:
        rows = [ln.split("|") for ln in f if ln.strip() and not ln.startswith("#")]
    for kw, amp in rows:
        kw = kw.strip()
        re_, im_ = [float(x) for x in amp.split()]
        got = oracle_mod.run_circuit(wl.circuit_text(1, [f"{kw} 0", f"{kw} 0"]))
        assert abs(got[0]) < 1e-16
        assert abs(got[1] - complex(re_, im_)) < 4e-16


# ----------------------------------------------------------------------------------------------
# Index logic: every rule against a textbook dense matrix built from Kronecker products
# ----------------------------------------------------------------------------------------------
I2 = np.eye(2)
P1 = np.diag([0.0, 1.0])


def kron_all(mats_by_qubit):
    """mats_by_qubit[q] acts on qubit q; qubit 0 is the least significant bit -> rightmost factor."""
    return functools.reduce(np.kron, [mats_by_qubit[q] for q in reversed(range(len(mats_by_qubit)))])


def controlled_dense(n, target, U, controls=()):
    """I - P + P(U on target), P = projector onto 'all controls are 1'."""
    ident = np.eye(2 ** n, dtype=np.complex128)
    proj = kron_all([P1 if q in controls else I2 for q in range(n)])
    full = kron_all([P1 if q in controls else (U if q == target else I2) for q in range(n)])
    return ident - proj + full


def haar(rng):
    return wl.haar_2x2(rng)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_unitary_rule_all_targets_and_controls(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    for t in range(n):
        others = [q for q in range(n) if q != t]
        for nc in range(0, min(3, n - 1) + 1):
            for ctrl in itertools.combinations(others, nc):
                U = haar(rng)
                psi = rand_state(n, int(rng.integers(1 << 30)))
                want = controlled_dense(n, t, U, ctrl) @ psi
                a = oracle_mod.to_interleaved(psi)
                cm = sum(1 << c for c in ctrl)
                oracle_mod.lib().or_unitary(oracle_mod._dp(a), n, t, cm, oracle_mod._dp(oracle_mod._u8(U)))
                assert np.max(np.abs(oracle_mod.to_complex(a) - want)) < 1e-14


@pytest.mark.parametrize("n", [2, 4, 6])
def test_cnot_toffoli_phase_cv_swap_rules(oracle_mod, n):
    rng = np.random.default_rng(200 + n)
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    for t in range(n):
        others = [q for q in range(n) if q != t]
        for nc in range(0, min(2, n - 1) + 1):
            for ctrl in itertools.combinations(others, nc):
                psi = rand_state(n, int(rng.integers(1 << 30)))
                cm = sum(1 << c for c in ctrl)
                # NUM6 / NUM8: a flip of the target on the controlled subspace
                a = oracle_mod.to_interleaved(psi)
                oracle_mod.lib().or_cnot(oracle_mod._dp(a), n, cm, t)
                got = oracle_mod.to_complex(a)
                want = controlled_dense(n, t, X, ctrl) @ psi
                assert np.array_equal(got, want)  # a permutation: exact
                # NUM5 / COMM5: phase on |1> of the target, controlled
                phi = float(rng.uniform(0, 2 * np.pi))
                a = oracle_mod.to_interleaved(psi)
                oracle_mod.lib().or_phase(oracle_mod._dp(a), n, t, cm, phi)
                want = controlled_dense(n, t, np.diag([1, cmath.exp(1j * phi)]), ctrl) @ psi
                assert np.max(np.abs(oracle_mod.to_complex(a) - want)) < 1e-15
                # NUM7: controlled V
                e = cmath.exp(1j * phi)
                V = 0.5 * np.array([[1 + e, 1 - e], [1 - e, 1 + e]])
                a = oracle_mod.to_interleaved(psi)
                oracle_mod.lib().or_cv(oracle_mod._dp(a), n, cm, t, phi)
                want = controlled_dense(n, t, V, ctrl) @ psi
                assert np.max(np.abs(oracle_mod.to_complex(a) - want)) < 1e-15
    # quantum swap: permutation matrix exchanging bits p and q of every index
    for p, q in itertools.permutations(range(n), 2):
        psi = rand_state(n, p * 31 + q)
        want = np.empty_like(psi)
        for x in range(2 ** n):
            bp, bq = (x >> p) & 1, (x >> q) & 1
            y = x & ~((1 << p) | (1 << q)) | (bq << p) | (bp << q)
            want[y] = psi[x]
        got = run(oracle_mod, n, [f"QSWAP {p} {q}"], psi)
        assert np.array_equal(got, want)


def test_hadamard_and_rotation_rules_dense(oracle_mod):
    """NUM2, NUM3, NUM4 for every target of a 4-qubit state, against the matrices of Eqs.
    Hadamard, Xoperation and Yoperation embedded with Kronecker products."""
    s = 1 / math.sqrt(2)
    mats = {
        "H": s * np.array([[1, 1], [1, -1]]),
        "RX90": s * np.array([[1, 1j], [1j, 1]]),
        "RY90": s * np.array([[1, 1], [-1, 1]]),
    }
    mats["RX90DG"] = mats["RX90"].conj().T
    mats["RY90DG"] = mats["RY90"].conj().T
    n = 4
    for kw, U in mats.items():
        for t in range(n):
            psi = rand_state(n, 300 + t)
            got = run(oracle_mod, n, [f"{kw} {t}"], psi)
            want = controlled_dense(n, t, U) @ psi
            assert np.max(np.abs(got - want)) < 1e-15, kw


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (5, 3), (6, 3), (7, 4), (6, 5)])
def test_dense_k_qubit_rule(oracle_mod, n, k):
    """A k-qubit dense gate on an unsorted qubit list equals the textbook embedding: permute the qubit
    order so that qubits[s] becomes position s, apply U (x) I, permute back."""
    rng = np.random.default_rng(400 + 10 * n + k)
    for _ in range(3):
        qubits = [int(x) for x in rng.permutation(n)[:k]]
        Z = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
        U, _ = np.linalg.qr(Z)
        psi = rand_state(n, int(rng.integers(1 << 30)))
        got = oracle_mod.apply_dense(psi, qubits, U)
        order = qubits + [q for q in range(n) if q not in qubits]  # new bit s <- old bit order[s]
        want = np.zeros_like(psi)
        for x in range(2 ** n):
            y = sum(((x >> order[s]) & 1) << s for s in range(n))
            lo, hi = y & (2 ** k - 1), y >> k
            for r in range(2 ** k):
                yy = (hi << k) | r
                xx = sum(((yy >> s) & 1) << order[s] for s in range(n))
                want[xx] += U[r, lo] * psi[x]
        assert np.max(np.abs(got - want)) < 1e-14


# ----------------------------------------------------------------------------------------------
# Closed-form identities between gates
# ----------------------------------------------------------------------------------------------
def _one_qubit_matrix(oracle_mod, lines):
    cols = []
    for b in range(2):
        cols.append(oracle_mod.run_circuit(wl.circuit_text(1, lines, initial_state=b)))
    return np.array(cols).T


def test_gate_identities(oracle_mod):
    m = lambda *ls: _one_qubit_matrix(oracle_mod, list(ls))
    I = np.eye(2)
    tol = 1e-15
    assert np.max(np.abs(m("H 0", "H 0") - I)) < 4 * tol
    # (paper's X)^4 = exp(2 pi i S^x) = -I, same for Y
    assert np.max(np.abs(m("RX90 0", "RX90 0", "RX90 0", "RX90 0") + I)) < 8 * tol
    assert np.max(np.abs(m("RY90 0", "RY90 0", "RY90 0", "RY90 0") + I)) < 8 * tol
    assert np.max(np.abs(m("RX90 0", "RX90DG 0") - I)) < 4 * tol
    assert np.max(np.abs(m("RY90 0", "RY90DG 0") - I)) < 4 * tol
    # the paper's X^2 = i sigma_x, Y^2 = i sigma_y
    assert np.max(np.abs(m("RX90 0", "RX90 0") - 1j * np.array([[0, 1], [1, 0]]))) < 4 * tol
    assert np.max(np.abs(m("RY90 0", "RY90 0") - 1j * np.array([[0, -1j], [1j, 0]]))) < 4 * tol
    # Pauli algebra: XYZ = iI, S^2 = Z, T^2 = S, S SDG = I, T TDG = I
    assert np.max(np.abs(m("Z 0", "Y 0", "X 0") - 1j * I)) < tol  # Z first, X last: XYZ = iI
    assert np.max(np.abs(m("S 0", "S 0") - m("Z 0"))) < tol
    assert np.max(np.abs(m("T 0", "T 0") - m("S 0"))) < 4 * tol
    assert np.max(np.abs(m("S 0", "SDG 0") - I)) < tol
    assert np.max(np.abs(m("T 0", "TDG 0") - I)) < 4 * tol
    # R(phi) = e^{i phi/2} RZ(phi) (Eq. singlephase); R(pi/2) = S, R(pi/4) = T, RK k = R(2pi/2^k)
    for phi in (0.3, 1.7, 4.0):
        h = float(phi).hex()
        assert np.max(np.abs(m(f"R 0 {h}") - cmath.exp(0.5j * phi) * m(f"RZ 0 {h}"))) < 4 * tol
    assert np.max(np.abs(m(f"R 0 {(math.pi / 2).hex()}") - m("S 0"))) < 4 * tol
    assert np.max(np.abs(m(f"R 0 {(math.pi / 4).hex()}") - m("T 0"))) < 4 * tol
    assert np.max(np.abs(m("RK 0 2") - m("S 0"))) < 4 * tol
    assert np.max(np.abs(m("RK 0 3") - m("T 0"))) < 4 * tol
    assert np.max(np.abs(m("RK 0 1") - m("Z 0"))) < 4 * tol
    assert np.max(np.abs(m("RK 0 5", "RKDG 0 5") - I)) < 4 * tol
    # H R(pi) H = sigma_x ; H Z H = X
    assert np.max(np.abs(m("H 0", "Z 0", "H 0") - m("X 0"))) < 4 * tol
    # every matrix is unitary
    for g in ["H 0", "X 0", "Y 0", "Z 0", "S 0", "T 0", "RX90 0", "RY90 0", "RX90DG 0",
              "RY90DG 0", f"RZ 0 {(2.5).hex()}", f"R 0 {(0.9).hex()}", "RK 0 7"]:
        u = m(g)
        assert np.max(np.abs(u.conj().T @ u - I)) < 4 * tol, g


def test_two_qubit_identities(oracle_mod):
    def mat(lines, n=2):
        return np.array([oracle_mod.run_circuit(wl.circuit_text(n, lines, initial_state=b))
                         for b in range(2 ** n)]).T
    tol = 4e-16
    # controlled V(pi) is the CNOT (Sec. II.C: CNOT is a special case of controlled V)
    assert np.max(np.abs(mat([f"CV 0 1 {math.pi.hex()}"]) - mat(["CNOT 0 1"]))) < 4 * tol
    # CZ = CPHASE(pi) = CRK 1, and is symmetric in its qubits
    assert np.max(np.abs(mat(["CZ 0 1"]) - mat([f"CPHASE 0 1 {math.pi.hex()}"]))) < tol
    assert np.max(np.abs(mat(["CZ 0 1"]) - mat(["CZ 1 0"]))) == 0
    assert np.max(np.abs(mat(["CRK 0 1 3"]) - mat(["CRK 1 0 3"]))) == 0
    # CNOT = (I x H) CZ (I x H) with the target in the middle
    assert np.max(np.abs(mat(["H 1", "CZ 0 1", "H 1"]) - mat(["CNOT 0 1"]))) < 4 * tol
    # SWAP = three CNOTs
    assert np.array_equal(mat(["QSWAP 0 1"]), mat(["CNOT 0 1", "CNOT 1 0", "CNOT 0 1"]))
    # Toffoli on 3 qubits: a permutation matrix swapping |011> and |111> (Eq. Toffoli)
    T = mat(["TOFFOLI 0 1 2"], n=3)
    P = np.eye(8)
    P[:, [3, 7]] = P[:, [7, 3]]
    assert np.array_equal(T, P)


# ----------------------------------------------------------------------------------------------
# Invariants and closed forms on whole circuits
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 5, 12, 16])
def test_hadamard_on_every_qubit(oracle_mod, n):
    """App. A example: H on every qubit of |0...0> gives the uniform superposition; <Q_i> = 1/2."""
    psi = oracle_mod.run_circuit(wl.circuit_text(n, [f"H {q}" for q in range(n)]))
    ref = 2.0 ** (-n / 2)
    assert np.max(np.abs(psi.real - ref)) <= 4 * np.spacing(ref) * n
    assert np.max(np.abs(psi.imag)) == 0
    assert np.allclose(oracle_mod.marginals(psi), 0.5, atol=1e-14)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_norm_preserved_random_circuit(oracle_mod, seed):
    text = wl.config0_circuit(12, 200, seed)
    psi = oracle_mod.run_circuit(text)
    assert abs(oracle_mod.norm(psi) - 1.0) < 1e-13


def _dft(psi):
    """2^{-n/2} sum_x psi_x e^{+2 pi i (x k mod 2^n) / 2^n}, twiddles reduced exactly."""
    N = psi.size
    x = np.arange(N)
    out = np.empty(N, dtype=np.complex128)
    for k in range(N):
        ph = (x * k) % N
        out[k] = np.sum(psi * np.exp(2j * np.pi * ph / N)) / math.sqrt(N)
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 6, 10])
def test_qft_equals_dft(oracle_mod, n):
    psi = rand_state(n, 12)
    got = oracle_mod.run_circuit(wl.qft_circuit(n), psi0=psi)
    assert np.max(np.abs(got - _dft(psi))) < 1e-13


def test_qft_equals_fft_library(oracle_mod):
    n = 16
    psi = rand_state(n, 12)
    got = oracle_mod.run_circuit(wl.qft_circuit(n), psi0=psi)
    want = np.fft.ifft(psi, norm="ortho")
    assert np.max(np.abs(got - want)) < 1e-13


def test_qft_inverse_round_trip(oracle_mod):
    n = 9
    psi = rand_state(n, 3)
    lines = wl.qft_lines(list(range(n))) + wl.iqft_lines(list(range(n)))
    got = run(oracle_mod, n, lines, psi)
    assert np.max(np.abs(got - psi)) < 1e-14


def _adder_check(oracle_mod, m, pairs):
    text, lay = wl.ripple_adder_circuit(m)
    n = lay["n"]
    for a, b in pairs:
        x = a | (b << m)
        c = oracle_mod.parse(text)
        st = oracle_mod.basis_state(n, x)
        for kw, args in c.ops:
            oracle_mod.apply_op(st, n, kw, args)
        psi = oracle_mod.to_complex(st)
        want = a | (((a + b) % 2 ** m) << m)
        assert psi[want] == 1.0 and np.count_nonzero(psi) == 1, (a, b)


def test_ripple_adder_exhaustive_small(oracle_mod):
    m = 3
    _adder_check(oracle_mod, m, [(a, b) for a in range(2 ** m) for b in range(2 ** m)])


def test_ripple_adder_random_8bit(oracle_mod):
    _adder_check(oracle_mod, 8, wl.adder_operands(8, 12, seed=11))


def test_probs_and_marginals_basis(oracle_mod):
    n = 7
    x = 0b1011001
    psi = oracle_mod.to_complex(oracle_mod.basis_state(n, x))
    q = oracle_mod.marginals(psi)
    assert list(q) == [float((x >> i) & 1) for i in range(n)]
    p = oracle_mod.probs(psi)
    assert p[x] == 1.0 and p.sum() == 1.0


# ----------------------------------------------------------------------------------------------
# The two error-metric and Fourier helpers used as references by the GPU tests
# ----------------------------------------------------------------------------------------------
def _orthogonal_to(psi, seed):
    """A normalised state orthogonal to psi (Gram-Schmidt of a seeded Gaussian vector)."""
    v = wl.gaussian_state(int(round(math.log2(psi.size))), seed).astype(np.complex128)
    u = psi / np.linalg.norm(psi)
    v = v - np.vdot(u, v) * u
    return v / np.linalg.norm(v)


def test_infidelity_closed_forms(oracle_mod):
    """1 - F with F = |<ref|psi>|^2 / (<ref|ref><psi|psi>): 0 for a global phase and any scaling,
    1 for orthogonal states, sin^2 t for cos t ref + sin t e^{ia} ref_perp (a missing conjugate, a
    missing norm factor or a swapped argument order changes at least one of these)."""
    n = 10
    ref = wl.gaussian_state(n, 41).astype(np.complex128)
    perp = _orthogonal_to(ref, 42)
    for phase in (0.0, 0.3, 2.1, math.pi):
        assert abs(oracle_mod.infidelity(np.exp(1j * phase) * ref, ref)) < 1e-14
    assert abs(oracle_mod.infidelity(3.0 * ref, ref)) < 1e-14
    assert abs(oracle_mod.infidelity(ref, 0.25j * ref)) < 1e-14
    assert abs(oracle_mod.infidelity(perp, ref) - 1.0) < 1e-14
    for t in (1e-3, 0.2, 0.7, 1.3):
        for a in (0.0, 1.1):
            psi = math.cos(t) * ref + math.sin(t) * np.exp(1j * a) * perp
            want = math.sin(t) ** 2
            assert abs(oracle_mod.infidelity(psi, ref) - want) < 1e-13 * max(1.0, want / 1e-6)
            # symmetric in its two arguments
            assert abs(oracle_mod.infidelity(ref, psi) - want) < 1e-13 * max(1.0, want / 1e-6)


def test_max_abs_diff_is_complex_modulus(oracle_mod):
    a = np.array([1 + 1j, 0.5, -2j])
    b = np.array([1 + 1j, 0.5 + 0.3j, 2j])
    assert oracle_mod.max_abs_diff(a, b) == 4.0
    assert oracle_mod.max_abs_diff(a, a) == 0.0
    assert abs(oracle_mod.max_abs_diff(np.array([3 + 4j]), np.array([0j])) - 5.0) < 1e-15


@pytest.mark.parametrize("n", [1, 4, 9, 12])
def test_qft_sample_equals_gate_level_qft(oracle_mod, n):
    """The sampled Fourier outputs (one O(2^n) sum per k) equal, at every k, the state that the
    gate-level QFT circuit (Hadamards, controlled phase shifts 2 pi / 2^k, bit-reversal swaps)
    produces in the oracle, whose circuit is pinned to the DFT and to numpy's FFT above."""
    psi = rand_state(n, 70 + n)
    full = oracle_mod.run_circuit(wl.qft_circuit(n), psi0=psi)
    ks = list(range(2 ** n))
    got = oracle_mod.qft_sample(psi, ks)
    assert np.max(np.abs(got - full)) < 1e-13


def test_qft_sample_equals_fft_library(oracle_mod):
    """numpy's inverse FFT with orthonormal scaling is the same transform (sign +2 pi i x k / N)."""
    n = 16
    psi = rand_state(n, 12)
    rng = np.random.default_rng(16)
    ks = [0, 1, 2, 2 ** (n - 1), 2 ** n - 1] + [int(k) for k in rng.integers(0, 2 ** n, size=27)]
    got = oracle_mod.qft_sample(psi, ks)
    want = np.fft.ifft(psi, norm="ortho")[ks]
    assert np.max(np.abs(got - want)) < 1e-13


def test_qft_sample_closed_forms(oracle_mod):
    """Basis state |x>: out_k = 2^{-n/2} e^{2 pi i x k / 2^n}; uniform state: out_k = [k = 0]."""
    n = 11
    N = 2 ** n
    for x in (0, 1, 5, N - 1, 1234):
        psi = np.zeros(N, dtype=np.complex128)
        psi[x] = 1.0
        ks = [0, 1, 3, 700, N - 1]
        want = np.array([cmath.exp(2j * math.pi * ((x * k) % N) / N) for k in ks]) / math.sqrt(N)
        assert np.max(np.abs(oracle_mod.qft_sample(psi, ks) - want)) < 1e-14
    u = np.full(N, 1.0 / math.sqrt(N), dtype=np.complex128)
    got = oracle_mod.qft_sample(u, [0, 1, 2, N // 2, N - 1])
    assert abs(got[0] - 1.0) < 1e-13 and np.max(np.abs(got[1:])) < 1e-13


# ----------------------------------------------------------------------------------------------
# Renormalisation points (Eq. STAT1)
# ----------------------------------------------------------------------------------------------
def test_renorm_rescales_to_unit_sum(oracle_mod):
    """RENORM divides every amplitude by the same positive number and leaves sum |a_i|^2 = 1 (Eq.
    STAT1); the factor is checked against numpy's own 2-norm, not the oracle's sum."""
    n = 7
    psi = 3.7 * rand_state(n, 11)
    out = run(oracle_mod, n, ["RENORM"], psi)
    r = float(np.linalg.norm(psi))
    assert abs(float(np.sum(np.abs(out) ** 2)) - 1.0) < 1e-14
    np.testing.assert_allclose(out * r, psi, rtol=0, atol=1e-13 * r)


def test_renorm_special_cases(oracle_mod):
    n = 5
    e = np.zeros(2 ** n, dtype=np.complex128)
    e[9] = 1.0
    assert np.array_equal(run(oracle_mod, n, ["RENORM"], e), e)  # already normalised: unchanged
    z = np.zeros(2 ** n, dtype=np.complex128)
    assert np.array_equal(run(oracle_mod, n, ["RENORM"], z), z)  # sum 0: left as it is
    neg = -2.0j * e
    np.testing.assert_allclose(run(oracle_mod, n, ["RENORM"], neg), -1.0j * e, rtol=0, atol=1e-16)  # phase kept


def test_renorm_commutes_with_unitary_gates(oracle_mod):
    """Unitary gates keep sum |a_i|^2, so a RENORM anywhere between them gives the unrenormalised
    result divided by the initial 2-norm; two RENORMs in a row act as one."""
    n = 6
    psi = 0.4 * rand_state(n, 5)
    gates = ["H 0", "CNOT 0 3", "RX90 2", "CRK 1 4 3", "QSWAP 2 5", "TOFFOLI 0 1 5", "RY90DG 4"]
    plain = run(oracle_mod, n, gates, psi)
    r = float(np.linalg.norm(psi))
    for k in (0, 3, len(gates)):
        for extra in (["RENORM"], ["RENORM", "RENORM"]):
            got = run(oracle_mod, n, gates[:k] + extra + gates[k:], psi)
            np.testing.assert_allclose(got, plain / r, rtol=0, atol=1e-14)
