"""GPU parity: every C-ABI call of libqsim against the FP64 CPU oracle on the same seeded inputs.

Bars: permutation work (X, CNOT, Toffoli, quantum swap, adders on basis states) is bit-exact;
complex128 results are within max|d amp| <= 1e-12 of the oracle; complex64 single-gate results
within 2e-6 and circuit results within 1 - F <= 1e-6 of the FP64 oracle.
"""
import itertools
import math

import numpy as np
import pytest

import qsim_workloads as wl

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64_GATE = 2e-6
TOL64_FID = 1e-6


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0608239_amd as q
    q.lib()
    return q


def gpu_state(q, psi, dtype):
    n = int(round(math.log2(psi.size)))
    s = q.State(n, dtype)
    s.upload(psi)
    return s


def oracle_line(oracle_mod, psi, line):
    n = int(round(math.log2(psi.size)))
    return oracle_mod.run_circuit(wl.circuit_text(n, [line]), psi0=psi)


def u_line_args(U):
    return " ".join(float(v).hex() for v in np.asarray(U, np.complex128).reshape(-1).view(np.float64))


def check(got, want, dtype, what=""):
    got = np.asarray(got, np.complex128)
    d = np.max(np.abs(got - want)) if got.size else 0.0
    tol = TOL128 if dtype == "c128" else TOL64_GATE
    assert d <= tol, f"{what}: max|d| = {d:.3e} > {tol}"


DTYPES = ["c128", "c64"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11])
def test_apply_1q_every_target(q, oracle_mod, dtype, n):
    rng = np.random.default_rng(1000 + n)
    psi = wl.gaussian_state(n, 77 + n)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    for t in range(n):
        U = wl.haar_2x2(rng)
        s.apply_1q(t, U)
        ref = oracle_line(oracle_mod, ref, f"U {t} {u_line_args(U)}")
    check(s.download(), ref, dtype, f"n={n}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_apply_1q_specialised_forms(q, oracle_mod, dtype):
    """Diagonal (Eq. NUM5 form and general diag), X as a swap, identity: the classified paths."""
    n = 9
    rng = np.random.default_rng(5)
    psi = wl.gaussian_state(n, 5)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    mats = [np.diag([1, np.exp(0.3j)]), np.diag([np.exp(-0.7j), np.exp(1.1j)]), np.array([[0, 1], [1, 0]]),
            np.eye(2), np.array([[0, -1j], [1j, 0]])]
    for t in [0, 1, 4, 8]:
        for U in mats:
            s.apply_1q(t, U)
            ref = oracle_line(oracle_mod, ref, f"U {t} {u_line_args(U)}")
    check(s.download(), ref, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [3, 6, 10])
def test_apply_ctrl_targets_and_control_sets(q, oracle_mod, dtype, n):
    rng = np.random.default_rng(2000 + n)
    psi = wl.gaussian_state(n, 88 + n)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    for t in range(n):
        others = [x for x in range(n) if x != t]
        for nc in range(1, min(3, n - 1) + 1):
            sets = list(itertools.combinations(others, nc))
            rng.shuffle(sets)
            for C in sets[:3]:
                U = wl.haar_2x2(rng)
                mask = sum(1 << c for c in C)
                s.apply_ctrl(mask, t, U)
                a = oracle_mod.to_interleaved(ref)
                oracle_mod.lib().or_unitary(oracle_mod._dp(a), n, t, mask, oracle_mod._dp(oracle_mod._u8(U)))
                ref = oracle_mod.to_complex(a).copy()
    check(s.download(), ref, dtype, f"n={n}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_permutations_bit_exact(q, oracle_mod, dtype):
    """CNOT, Toffoli, 3-control X and quantum swaps move amplitudes without arithmetic."""
    n = 11
    psi = wl.gaussian_state(n, 9)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)  # exactly representable input
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    X = np.array([[0, 1], [1, 0]])
    rng = np.random.default_rng(3)
    for _ in range(40):
        k = int(rng.integers(0, 4))
        qs = [int(x) for x in rng.permutation(n)[:k + 1]]
        t, C = qs[0], qs[1:]
        mask = sum(1 << c for c in C)
        s.apply_ctrl(mask, t, X)
        a = oracle_mod.to_interleaved(ref)
        oracle_mod.lib().or_cnot(oracle_mod._dp(a), n, mask, t)
        ref = oracle_mod.to_complex(a).copy()
        a0, b0 = [int(x) for x in rng.permutation(n)[:2]]
        s.apply_swap(a0, b0)
        ref = oracle_line(oracle_mod, ref, f"QSWAP {a0} {b0}")
    got = s.download().astype(np.complex128)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_apply_phase_device_angles(q, oracle_mod, dtype):
    n = 10
    psi = wl.gaussian_state(n, 21)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    rng = np.random.default_rng(4)
    for t in range(n):
        for nc in range(0, 3):
            C = [int(x) for x in rng.permutation([x for x in range(n) if x != t])[:nc]]
            mask = sum(1 << c for c in C)
            th = float(rng.uniform(0, 2 * np.pi))
            s.apply_phase(mask, t, th)
            a = oracle_mod.to_interleaved(ref)
            oracle_mod.lib().or_phase(oracle_mod._dp(a), n, t, mask, th)
            ref = oracle_mod.to_complex(a).copy()
    check(s.download(), ref, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,k", [(3, 1), (5, 2), (7, 3), (8, 4), (9, 5), (12, 4), (12, 5), (16, 5), (17, 3)])
def test_apply_fused_unsorted_qubits(q, oracle_mod, dtype, n, k):
    rng = np.random.default_rng(3000 + 10 * n + k)
    psi = wl.gaussian_state(n, 31 + n)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    for rep in range(3):
        qubits = [int(x) for x in rng.permutation(n)[:k]]
        if rep == 0:
            qubits = sorted(qubits)
        Z = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
        U, _ = np.linalg.qr(Z)
        s.apply_fused(qubits, U)
        ref = oracle_mod.apply_dense(ref, qubits, U)
    check(s.download(), ref, dtype, f"n={n} k={k}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_fused_low_qubits(q, oracle_mod, dtype):
    """Fused gates on the lowest qubits (partners inside one 64-byte run) and on mixed low/high sets."""
    n = 14
    rng = np.random.default_rng(17)
    psi = wl.gaussian_state(n, 17)
    s = gpu_state(q, psi, dtype)
    ref = psi.copy()
    for qubits in ([0, 1, 2, 3, 4], [4, 3, 2, 1, 0], [0, 13, 5, 2], [13, 12, 11, 10, 9], [1, 7, 3]):
        k = len(qubits)
        Z = rng.standard_normal((2 ** k, 2 ** k)) + 1j * rng.standard_normal((2 ** k, 2 ** k))
        U, _ = np.linalg.qr(Z)
        s.apply_fused(qubits, U)
        ref = oracle_mod.apply_dense(ref, qubits, U)
    check(s.download(), ref, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 4, 9, 13, 20])
def test_reductions(q, oracle_mod, dtype, n):
    psi = wl.gaussian_state(n, 40 + n) * 0.75
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    s = gpu_state(q, psi, dtype)
    nrm = s.norm()
    assert abs(nrm - oracle_mod.norm(psi)) <= 1e-14
    p = s.probs()
    assert np.max(np.abs(p - oracle_mod.probs(psi))) <= 1e-16
    pd = s.probs(device=True).cpu().numpy()
    assert np.array_equal(pd, p)
    m = s.marginals()
    assert np.max(np.abs(m - oracle_mod.marginals(psi))) <= 1e-14
    before = s.renormalize()
    assert abs(before - nrm) <= 1e-15 * max(1.0, nrm)
    got = s.download().astype(np.complex128)
    want = psi / math.sqrt(oracle_mod.norm(psi))
    check(got, want, dtype)
    assert abs(s.norm() - 1.0) <= (1e-14 if dtype == "c128" else 1e-6)


def test_reduction_determinism(q):
    n = 22
    psi = wl.gaussian_state(n, 3)
    s = gpu_state(q, psi, "c128")
    vals = {s.norm() for _ in range(3)}
    assert len(vals) == 1


@pytest.mark.parametrize("dtype", DTYPES)
def test_sampling(q, dtype):
    """Sampling of the final state (Sec. V): a basis state always yields its index; a two-outcome
    state yields each index at the inverse-CDF cut."""
    n = 15
    s = q.State(n, dtype)
    s.set_basis(12345)
    assert list(s.sample([0.0, 0.5, 0.999999])) == [12345] * 3
    psi = np.zeros(2 ** n, np.complex128)
    psi[3] = math.sqrt(0.25)
    psi[2 ** n - 2] = math.sqrt(0.75) * 1j
    s.upload(psi)
    out = s.sample([0.0, 0.1, 0.2499, 0.2501, 0.6, 0.99])
    assert list(out) == [3, 3, 3, 2 ** n - 2, 2 ** n - 2, 2 ** n - 2]


def run_gpu(q, text, dtype, method="plain", psi0=None, fuse_k=5, use_graph=False, reps=1):
    c = q.parse_circuit(text)
    s = q.State(c.n, dtype)
    p = q.Plan(c, dtype, method=method, fuse_k=fuse_k, use_graph=use_graph)
    outs = []
    for _ in range(reps):
        if psi0 is None:
            s.set_basis(c.init)
        else:
            s.upload(psi0)
        p.execute(s)
        outs.append(s.download().astype(np.complex128))
    return outs[-1] if reps == 1 else outs, p


def compare_circuit(got, ref, dtype, what):
    if dtype == "c128":
        d = np.max(np.abs(got - ref))
        assert d <= TOL128, f"{what}: max|d| = {d:.3e}"
    else:
        import oracle
        f = oracle.infidelity(got, ref)
        assert f <= TOL64_FID, f"{what}: 1-F = {f:.3e}"


@pytest.mark.parametrize("method", ["plain", "fused"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_config0_random_circuit(q, oracle_mod, method, seed):
    """16 qubits, complex128: H on every qubit then 200 random gates (start |0...0>)."""
    text = wl.config0_circuit(16, 200, seed)
    ref = oracle_mod.run_circuit(text)
    got, p = run_gpu(q, text, "c128", method)
    compare_circuit(got, ref, "c128", f"seed {seed} {method}")
    assert abs(np.sum(np.abs(got) ** 2) - 1) < 1e-13


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("method,k", [("plain", 5), ("fused", 2), ("fused", 3), ("fused", 4), ("fused", 5)])
def test_brickwork_small(q, oracle_mod, dtype, method, k):
    text = wl.brickwork_circuit(14, 6, seed=21)
    ref = oracle_mod.run_circuit(text)
    got, p = run_gpu(q, text, dtype, method, fuse_k=k)
    compare_circuit(got, ref, dtype, f"{method} k={k}")
    if method == "fused":
        assert p.info["launches"] < p.info["gates"]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("method", ["plain", "fused"])
@pytest.mark.parametrize("n", [6, 12, 18])
def test_qft_gaussian_state(q, oracle_mod, dtype, method, n):
    psi = wl.gaussian_state(n, 12)
    text = wl.qft_circuit(n)
    ref = oracle_mod.run_circuit(text, psi0=psi)
    got, _ = run_gpu(q, text, dtype, method, psi0=psi)
    compare_circuit(got, ref, dtype, f"qft n={n} {method}")


@pytest.mark.parametrize("method", ["plain", "fused"])
def test_ripple_adder_bit_exact_small(q, method):
    m = 4
    text, lay = wl.ripple_adder_circuit(m)
    c = q.parse_circuit(text)
    p = q.Plan(c, "c128", method=method)
    s = q.State(lay["n"], "c128")
    for a in range(2 ** m):
        for b in range(0, 2 ** m, 3):
            s.set_basis(a | (b << m))
            p.execute(s)
            got = s.download()
            want = a | (((a + b) % 2 ** m) << m)
            assert got[want] == 1.0 and np.count_nonzero(got) == 1, (a, b)


def test_graph_replay_matches_eager(q, oracle_mod):
    """A plan recorded in a HIP graph, replayed several times with eager work in between."""
    import torch
    text = wl.config0_circuit(12, 120, seed=5)
    ref = oracle_mod.run_circuit(text)
    c = q.parse_circuit(text)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        s = q.State(c.n, "c128")
        p = q.Plan(c, "c128", method="fused", use_graph=True)
        for rep in range(4):
            s.set_basis(0)
            p.execute(s)
            got = s.download()
            compare_circuit(got, ref, "c128", f"replay {rep}")
            s.apply_1q(0, np.eye(2) * 1j)  # eager work between replays
            s.sync()


# ----------------------------------------------------------------------------------------------
# LDS-staged plans: several gates per read/write of the state
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("lds", [0, 10, 11])
def test_staged_brickwork(q, oracle_mod, dtype, lds):
    if dtype == "c64" and lds == 10:
        pytest.skip("complex64 blocks hold at least 2^11 amplitudes")
    text = wl.brickwork_circuit(15, 8, seed=23)
    ref = oracle_mod.run_circuit(text)
    c = q.parse_circuit(text)
    s = q.State(c.n, dtype)
    p = q.Plan(c, dtype, method="staged", lds_qubits=lds)
    assert p.info["passes"] < len(c.gates) // 4
    p.execute(s)
    compare_circuit(s.download().astype(np.complex128), ref, dtype, f"staged lds={lds}")


# every kernel variant (resident qubits m, 2^le amplitudes per thread): up to 2^10 threads per
# workgroup, so the stage records carry up to 10 thread bits
STAGED_VARIANTS = [("c128", m, le) for m, le in ((10, 3), (11, 3), (12, 3), (10, 4), (11, 4), (12, 4), (13, 4))] + \
                  [("c64", m, le) for m, le in ((11, 4), (12, 4), (13, 4), (14, 4), (11, 5), (12, 5), (13, 5), (14, 5))]


@pytest.mark.parametrize("dtype,m,le", STAGED_VARIANTS)
def test_staged_every_variant(q, oracle_mod, dtype, m, le):
    """Each block shape on two circuit families; each run twice: on a state set to |0...0>, and from
    zero on a state holding other values (the first pass then generates |0...0> in its loads)."""
    n = 16
    junk = wl.gaussian_state(n, 77)
    for text in (wl.brickwork_circuit(n, 6, seed=29), wl.config0_circuit(n, 80, seed=5)):
        ref = oracle_mod.run_circuit(text)
        c = q.parse_circuit(text)
        s = q.State(c.n, dtype)
        p = q.Plan(c, dtype, method="staged", lds_qubits=m, lds_regs=le)
        assert p.info["lds_qubits"] == m and p.info["lds_regs"] == le
        kind, var = p.launches()
        print(f"staged m={m} le={le}: forms {''.join('FHW'[v] for v in var)}", flush=True)
        p.execute(s)
        compare_circuit(s.download().astype(np.complex128), ref, dtype, f"staged m={m} le={le}")
        s.upload(junk)
        p.execute_from_zero(s)
        compare_circuit(s.download().astype(np.complex128), ref, dtype, f"staged m={m} le={le} from zero")
        p.close()
        s.close()


# renormalisation points: before the first layer (no pass before it), in the middle, twice in a row,
# and at the end (no pass after it)
RENORM_AFTER = (0, 2, 4, 4, 6)
RENORM_PLANS = [("c128", "plain", 0, 0), ("c128", "fused", 0, 0), ("c128", "staged", 12, 4), ("c128", "staged", 11, 3),
                ("c64", "plain", 0, 0), ("c64", "staged", 13, 5), ("c64", "staged", 12, 4)]


@pytest.mark.parametrize("dtype,method,m,le", RENORM_PLANS)
def test_plan_renormalisation_points(q, oracle_mod, dtype, method, m, le):
    """RENORM inside plans (Eq. STAT1) against the oracle, which renormalises at the same points: the
    final state, and the squared norm found at every point, from an unnormalised start state; again
    from |0...0>, and (staged) timed and through a replayed graph. A staged plan folds the norm into
    the pass before a point and the factor into the pass after it, so only the points with no pass on
    one side run sweeps: the norm of the first point, a factor and a norm around the repeated point,
    and the factor of the last."""
    n, layers, seed = 16, 6, 31
    text = wl.brickwork_circuit(n, layers, seed, renorm_after=RENORM_AFTER)
    c = q.parse_circuit(text)
    psi0 = 2.5 * wl.gaussian_state(n, 8)
    ref = oracle_mod.run_circuit(text, psi0=psi0)
    ops = [ln.split()[0] for ln in text.splitlines() if ln.strip() and not ln.startswith(("!", "#", "QUBITS"))]
    at = [i for i, kw in enumerate(ops) if kw == "RENORM"]
    want_norms = np.array([oracle_mod.norm(oracle_mod.run_circuit(text, psi0=psi0, ops_limit=k)) for k in at])
    rtol = 1e-12 if dtype == "c128" else 1e-5
    opts = dict(method=method, lds_qubits=m, lds_regs=le)
    p = q.Plan(c, dtype, **opts)
    assert p.info["renorms"] == len(RENORM_AFTER)
    kind, var = p.launches()
    sweeps = int(np.sum(kind == q.KERNEL_RENORM))
    assert sweeps == (4 if method == "staged" else len(RENORM_AFTER)), (method, list(kind))
    print(f"renorm {dtype} {method} m={m} le={le}: {len(kind)} launches, {sweeps} sweeps", flush=True)
    s = gpu_state(q, psi0, dtype)
    p.execute(s)
    compare_circuit(s.download().astype(np.complex128), ref, dtype, f"{method} renorm")
    np.testing.assert_allclose(p.norms(), want_norms, rtol=rtol)
    # from |0...0>: the first point's norm is 1
    ref0 = oracle_mod.run_circuit(text)
    want0 = np.array([oracle_mod.norm(oracle_mod.run_circuit(text, ops_limit=k)) for k in at])
    s.upload(psi0)
    p.execute_from_zero(s)
    compare_circuit(s.download().astype(np.complex128), ref0, dtype, f"{method} renorm from zero")
    np.testing.assert_allclose(p.norms(), want0, rtol=rtol)
    s.upload(psi0)
    ms, kd, fk = p.execute_timed(s)
    assert len(ms) == p.info["launches"] and np.array_equal(kd, kind)
    compare_circuit(s.download().astype(np.complex128), ref, dtype, f"{method} renorm timed")
    p.close()
    s.close()
    if method == "staged":
        import torch
        with torch.cuda.stream(torch.cuda.Stream()):
            g = q.Plan(c, dtype, use_graph=True, **opts)
            s2 = q.State(n, dtype)
            for rep in range(3):  # capture, then replays, with eager work and synchronisation between
                s2.upload(psi0)
                g.execute(s2)
                compare_circuit(s2.download().astype(np.complex128), ref, dtype, f"staged renorm graph run {rep}")
                np.testing.assert_allclose(g.norms(), want_norms, rtol=rtol)
            g.close()
            s2.close()


@pytest.mark.parametrize("dtype,method", [("c128", "plain"), ("c128", "staged"), ("c64", "staged")])
def test_renorm_only_plan(q, oracle_mod, dtype, method):
    """A plan of two renormalisation points and no gate: its norms read 0 before the first execution;
    on an unnormalised state it runs a norm sweep and a scaling sweep per point and leaves the
    normalised state; the points report the state's squared norm, then 1."""
    n = 13
    text = wl.circuit_text(n, ["RENORM", "RENORM"])
    psi0 = 3.0 * wl.gaussian_state(n, 4)
    ref = oracle_mod.run_circuit(text, psi0=psi0)
    p = q.Plan(q.parse_circuit(text), dtype, method=method)
    assert np.array_equal(p.norms(), np.zeros(2))
    s = gpu_state(q, psi0, dtype)
    p.execute(s)
    compare_circuit(s.download().astype(np.complex128), ref, dtype, f"{method} renorm only")
    rtol = 1e-12 if dtype == "c128" else 1e-5
    np.testing.assert_allclose(p.norms(), [oracle_mod.norm(psi0), 1.0], rtol=rtol)
    p.execute_from_zero(s)  # |0...0> first, then the points
    np.testing.assert_allclose(p.norms(), [1.0, 1.0], rtol=rtol)
    p.close()
    s.close()


def test_renorm_point_rejected_outside_plans(q):
    c = q.parse_circuit(wl.circuit_text(4, ["H 0", "RENORM"]))
    with pytest.raises(q.QsimError):
        q.Batch([c], "c128")


@pytest.mark.parametrize("method", ["plain", "fused"])
def test_execute_from_zero_unstaged(q, oracle_mod, method):
    n = 12
    text = wl.config0_circuit(n, 60, seed=2)
    ref = oracle_mod.run_circuit(text)
    s = q.State(n, "c128")
    s.upload(wl.gaussian_state(n, 5))
    p = q.Plan(q.parse_circuit(text), "c128", method=method)
    p.execute_from_zero(s)
    compare_circuit(s.download(), ref, "c128", f"{method} from zero")
    ms, kind, fk = p.execute_timed(s, from_zero=True)
    assert len(ms) == p.info["launches"]
    compare_circuit(s.download(), ref, "c128", f"{method} timed from zero")


@pytest.mark.parametrize("n,dtype,m,le,most", [(33, "c128", 12, 4, 14), (33, "c128", 11, 4, 19), (33, "c128", 10, 4, 24),
                                                 (34, "c64", 12, 4, 17)])
def test_staged_pass_count_full_size(q, n, dtype, m, le, most):
    """The scheduler's resident-set choice on the full-size brickwork (the plan alone: no state is
    allocated). Each pass can run a light cone of several layers over a window of neighbouring
    qubits; the pass count bounds the HBM traffic of the plan."""
    c = q.parse_circuit(wl.brickwork_circuit(n, 20, seed=21 if dtype == "c128" else 31))
    p = q.Plan(c, dtype, method="staged", lds_qubits=m, lds_regs=le)
    print(f"brickwork {n} {dtype} m={m}: {p.info['passes']} passes", flush=True)
    assert p.info["passes"] <= most
    p.close()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("seed", [1, 2])
def test_staged_config0(q, oracle_mod, dtype, seed):
    """Random gates from the nine-name set: controls and diagonal gates inside and outside the
    resident set, Pauli Y (general), CNOT with non-resident targets."""
    text = wl.config0_circuit(16, 200, seed)
    ref = oracle_mod.run_circuit(text)
    got, p = run_gpu(q, text, dtype, "staged")
    compare_circuit(got, ref, dtype, f"staged seed {seed}")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [13, 17])
def test_staged_qft_with_swaps(q, oracle_mod, dtype, n):
    psi = wl.gaussian_state(n, 12)
    text = wl.qft_circuit(n)
    ref = oracle_mod.run_circuit(text, psi0=psi)
    got, p = run_gpu(q, text, dtype, "staged", psi0=psi)
    compare_circuit(got, ref, dtype, f"staged qft n={n}")
    assert p.info["passes"] <= 8


def test_staged_adder_bit_exact(q):
    m = 7
    text, lay = wl.ripple_adder_circuit(m)
    c = q.parse_circuit(text)
    p = q.Plan(c, "c128", method="staged", lds_qubits=10)
    s = q.State(lay["n"], "c128")
    for a, b in wl.adder_operands(m, 16, seed=11):
        s.set_basis(a | (b << m))
        p.execute(s)
        got = s.download()
        want = a | (((a + b) % 2 ** m) << m)
        assert got[want] == 1.0 and np.count_nonzero(got) == 1, (a, b)


def test_staged_controlled_everything(q, oracle_mod):
    """Controlled general gates, Toffolis and controlled swaps with controls on every kind of bit."""
    n = 14
    rng = np.random.default_rng(99)
    lines = []
    for _ in range(120):
        kind = rng.integers(0, 5)
        qs = [int(x) for x in rng.permutation(n)[:3]]
        if kind == 0:
            lines.append(f"CV {qs[0]} {qs[1]} {float(rng.uniform(0, 6)).hex()}")
        elif kind == 1:
            lines.append(f"TOFFOLI {qs[0]} {qs[1]} {qs[2]}")
        elif kind == 2:
            lines.append(f"QSWAP {qs[0]} {qs[1]}")
        elif kind == 3:
            lines.append(wl.u_line(qs[0], wl.haar_2x2(rng)))
        else:
            lines.append(f"CRK {qs[0]} {qs[1]} {int(rng.integers(1, 9))}")
    text = wl.circuit_text(n, lines)
    psi = wl.gaussian_state(n, 5)
    ref = oracle_mod.run_circuit(text, psi0=psi)
    for lds in (10, 12):
        c = q.parse_circuit(text)
        s = q.State(n, "c128")
        s.upload(psi)
        q.Plan(c, "c128", method="staged", lds_qubits=lds).execute(s)
        compare_circuit(s.download(), ref, "c128", f"lds={lds}")


# ----------------------------------------------------------------------------------------------
# Batches of independent circuits in one persistent launch
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_against_oracle(q, oracle_mod, dtype):
    texts = wl.batch_circuits(count=24, nmin=3, nmax=15, depth=50, seed=41)
    texts.append(wl.circuit_text(5, []))                       # no gates at all
    texts.append(wl.config0_circuit(13, 80, seed=9))            # H prefix, above one block
    b = q.Batch(texts, dtype)
    st = b.run()
    assert st["circuits"] == len(texts)
    for rep in range(2):  # the second run starts again from |0...0>
        if rep:
            b.run()
        for c, text in enumerate(texts):
            ref = oracle_mod.run_circuit(text)
            got = b.download(c).astype(np.complex128)
            compare_circuit(got, ref, dtype, f"circuit {c} rep {rep}")
    lat = b.latencies_us()
    assert np.all(lat > 0) and np.all(np.isfinite(lat))


def test_batch_graph_replay(q, oracle_mod):
    import torch
    texts = wl.batch_circuits(count=16, nmin=10, nmax=14, depth=30, seed=5)
    refs = [oracle_mod.run_circuit(t) for t in texts]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b = q.Batch(texts, "c128", use_graph=True)
        for rep in range(3):
            b.run()
            for c in range(len(texts)):
                compare_circuit(b.download(c), refs[c], "c128", f"replay {rep} circuit {c}")


@pytest.mark.parametrize("dtype,variant", [("c128", (11, 3)), ("c128", (11, 4)), ("c128", (12, 4)), ("c64", (11, 4)),
                                           ("c64", (12, 4)), ("c64", (13, 5))])
def test_batch_variants(q, oracle_mod, dtype, variant):
    """Every block shape a batch can use, on circuits from below one block to 2^5 blocks: the larger
    ones are split over workgroups (pass p of each in launch step p, in the wave-split, half-buffer or
    full-buffer kernel that the pass allows), the smaller ones run whole."""
    texts = wl.batch_circuits(count=10, nmin=9, nmax=13, depth=40, seed=77)
    texts += wl.batch_circuits(count=6, nmin=variant[0] + 3, nmax=variant[0] + 5, depth=60, seed=78)
    b = q.Batch(texts, dtype, lds_qubits=variant[0], lds_regs=variant[1])
    assert b.info["split_circuits"] >= 6 and b.info["lds_qubits"] == variant[0]
    for rep in range(2):
        b.run()
        for c, t in enumerate(texts):
            compare_circuit(b.download(c).astype(np.complex128), oracle_mod.run_circuit(t), dtype, f"{variant} circuit {c} rep {rep}")
    lat = b.latencies_us()
    assert np.all(lat > 0) and np.all(np.isfinite(lat))
    b.close()


def test_batch_tuned_shape_matches_oracle(q, oracle_mod):
    """The batch autotuner builds and times every block shape; the batch built with its choice runs
    through a HIP graph on a stream of its own and reproduces the oracle on every circuit."""
    import torch
    from paper_quant_ph_0608239_amd import tuning
    texts = wl.batch_circuits(count=48, nmin=10, nmax=18, depth=50, seed=43)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        t = tuning.tune_batch(texts, "c128", reps=1)
        print(f"batch tune: m={t['lds_qubits']} r={t['lds_regs']} {t['ms']:.3f} ms; tried {t['tried']}", flush=True)
        assert len(t["tried"]) == 3 and t["ms"] == min(x["ms"] for x in t["tried"])
        b = q.Batch(texts, "c128", lds_qubits=t["lds_qubits"], lds_regs=t["lds_regs"], use_graph=True)
        for rep in range(2):
            b.run()
            for c, text in enumerate(texts):
                compare_circuit(b.download(c), oracle_mod.run_circuit(text), "c128", f"tuned circuit {c} rep {rep}")
        b.close()


# ----------------------------------------------------------------------------------------------
# The autotuner's choice, and the library-owned allocation
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,n", [("c128", 20), ("c64", 21)])
def test_tuned_plan_matches_oracle(q, oracle_mod, dtype, n, tmp_path, monkeypatch):
    """qsim_plan_tune times every candidate (plain, fused k = 2..5, the staged block shapes) on a
    scratch state; the plan it picks, built again from the returned options, reproduces the oracle,
    and the JSON cache returns the same choice on a second call."""
    from paper_quant_ph_0608239_amd import tuning
    monkeypatch.setenv("QSIM_TUNE_CACHE", str(tmp_path / "tune.json"))
    text = wl.brickwork_circuit(n, 8, seed=21)
    c = q.parse_circuit(text)
    s = q.State(n, dtype)
    t = tuning.tune(c, s, reps=1, include_plain=True, use_cache=True)
    ran = [x for x in t["tried"] if x["ms"] > 0]
    print(f"tune {dtype} n={n}: {t['method']} k={t['fuse_k']} m={t['lds_qubits']} r={t['lds_regs']} "
          f"{t['ms']:.3f} ms; {len(ran)} of {len(t['tried'])} candidates timed", flush=True)
    assert t["ms"] > 0 and len(ran) >= 1 and t["method"] in ("plain", "fused", "staged")
    assert t["ms"] <= min(x["ms"] for x in ran) + 1e-9
    again = tuning.tune(c, s, reps=1, include_plain=True, use_cache=True)
    assert again["cached"] and {k: again[k] for k in ("method", "fuse_k", "lds_qubits", "lds_regs")} == \
        {k: t[k] for k in ("method", "fuse_k", "lds_qubits", "lds_regs")}
    p = q.Plan(c, dtype, method=t["method"], fuse_k=t["fuse_k"] or 5, lds_qubits=t["lds_qubits"], lds_regs=t["lds_regs"])
    s.set_basis(0)
    p.execute(s)
    got = s.download().astype(np.complex128)
    ref = oracle_mod.run_circuit(text)
    if dtype == "c128":
        assert np.max(np.abs(got - ref)) <= TOL128
    else:
        assert oracle_mod.infidelity(got, ref) <= TOL64_FID
    p.close()
    s.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_library_owned_state(q, oracle_mod, dtype):
    """qsim_alloc: the library allocates the state and sets it to |0...0>; gates and reductions run on
    it like on a wrapped buffer; qsim_free releases it. A state larger than the free device memory is
    refused with ENOMEM before anything is allocated."""
    import ctypes
    from paper_quant_ph_0608239_amd import _lib
    L = q.lib()
    n = 14
    code = q.dtype_code(dtype)
    h = ctypes.c_void_p()
    assert L.qsim_alloc(n, code, None, ctypes.byref(h)) == _lib.OK
    try:
        assert L.qsim_num_qubits(h) == n and L.qsim_get_dtype(h) == code and L.qsim_data(h)
        cd = np.complex128 if dtype == "c128" else np.complex64
        out = np.empty(2 ** n, dtype=cd)
        assert L.qsim_download(h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes) == _lib.OK
        assert out[0] == 1 and np.count_nonzero(out) == 1
        H = np.array([[1, 1], [1, -1]]) / np.sqrt(2)
        flat = (ctypes.c_double * 8)(*np.asarray(H, np.complex128).reshape(-1).view(np.float64).tolist())
        for t in range(n):
            assert L.qsim_apply_1q(h, t, flat) == _lib.OK
        nrm = ctypes.c_double()
        assert L.qsim_norm(h, ctypes.byref(nrm)) == _lib.OK
        assert abs(nrm.value - 1.0) <= (1e-13 if dtype == "c128" else 1e-6)
        assert L.qsim_download(h, out.ctypes.data_as(ctypes.c_void_p), out.nbytes) == _lib.OK
        ref = oracle_mod.run_circuit(wl.circuit_text(n, [f"H {t}" for t in range(n)]))
        check(out, ref, dtype, "H on every qubit of an owned state")
    finally:
        assert L.qsim_free(h) == _lib.OK
    big = ctypes.c_void_p()
    assert L.qsim_alloc(40, code, None, ctypes.byref(big)) == _lib.ENOMEM
    assert not big.value
