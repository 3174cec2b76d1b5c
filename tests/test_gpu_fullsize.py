"""GPU parity at the full sizes of the benchmark workloads, in the plan configurations the benchmark
times (the fused k = 5 plan, the LDS-staged plans the tuner chooses from, the plain per-gate plan).

Where the oracle cannot hold or sweep the whole state in seconds, the GPU result is checked on
outputs the oracle computes one at a time (sampled Fourier coefficients) or through properties that
hold at any size: exact basis-state outputs of permutation circuits, preservation of the norm
(Eq. STAT1), and exact uncomputation (a circuit followed by its inverse returns |0...0>).

Bars: permutations bit-exact; complex128 within 1e-12 in max|d amp|; complex64 within 1 - F <= 1e-6
of the FP64 oracle, with the norm drift bounded as stated per test.
"""
import gc
import math

import numpy as np
import pytest

import qsim_workloads as wl

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64_FID = 1e-6


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def q():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_quant_ph_0608239_amd as q
    q.lib()
    yield q
    release()


def release():
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def amp(s, i):
    """One amplitude of a device state, read through the tensor that owns the memory."""
    v = s.tensor[2 * i:2 * i + 2].cpu().numpy().astype(np.float64)
    return complex(v[0], v[1])


def inverse_text(text):
    return wl.circuit_text(int(text.split("QUBITS")[1].split()[0]), wl.inverse_lines(text))


PLANS_BIG = [("staged", 0, 0), ("staged", 12, 3), ("fused", 0, 0)]


def plan_for(q, circ, dtype, method, lds=0, regs=0):
    return q.Plan(circ, dtype, method=method, fuse_k=5, lds_qubits=lds, lds_regs=regs)


# ----------------------------------------------------------------------------------------------
# Ripple-carry adder of two 14-bit registers plus a carry qubit (29 qubits), 64 seeded operands
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("method,count", [("auto", 64), ("staged", 8), ("fused", 8), ("plain", 4)])
def test_adder_29q_bit_exact(q, method, count):
    import torch
    m = 14
    text, lay = wl.ripple_adder_circuit(m)
    assert lay["n"] == 29
    c = q.parse_circuit(text)
    s = q.State(lay["n"], "c128")
    p = q.Plan(c, "c128", method=method)
    try:
        for idx, (a, b) in enumerate(wl.adder_operands(m, 64, seed=11)[:count]):
            say(f"adder29 {method} case {idx}: a={a} b={b}")
            s.set_basis(a | (b << m))
            p.execute(s)
            want = a | (((a + b) % 2 ** m) << m)
            assert amp(s, want) == 1.0 + 0.0j, (a, b)
            assert int(torch.count_nonzero(s.tensor)) == 1, (a, b)
    finally:
        p.close()
        s.close()
        del s
        release()


# ----------------------------------------------------------------------------------------------
# 28-qubit QFT on a seeded complex-Gaussian normalised state
# ----------------------------------------------------------------------------------------------
QFT_N = 28


@pytest.fixture(scope="module")
def qft28(oracle_mod):
    psi = wl.gaussian_state(QFT_N, 12)
    say("qft28: FP64 oracle on the whole 28-qubit QFT (420 gates)")
    ref = oracle_mod.run_circuit(wl.qft_circuit(QFT_N), psi0=psi)
    N = 2 ** QFT_N
    rng = np.random.default_rng(2828)
    ks = [0, 1, 2, 3, N // 2, N - 1] + [int(k) for k in rng.integers(0, N, size=4)]
    # the Fourier sum of Sec. V evaluated one output at a time, independently of the gate sequence
    sampled = oracle_mod.qft_sample(psi, ks)
    assert np.max(np.abs(ref[ks] - sampled)) <= TOL128
    return psi, ref


@pytest.mark.parametrize("method", ["auto", "fused", "plain"])
def test_qft_28q_full_state_vs_oracle_and_round_trip(q, qft28, method):
    psi, ref = qft28
    text = wl.qft_circuit(QFT_N)
    c = q.parse_circuit(text)
    ci = q.parse_circuit(wl.circuit_text(QFT_N, wl.iqft_lines(list(range(QFT_N)))))
    s = q.State(QFT_N, "c128")
    p = q.Plan(c, "c128", method=method)
    pi = q.Plan(ci, "c128", method=method)
    try:
        say(f"qft28 {method}: forward ({p.info['launches']} launches)")
        s.upload(psi)
        p.execute(s)
        got = s.download()
        d = float(np.max(np.abs(got - ref)))
        say(f"qft28 {method}: max|d amp| over all 2^28 outputs = {d:.3e}")
        assert d <= TOL128
        del got
        assert abs(s.norm() - 1.0) <= 1e-12
        say(f"qft28 {method}: inverse")
        pi.execute(s)
        back = s.download()
        d = np.max(np.abs(back - psi))
        say(f"qft28 {method}: round trip max|d| = {d:.3e}")
        assert d <= TOL128
    finally:
        p.close()
        pi.close()
        s.close()
        del s
        release()


# ----------------------------------------------------------------------------------------------
# 28-qubit complex128 brickwork, element by element against the oracle, in the plan shapes the
# benchmark tunes over; each staged plan's launches are checked for the kernel form they run
# ----------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def brick28_c128_ref(oracle_mod):
    say("brick28 c128: FP64 oracle on the 28-qubit brickwork (20 layers, seed 21)")
    return oracle_mod.run_circuit(wl.brickwork_circuit(28, 20, seed=21))


@pytest.mark.parametrize("method,lds,regs", [("staged", 12, 4), ("staged", 11, 4), ("staged", 10, 4), ("fused", 0, 0)])
def test_brickwork_c128_28q_vs_oracle(q, brick28_c128_ref, method, lds, regs):
    n = 28
    c = q.parse_circuit(wl.brickwork_circuit(n, 20, seed=21))
    s = q.State(n, "c128")
    p = plan_for(q, c, "c128", method, lds, regs)
    try:
        kind, var = p.launches()
        if method == "staged":
            assert (kind == q.KERNEL_STAGED).all()
            forms = "".join("FHW"[v] for v in var)
            say(f"brick28 c128 staged m{lds}r{regs}: {len(var)} passes, forms {forms} (F full, H half, W wave-split)")
            if lds == 12:
                assert (var == q.STAGED_WAVE).all()  # every pass of this schedule splits at wave positions
            elif lds == 11:
                assert (var == q.STAGED_WAVE).sum() >= 10 and (var == q.STAGED_HALF).sum() >= 1
            else:
                assert (var == q.STAGED_HALF).all()  # no wave-split kernel at 64 threads per block
        else:
            assert (var[kind == q.KERNEL_FUSED_MFMA] == 5).sum() >= 1
            say(f"brick28 c128 fused: {len(kind)} launches, {(kind == q.KERNEL_FUSED_MFMA).sum()} on the matrix cores")
        s.set_basis(0)
        p.execute(s)
        got = s.download()
        d = float(np.max(np.abs(got - brick28_c128_ref)))
        say(f"brick28 c128 {method} m{lds}r{regs}: max|d amp| = {d:.3e}")
        assert d <= TOL128
    finally:
        p.close()
        s.close()
        del s
        release()


# ----------------------------------------------------------------------------------------------
# 33-qubit complex128 brickwork (128 GiB): norm and exact uncomputation
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("method,lds,regs", PLANS_BIG)
def test_brickwork_33q_uncompute(q, method, lds, regs):
    n = 33
    text = wl.brickwork_circuit(n, 20, seed=21)
    c = q.parse_circuit(text)
    ci = q.parse_circuit(inverse_text(text))
    s = q.State(n, "c128")
    p = plan_for(q, c, "c128", method, lds, regs)
    pi = plan_for(q, ci, "c128", method, lds, regs)
    try:
        say(f"brick33 {method} lds={lds} regs={regs}: forward {p.info['gates']} gates")
        s.set_basis(0)
        p.execute(s)
        nrm = s.norm()
        say(f"brick33 {method}: |norm-1| = {abs(nrm - 1):.3e}")
        assert abs(nrm - 1.0) <= 1e-12
        assert abs(amp(s, 0)) < 1e-3  # the circuit has spread the state
        say(f"brick33 {method}: inverse")
        pi.execute(s)
        a0 = amp(s, 0)
        say(f"brick33 {method}: |a0 - 1| = {abs(a0 - 1):.3e}")
        assert abs(a0 - 1.0) <= TOL128
        assert abs(s.norm() - 1.0) <= 1e-12
    finally:
        p.close()
        pi.close()
        s.close()
        del s
        release()


def test_brickwork_33q_plain_two_layers_uncompute(q):
    """The unfused per-gate sweep at 33 qubits (two layers forward, then inverse)."""
    n = 33
    text = wl.brickwork_circuit(n, 20, seed=21, layer_range=(0, 2))
    c = q.parse_circuit(text)
    ci = q.parse_circuit(inverse_text(text))
    s = q.State(n, "c128")
    p = q.Plan(c, "c128", method="plain")
    pi = q.Plan(ci, "c128", method="plain")
    try:
        say("brick33 plain 2 layers: forward + inverse")
        s.set_basis(0)
        p.execute(s)
        pi.execute(s)
        assert abs(amp(s, 0) - 1.0) <= TOL128
        assert abs(s.norm() - 1.0) <= 1e-12
    finally:
        p.close()
        pi.close()
        s.close()
        del s
        release()


def test_brickwork_33q_staged_equals_fused_on_samples(q):
    """The two fast plans agree amplitude by amplitude on 64 sampled indices (both are FP64; the
    difference is rounding order only)."""
    n = 33
    text = wl.brickwork_circuit(n, 20, seed=21)
    c = q.parse_circuit(text)
    idx = [0, 2 ** n - 1] + [int(i) for i in np.random.default_rng(33).integers(0, 2 ** n, size=62)]
    s = q.State(n, "c128")
    vals = {}
    try:
        for method in ("staged", "fused"):
            p = q.Plan(c, "c128", method=method, fuse_k=5)
            say(f"brick33 samples: {method}")
            s.set_basis(0)
            p.execute(s)
            vals[method] = np.array([amp(s, i) for i in idx])
            p.close()
        d = np.max(np.abs(vals["staged"] - vals["fused"]))
        say(f"brick33 staged vs fused on 64 samples: max|d| = {d:.3e}")
        assert d <= TOL128
    finally:
        s.close()
        del s
        release()


# ----------------------------------------------------------------------------------------------
# Complex64 brickwork with FP64 renormalisation after every 10 layers
# ----------------------------------------------------------------------------------------------
C64_SEED = 31  # the complex64 brickwork uses its own seed


def run_renormalised(q, s, n, layers, method, every=10, lds=0, regs=0):
    """The brickwork as one plan with a RENORM point after every `every` layers (a staged plan folds
    each point into the passes around it), run from |0...0>. Returns the squared norms found at the
    points, each just before its rescaling."""
    points = tuple(range(every, layers + 1, every))
    c = q.parse_circuit(wl.brickwork_circuit(n, layers, seed=C64_SEED, renorm_after=points))
    p = plan_for(q, c, "c64", method, lds, regs)
    p.execute_from_zero(s)
    norms = [float(x) for x in p.norms()]
    kind, _ = p.launches()
    p.close()
    say(f"  {method}: {len(kind)} launches, {int(np.sum(kind == q.KERNEL_RENORM))} renormalisation sweeps; "
        f"squared norms at the points = {norms}")
    return norms


@pytest.fixture(scope="module")
def brick28_ref(oracle_mod):
    say("brick28: FP64 oracle on the 28-qubit brickwork (20 layers, renormalised after layers 10 and 20)")
    return oracle_mod.run_circuit(wl.brickwork_circuit(28, 20, seed=C64_SEED, renorm_after=(10, 20)))


@pytest.mark.parametrize("method", ["fused", "staged"])
def test_brickwork_c64_28q_renormalised_vs_oracle(q, oracle_mod, brick28_ref, method):
    n = 28
    s = q.State(n, "c64")
    try:
        say(f"brick28 c64 {method}")
        norms = run_renormalised(q, s, n, 20, method)
        got = s.download().astype(np.complex128)
        f = oracle_mod.infidelity(got, brick28_ref)
        d = np.max(np.abs(got - brick28_ref))
        say(f"brick28 c64 {method}: 1-F = {f:.3e}, max|d amp| = {d:.3e}, norms = {norms}")
        assert f <= TOL64_FID
        assert all(abs(x - 1.0) <= 1e-4 for x in norms)
        assert abs(s.norm() - 1.0) <= 1e-6
    finally:
        s.close()
        del s
        release()


@pytest.mark.parametrize("method", ["fused", "staged"])
def test_brickwork_c64_34q_norm_drift_and_uncompute(q, method):
    """34 qubits complex64 (128 GiB): the norm drift before each FP64 renormalisation is small, and
    running the inverse circuit afterwards returns |0...0> to FP32 accuracy."""
    n = 34
    s = q.State(n, "c64")
    try:
        say(f"brick34 c64 {method}")
        norms = run_renormalised(q, s, n, 20, method)
        assert all(abs(x - 1.0) <= 1e-4 for x in norms), norms
        assert abs(s.norm() - 1.0) <= 1e-6
        ci = q.parse_circuit(inverse_text(wl.brickwork_circuit(n, 20, seed=C64_SEED)))
        pi = plan_for(q, ci, "c64", method)
        pi.execute(s)
        pi.close()
        a0 = amp(s, 0)
        fid = abs(a0) ** 2 / s.norm()
        say(f"brick34 c64 {method}: 1 - |a0|^2/norm after uncompute = {1 - fid:.3e}")
        assert 1.0 - fid <= TOL64_FID
    finally:
        s.close()
        del s
        release()


# ----------------------------------------------------------------------------------------------
# 2048 independent circuits (n uniform in [10, 22], depth 50) in one persistent launch
# ----------------------------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_2048_sampled_circuits_vs_oracle(q, oracle_mod, dtype):
    texts = wl.batch_circuits(count=2048, nmin=10, nmax=22, depth=50, seed=41)
    ns = np.array([int(t.split("QUBITS")[1].split()[0]) for t in texts])
    rng = np.random.default_rng(2048)
    pick = sorted(set([int(np.argmax(ns)), int(np.argmin(ns)), 0, 2047] +
                      [int(i) for i in rng.integers(0, 2048, size=12)]))
    b = q.Batch(texts, dtype, use_graph=False)
    try:
        for rep in range(2):
            say(f"batch2048 {dtype}: launch {rep}")
            b.run()
            for i in pick:
                got = b.download(i).astype(np.complex128)
                ref = oracle_mod.run_circuit(texts[i])
                if dtype == "c128":
                    d = np.max(np.abs(got - ref))
                    assert d <= TOL128, (i, ns[i], d)
                else:
                    f = oracle_mod.infidelity(got, ref)
                    assert f <= TOL64_FID, (i, ns[i], f)
    finally:
        b.close()
        del b
        release()


@pytest.mark.timeout(1200)
def test_batch_2048_every_circuit_vs_oracle(q, oracle_mod):
    """Every one of the 2048 circuits, in both precisions, against the oracle run on that circuit."""
    texts = wl.batch_circuits(count=2048, nmin=10, nmax=22, depth=50, seed=41)
    b64 = q.Batch(texts, "c64", use_graph=False)
    b128 = q.Batch(texts, "c128", use_graph=False)
    try:
        say("batch2048 every circuit: launching both precisions")
        b64.run()
        b128.run()
        worst128 = worst64 = 0.0
        for i, t in enumerate(texts):
            ref = oracle_mod.run_circuit(t)
            d = float(np.max(np.abs(b128.download(i).astype(np.complex128) - ref)))
            f = float(oracle_mod.infidelity(b64.download(i).astype(np.complex128), ref))
            worst128, worst64 = max(worst128, d), max(worst64, f)
            assert d <= TOL128, (i, d)
            assert f <= TOL64_FID, (i, f)
            if i % 256 == 255:
                say(f"  {i + 1} circuits checked: worst max|d| (c128) = {worst128:.3e}, worst 1-F (c64) = {worst64:.3e}")
    finally:
        b64.close()
        b128.close()
        del b64, b128
        release()
