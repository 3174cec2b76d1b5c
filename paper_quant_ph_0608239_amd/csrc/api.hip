// C ABI of libqsim: state management, argument validation, gate classification and dispatch to
// the sweep / fused / reduction kernels. Nothing is launched when an argument is rejected.
#include <cmath>
#include <cstring>

#include "qsim_internal.h"

namespace qsim {

static thread_local std::string g_err;

int set_error(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

int hip_error(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? QSIM_ENOMEM : QSIM_EDEVICE;
}

static int check_state(const qsim_state *s)
{
    if (!s || !s->data) return set_error(QSIM_EINVAL, "null state");
    return QSIM_OK;
}

static int check_qubit(const qsim_state *s, int q, const char *what)
{
    if (q < 0 || q >= s->n) return set_error(QSIM_EINVAL, std::string(what) + " out of range");
    return QSIM_OK;
}

static int check_mask(const qsim_state *s, uint64_t mask)
{
    if (s->n < 64 && (mask >> s->n) != 0) return set_error(QSIM_EINVAL, "control mask has bits >= n");
    return QSIM_OK;
}

Kind classify(const double u[8])
{
    const bool off0 = u[2] == 0.0 && u[3] == 0.0 && u[4] == 0.0 && u[5] == 0.0;
    const bool diag0 = u[0] == 0.0 && u[1] == 0.0 && u[6] == 0.0 && u[7] == 0.0;
    if (off0) {
        if (u[0] == 1.0 && u[1] == 0.0) return Kind::Phase1;
        return Kind::Diag;
    }
    if (diag0 && u[2] == 1.0 && u[3] == 0.0 && u[4] == 1.0 && u[5] == 0.0) return Kind::Swap;
    return Kind::General;
}

static int apply_matrix(qsim_state *s, uint64_t cmask, int target, const double u[8])
{
    const uint64_t tbit = uint64_t(1) << target;
    switch (classify(u)) {
    case Kind::Swap: return launch_swap(s, make_index_map(cmask | tbit, cmask), tbit);
    case Kind::Phase1: {
        if (u[6] == 1.0 && u[7] == 0.0) return QSIM_OK;  // identity
        const double c[2] = {u[6], u[7]};
        return launch_phase(s, make_index_map(cmask | tbit, cmask | tbit), c, DiagMode::Values);
    }
    case Kind::Diag: {
        const double d[4] = {u[0], u[1], u[6], u[7]};
        return launch_diag(s, make_index_map(cmask, cmask), target, d, DiagMode::Values);
    }
    default: {
        Mat2 m;
        memcpy(m.m, u, sizeof(m.m));
        return launch_general(s, make_index_map(cmask | tbit, cmask), target, m);
    }
    }
}

double phase_angle(const qsim_gate &g)
{
    if (g.op == QSIM_OP_RK) return std::ldexp(kTwoPi, -g.target2);
    if (g.op == QSIM_OP_RKDG) return -std::ldexp(kTwoPi, -g.target2);
    return g.theta;
}

// FP64 matrices of the named gates (host); the per-gate path and the staged passes evaluate angle
// gates on the device instead
int gate_matrix(const qsim_gate &g, double u[8])
{
    const double h = 1.0 / std::sqrt(2.0);
    auto setm = [&](double a, double b, double c, double d, double e, double f, double gg, double hh) {
        u[0] = a; u[1] = b; u[2] = c; u[3] = d; u[4] = e; u[5] = f; u[6] = gg; u[7] = hh;
    };
    switch (g.op) {
    case QSIM_OP_MATRIX: memcpy(u, g.u, 8 * sizeof(double)); break;
    case QSIM_OP_H: setm(h, 0, h, 0, h, 0, -h, 0); break;
    case QSIM_OP_X: setm(0, 0, 1, 0, 1, 0, 0, 0); break;
    case QSIM_OP_Y: setm(0, 0, 0, -1, 0, 1, 0, 0); break;
    case QSIM_OP_Z: setm(1, 0, 0, 0, 0, 0, -1, 0); break;
    case QSIM_OP_S: setm(1, 0, 0, 0, 0, 0, 0, 1); break;
    case QSIM_OP_SDG: setm(1, 0, 0, 0, 0, 0, 0, -1); break;
    case QSIM_OP_T: setm(1, 0, 0, 0, 0, 0, h, h); break;
    case QSIM_OP_TDG: setm(1, 0, 0, 0, 0, 0, h, -h); break;
    case QSIM_OP_RX90: setm(h, 0, 0, h, 0, h, h, 0); break;       // (1/sqrt2)[[1, i], [i, 1]]
    case QSIM_OP_RX90DG: setm(h, 0, 0, -h, 0, -h, h, 0); break;   // conjugate transpose
    case QSIM_OP_RY90: setm(h, 0, h, 0, -h, 0, h, 0); break;      // (1/sqrt2)[[1, 1], [-1, 1]]
    case QSIM_OP_RY90DG: setm(h, 0, -h, 0, h, 0, h, 0); break;    // transpose
    case QSIM_OP_PHASE:
    case QSIM_OP_RK:
    case QSIM_OP_RKDG: {
        const double th = phase_angle(g);
        setm(1, 0, 0, 0, 0, 0, std::cos(th), std::sin(th));
        break;
    }
    case QSIM_OP_RZ:
        setm(std::cos(0.5 * g.theta), -std::sin(0.5 * g.theta), 0, 0, 0, 0, std::cos(0.5 * g.theta), std::sin(0.5 * g.theta));
        break;
    case QSIM_OP_V: {
        const double er = std::cos(g.theta), ei = std::sin(g.theta);
        // V = (1/2)[[1 + e, 1 - e], [1 - e, 1 + e]], e = e^{i theta}
        setm(0.5 * (1 + er), 0.5 * ei, 0.5 * (1 - er), -0.5 * ei, 0.5 * (1 - er), -0.5 * ei, 0.5 * (1 + er), 0.5 * ei);
        break;
    }
    default: return set_error(QSIM_EINVAL, "gate_matrix: op has no 2x2 matrix");
    }
    return QSIM_OK;
}

int validate_gate(const qsim_gate &g, int n)
{
    if (g.op < 0 || g.op >= QSIM_OP_COUNT_) return set_error(QSIM_EINVAL, "gate: unknown op code");
    if (g.op == QSIM_OP_RENORM && (g.target != 0 || g.controls != 0))
        return set_error(QSIM_EINVAL, "gate: a renormalisation point takes no qubits (target 0, no controls)");
    if (g.target < 0 || g.target >= n) return set_error(QSIM_EINVAL, "gate: target out of range");
    if (n < 64 && (g.controls >> n) != 0) return set_error(QSIM_EINVAL, "gate: control mask has bits >= n");
    if ((g.controls >> g.target) & 1) return set_error(QSIM_EINVAL, "gate: control mask contains the target");
    if (g.op == QSIM_OP_SWAP) {
        if (g.target2 < 0 || g.target2 >= n || g.target2 == g.target)
            return set_error(QSIM_EINVAL, "gate: swap needs two distinct qubits");
        if ((g.controls >> g.target2) & 1) return set_error(QSIM_EINVAL, "gate: control mask contains a swap qubit");
    }
    if ((g.op == QSIM_OP_PHASE || g.op == QSIM_OP_RZ || g.op == QSIM_OP_V) && !std::isfinite(g.theta))
        return set_error(QSIM_EINVAL, "gate: angle is not finite");
    if ((g.op == QSIM_OP_RK || g.op == QSIM_OP_RKDG) && (g.target2 < 0 || g.target2 > 63))
        return set_error(QSIM_EINVAL, "gate: RK needs 0 <= k <= 63 in target2");
    return QSIM_OK;
}

// one gate record as one sweep (the per-gate path); phase angles are evaluated on the device
int apply_gate_record(qsim_state *s, const qsim_gate &g)
{
    if (g.op == QSIM_OP_RENORM) return set_error(QSIM_EINVAL, "a renormalisation point runs only inside a plan");
    const uint64_t tbit = uint64_t(1) << g.target;
    if (g.op == QSIM_OP_SWAP) {
        const uint64_t b2 = uint64_t(1) << g.target2;
        return launch_swap(s, make_index_map(g.controls | tbit | b2, g.controls | tbit), tbit | b2);
    }
    if (g.op == QSIM_OP_PHASE) {
        const double c[2] = {g.theta, 0.0};
        return launch_phase(s, make_index_map(g.controls | tbit, g.controls | tbit), c, DiagMode::Angles);
    }
    if (g.op == QSIM_OP_RK || g.op == QSIM_OP_RKDG) {
        const double c[2] = {g.op == QSIM_OP_RK ? 1.0 : -1.0, double(g.target2)};
        return launch_phase(s, make_index_map(g.controls | tbit, g.controls | tbit), c, DiagMode::Pow2);
    }
    if (g.op == QSIM_OP_RZ) {
        const double d[4] = {-0.5 * g.theta, 0.0, 0.5 * g.theta, 0.0};
        return launch_diag(s, make_index_map(g.controls, g.controls), g.target, d, DiagMode::Angles);
    }
    double u[8];
    int rc = gate_matrix(g, u);
    if (rc) return rc;
    return apply_matrix(s, g.controls, g.target, u);
}

}  // namespace qsim

using namespace qsim;

extern "C" {

const char *qsim_last_error(void) { return g_err.c_str(); }

const char *qsim_version(void) { return "qsim-gfx950 1.0"; }

static int new_state(int n, int dtype, void *stream, qsim_state **out)
{
    if (!out) return set_error(QSIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > QSIM_MAX_QUBITS) return set_error(QSIM_EINVAL, "n out of range");
    if (dtype != QSIM_C64 && dtype != QSIM_C128) return set_error(QSIM_EINVAL, "unknown dtype");
    qsim_state *s = new qsim_state();
    s->n = n;
    s->dtype = dtype;
    s->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "hipGetDevice");
    }
    e = hipMalloc(reinterpret_cast<void **>(&s->scratch), sizeof(double) * kScratchDoubles);
    if (e != hipSuccess) {
        delete s;
        return hip_error(e, "hipMalloc(scratch)");
    }
    *out = s;
    return QSIM_OK;
}

int qsim_alloc(int n, int dtype, void *stream, qsim_state **out)
{
    int rc = new_state(n, dtype, stream, out);
    if (rc) return rc;
    qsim_state *s = *out;
    const size_t bytes = size_t(dim(n)) * amp_bytes(dtype);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && bytes > free_b) {
        qsim_free(s);
        *out = nullptr;
        return set_error(QSIM_ENOMEM, "state does not fit in free device memory");
    }
    hipError_t e = hipMalloc(&s->data, bytes);
    if (e != hipSuccess) {
        s->data = nullptr;
        qsim_free(s);
        *out = nullptr;
        return hip_error(e, "hipMalloc(state)");
    }
    s->owned = true;
    rc = launch_set_basis(s, 0);
    if (rc) {
        qsim_free(s);
        *out = nullptr;
    }
    return rc;
}

int qsim_wrap(void *dev_ptr, int n, int dtype, void *stream, qsim_state **out)
{
    if (!dev_ptr) return set_error(QSIM_EINVAL, "dev_ptr is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ptr) % 16) return set_error(QSIM_EINVAL, "dev_ptr must be 16-byte aligned");
    int rc = new_state(n, dtype, stream, out);
    if (rc) return rc;
    (*out)->data = dev_ptr;
    (*out)->owned = false;
    return QSIM_OK;
}

int qsim_free(qsim_state *s)
{
    if (!s) return QSIM_OK;
    if (s->graph_exec) hipGraphExecDestroy(s->graph_exec);
    if (s->graph) hipGraphDestroy(s->graph);
    if (s->owned && s->data) hipFree(s->data);
    if (s->scratch) hipFree(s->scratch);
    delete s;
    return QSIM_OK;
}

void *qsim_data(qsim_state *s) { return s ? s->data : nullptr; }
int qsim_num_qubits(const qsim_state *s) { return s ? s->n : -1; }
int qsim_get_dtype(const qsim_state *s) { return s ? s->dtype : -1; }

int qsim_set_stream(qsim_state *s, void *stream)
{
    if (int rc = check_state(s)) return rc;
    s->stream = static_cast<hipStream_t>(stream);
    return QSIM_OK;
}

int qsim_set_basis(qsim_state *s, uint64_t x)
{
    if (int rc = check_state(s)) return rc;
    if (x >= dim(s->n)) return set_error(QSIM_EINVAL, "basis index >= 2^n");
    return launch_set_basis(s, x);
}

int qsim_upload(qsim_state *s, const void *host, size_t bytes)
{
    if (int rc = check_state(s)) return rc;
    if (!host) return set_error(QSIM_EINVAL, "host is NULL");
    if (bytes != size_t(dim(s->n)) * amp_bytes(s->dtype)) return set_error(QSIM_EINVAL, "byte count != 2^n * amplitude size");
    QSIM_HIP(hipMemcpyAsync(s->data, host, bytes, hipMemcpyHostToDevice, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

int qsim_download(qsim_state *s, void *host, size_t bytes)
{
    if (int rc = check_state(s)) return rc;
    if (!host) return set_error(QSIM_EINVAL, "host is NULL");
    if (bytes != size_t(dim(s->n)) * amp_bytes(s->dtype)) return set_error(QSIM_EINVAL, "byte count != 2^n * amplitude size");
    QSIM_HIP(hipMemcpyAsync(host, s->data, bytes, hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

int qsim_sync(qsim_state *s)
{
    if (int rc = check_state(s)) return rc;
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

int qsim_apply_1q(qsim_state *s, int target, const double U[8])
{
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, target, "target")) return rc;
    if (!U) return set_error(QSIM_EINVAL, "U is NULL");
    return apply_matrix(s, 0, target, U);
}

int qsim_apply_ctrl(qsim_state *s, uint64_t control_mask, int target, const double U[8])
{
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, target, "target")) return rc;
    if (int rc = check_mask(s, control_mask)) return rc;
    if ((control_mask >> target) & 1) return set_error(QSIM_EINVAL, "control mask contains the target");
    if (!U) return set_error(QSIM_EINVAL, "U is NULL");
    return apply_matrix(s, control_mask, target, U);
}

int qsim_apply_phase(qsim_state *s, uint64_t control_mask, int target, double theta)
{
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, target, "target")) return rc;
    if (int rc = check_mask(s, control_mask)) return rc;
    if ((control_mask >> target) & 1) return set_error(QSIM_EINVAL, "control mask contains the target");
    if (!std::isfinite(theta)) return set_error(QSIM_EINVAL, "theta is not finite");
    const uint64_t tbit = uint64_t(1) << target;
    const double c[2] = {theta, 0.0};
    return launch_phase(s, make_index_map(control_mask | tbit, control_mask | tbit), c, DiagMode::Angles);
}

int qsim_apply_swap(qsim_state *s, uint64_t control_mask, int q0, int q1)
{
    if (int rc = check_state(s)) return rc;
    if (int rc = check_qubit(s, q0, "q0")) return rc;
    if (int rc = check_qubit(s, q1, "q1")) return rc;
    if (q0 == q1) return set_error(QSIM_EINVAL, "swap qubits must differ");
    if (int rc = check_mask(s, control_mask)) return rc;
    const uint64_t b0 = uint64_t(1) << q0, b1 = uint64_t(1) << q1;
    if (control_mask & (b0 | b1)) return set_error(QSIM_EINVAL, "control mask contains a swap qubit");
    return launch_swap(s, make_index_map(control_mask | b0 | b1, control_mask | b0), b0 | b1);
}

int qsim_apply_modexp(qsim_state *s, int x_first, int x_qubits, int f_first, int f_qubits, uint64_t y, uint64_t G)
{
    if (int rc = check_state(s)) return rc;
    if (x_qubits < 1 || x_qubits > 30 || f_qubits < 1 || f_qubits > 32)
        return set_error(QSIM_EINVAL, "modexp: register sizes out of range (x: 1..30, f: 1..32 qubits)");
    if (x_first < 0 || f_first < 0 || x_first + x_qubits > s->n || f_first + f_qubits > s->n)
        return set_error(QSIM_EINVAL, "modexp: a register extends beyond the state");
    if (!(x_first + x_qubits <= f_first || f_first + f_qubits <= x_first))
        return set_error(QSIM_EINVAL, "modexp: the x- and f-registers overlap");
    if (G < 2 || G > (uint64_t(1) << f_qubits) || G > 0xffffffffull)
        return set_error(QSIM_EINVAL, "modexp: need 2 <= G <= 2^f_qubits and G < 2^32");
    return launch_modexp(s, x_first, x_qubits, f_first, y, G);
}

int qsim_apply_fused(qsim_state *s, int k, const int *qubits, const double *U)
{
    if (int rc = check_state(s)) return rc;
    if (!qubits || !U) return set_error(QSIM_EINVAL, "qubits or U is NULL");
    if (k < 1 || k > 5 || k > s->n) return set_error(QSIM_EINVAL, "k out of range (1..min(5, n))");
    uint64_t seen = 0;
    for (int i = 0; i < k; ++i) {
        if (int rc = check_qubit(s, qubits[i], "fused qubit")) return rc;
        if ((seen >> qubits[i]) & 1) return set_error(QSIM_EINVAL, "fused qubits repeat");
        seen |= uint64_t(1) << qubits[i];
    }
    return launch_fused(s, k, qubits, U);
}

int qsim_norm(qsim_state *s, double *out)
{
    if (int rc = check_state(s)) return rc;
    if (!out) return set_error(QSIM_EINVAL, "out is NULL");
    return run_norm(s, out);
}

int qsim_probs(qsim_state *s, double *out, int out_is_device)
{
    if (int rc = check_state(s)) return rc;
    if (!out) return set_error(QSIM_EINVAL, "out is NULL");
    const uint64_t N = dim(s->n);
    if (out_is_device) return launch_probs(s, out, 0, N);
    // host output: stream through the scratch buffer in chunks
    const uint64_t chunk = uint64_t(kScratchDoubles) / 2;
    double *stage = s->scratch + chunk;
    for (uint64_t first = 0; first < N; first += chunk) {
        const uint64_t cnt = (N - first < chunk) ? (N - first) : chunk;
        if (int rc = launch_probs(s, stage, first, cnt)) return rc;
        QSIM_HIP(hipMemcpyAsync(out + first, stage, sizeof(double) * cnt, hipMemcpyDeviceToHost, s->stream));
        QSIM_HIP(hipStreamSynchronize(s->stream));
    }
    return QSIM_OK;
}

int qsim_marginals(qsim_state *s, double *out)
{
    if (int rc = check_state(s)) return rc;
    if (!out) return set_error(QSIM_EINVAL, "out is NULL");
    return run_marginals(s, out);
}

int qsim_renormalize(qsim_state *s, double *norm_before)
{
    if (int rc = check_state(s)) return rc;
    return run_renormalize(s, norm_before);
}

int qsim_sample(qsim_state *s, int64_t shots, const double *uniforms, uint64_t *out)
{
    if (int rc = check_state(s)) return rc;
    if (shots < 0) return set_error(QSIM_EINVAL, "shots < 0");
    if (shots == 0) return QSIM_OK;
    if (!uniforms || !out) return set_error(QSIM_EINVAL, "uniforms or out is NULL");
    return run_sample(s, shots, uniforms, out);
}

}  // extern "C"
