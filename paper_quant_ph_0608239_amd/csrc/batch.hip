// Many independent small circuits in one persistent launch.
//
// Every circuit gets its own LDS-staged schedule (the passes of staged.hip) and its own slot in a
// device state pool. A persistent grid of workgroups (as many as fit on the device at once) walks
// the circuits sorted largest state first, workgroup w taking entries w, w + G, w + 2G, ...; the
// workgroup that takes a circuit runs all of its passes, block by block, generating |0...0> inside
// the first pass instead of reading it. A circuit smaller than one LDS block runs padded to the block size: its extra high qubits are
// never touched by a gate and stay |0>, so the first 2^n amplitudes of the slot are its state.
// Device wall-clock timestamps are taken when a workgroup starts a circuit and when it finishes.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "qsim_internal.h"
#include "staged_device.h"

using namespace qsim;
using namespace qsim::staged;

namespace {

struct BatchCirc {
    int32_t n;          // qubits of the circuit
    int32_t n_eff;      // qubits simulated (>= block size)
    int32_t pass_begin, pass_end;
    uint64_t slot;      // offset of the state in the pool, in amplitudes
};

template <typename T, int LOG_E, int LOG_T, int MINW>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_batch(T *__restrict__ pool, const BatchCirc *__restrict__ circs,
                                                            const int *__restrict__ order, int count,
                                                            const SPass *__restrict__ passes, const SStage *__restrict__ stages,
                                                            const SRound *__restrict__ rounds, const SOp *__restrict__ ops,
                                                            uint64_t *__restrict__ t_claim,
                                                            uint64_t *__restrict__ t_done)
{
    using C = typename Vec<T>::C;
    constexpr int M = LOG_E + LOG_T;
    __shared__ C lds[lds_slots<T>(M)];
    // circuits in a fixed cyclic order over the largest-first list: loop bounds are kernel
    // constants, so every barrier below sits in uniform control flow
    for (int qi = blockIdx.x; qi < count; qi += gridDim.x) {
        const int c = order[qi];
        const BatchCirc bc = circs[c];
        const uint64_t t0 = wall_clock64();
        T *a = pool + 2 * bc.slot;
        const uint64_t nblocks = uint64_t(1) << (bc.n_eff - M);
        for (int p = bc.pass_begin; p < bc.pass_end; ++p) {
            const SPass pass = ldc<SPass>(as_const(passes) + p);
            for (uint64_t b = 0; b < nblocks; ++b) run_block<T, LOG_E, LOG_T>(a, pass, b, as_const(stages), as_const(rounds), as_const(ops), lds, p == bc.pass_begin);
            // the next pass reads, from other threads of this workgroup, what this one wrote:
            // a workgroup-scope barrier (release/acquire) orders it; all threads share the CU's L1
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            t_claim[c] = t0;
            t_done[c] = wall_clock64();
        }
    }
}

}  // namespace

struct qsim_batch {
    int count = 0, dtype = 0, m = 0, log_e = 0, log_t = 0;
    bool use_graph = false;
    hipStream_t stream = nullptr;
    std::vector<BatchCirc> circs;
    std::vector<int> order;
    int64_t total_gates = 0;
    void *pool = nullptr;
    BatchCirc *d_circs = nullptr;
    int *d_order = nullptr;
    SPass *d_passes = nullptr;
    SStage *d_stages = nullptr;
    SRound *d_rounds = nullptr;
    SOp *d_ops = nullptr;
    uint64_t *d_tclaim = nullptr, *d_tdone = nullptr;
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double wall_khz = 0.0;
};

namespace {

template <typename T, int LE, int LT, int MW> int batch_grid(int *grid)
{
    int per_cu = 0, dev = 0, cus = 0;
    QSIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<T, LE, LT, MW>, 1 << LT, 0));
    QSIM_HIP(hipGetDevice(&dev));
    QSIM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *grid = std::max(1, per_cu) * cus;
    return QSIM_OK;
}

template <typename T, int LE, int LT, int MW> int batch_launch(qsim_batch *b)
{
    hipLaunchKernelGGL((k_batch<T, LE, LT, MW>), dim3(b->grid), dim3(1 << LT), 0, b->stream, static_cast<T *>(b->pool),
                       b->d_circs, b->d_order, b->count, b->d_passes, b->d_stages, b->d_rounds, b->d_ops, b->d_tclaim, b->d_tdone);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

// the kernel variants the batch can use (same set as the per-pass staged kernel)
int dispatch_grid(qsim_batch *b)
{
    const int v = b->log_e * 16 + b->log_t;
    if (b->dtype == QSIM_C128) {
        switch (v) {
        case 3 * 16 + 8: return batch_grid<double, 3, 8, 4>(&b->grid);
        case 4 * 16 + 7: return batch_grid<double, 4, 7, 2>(&b->grid);
        default: return batch_grid<double, 4, 8, 2>(&b->grid);
        }
    }
    switch (v) {
    case 4 * 16 + 7: return batch_grid<float, 4, 7, 3>(&b->grid);
    case 5 * 16 + 8: return batch_grid<float, 5, 8, 1>(&b->grid);
    default: return batch_grid<float, 4, 8, 3>(&b->grid);
    }
}

int dispatch_launch(qsim_batch *b)
{
    const int v = b->log_e * 16 + b->log_t;
    if (b->dtype == QSIM_C128) {
        switch (v) {
        case 3 * 16 + 8: return batch_launch<double, 3, 8, 4>(b);
        case 4 * 16 + 7: return batch_launch<double, 4, 7, 2>(b);
        default: return batch_launch<double, 4, 8, 2>(b);
        }
    }
    switch (v) {
    case 4 * 16 + 7: return batch_launch<float, 4, 7, 3>(b);
    case 5 * 16 + 8: return batch_launch<float, 5, 8, 1>(b);
    default: return batch_launch<float, 4, 8, 3>(b);
    }
}

bool batch_variant_ok(int dtype, int log_e, int log_t)
{
    if (dtype == QSIM_C128) return (log_e == 3 && log_t == 8) || (log_e == 4 && (log_t == 7 || log_t == 8));
    return (log_e == 4 && (log_t == 7 || log_t == 8)) || (log_e == 5 && log_t == 8);
}

template <typename P> void free_dev(P *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

}  // namespace

extern "C" {

int qsim_batch_create(int count, const int *nqubits, const int64_t *offsets, const qsim_gate *gates, int dtype,
                      const qsim_plan_opts *opts, void *stream, qsim_batch **out)
{
    if (!out) return set_error(QSIM_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !nqubits || !offsets) return set_error(QSIM_EINVAL, "batch: count < 1 or NULL tables");
    if (dtype != QSIM_C64 && dtype != QSIM_C128) return set_error(QSIM_EINVAL, "unknown dtype");
    const int log_e = (opts && opts->lds_regs) ? opts->lds_regs : 4;
    const int m = (opts && opts->lds_qubits) ? opts->lds_qubits : 12;
    if (!batch_variant_ok(dtype, log_e, m - log_e)) return set_error(QSIM_EINVAL, "batch: lds_qubits / lds_regs not available");
    if (offsets[0] != 0) return set_error(QSIM_EINVAL, "batch: offsets[0] must be 0");
    for (int c = 0; c < count; ++c) {
        if (nqubits[c] < 1 || nqubits[c] > 26) return set_error(QSIM_EINVAL, "batch: qubit counts must lie in 1..26");
        if (offsets[c + 1] < offsets[c]) return set_error(QSIM_EINVAL, "batch: offsets must not decrease");
    }
    if (offsets[count] > 0 && !gates) return set_error(QSIM_EINVAL, "batch: gates is NULL");
    qsim_batch *b = new qsim_batch();
    b->count = count;
    b->dtype = dtype;
    b->m = m;
    b->log_e = log_e;
    b->log_t = m - log_e;
    b->use_graph = opts && opts->use_graph && stream != nullptr;
    b->stream = static_cast<hipStream_t>(stream);
    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SRound> rounds;
    std::vector<SOp> ops;
    uint64_t slot = 0;
    for (int c = 0; c < count; ++c) {
        BatchCirc bc{};
        bc.n = nqubits[c];
        bc.n_eff = std::max(bc.n, m);
        std::vector<qsim_gate> gl(gates + offsets[c], gates + offsets[c + 1]);
        for (const qsim_gate &g : gl)
            if (int rc = validate_gate(g, bc.n)) {
                delete b;
                return rc;
            }
        b->total_gates += int64_t(gl.size());
        bc.pass_begin = int(passes.size());
        if (int rc = staged_schedule(bc.n_eff, dtype, m, log_e, gl, passes, stages, rounds, ops)) {
            delete b;
            return rc;
        }
        if (int(passes.size()) == bc.pass_begin) {  // no gates: one empty pass writes |0...0>
            SPass ps{};
            ps.m = m;
            for (int s = 0; s < m; ++s) ps.R[s] = uint8_t(s);
            ps.stage_begin = ps.stage_end = int(stages.size());
            passes.push_back(ps);
        }
        bc.pass_end = int(passes.size());
        bc.slot = slot;
        slot += uint64_t(1) << bc.n_eff;
        b->circs.push_back(bc);
    }
    b->order.resize(count);
    std::iota(b->order.begin(), b->order.end(), 0);
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return b->circs[x].n_eff > b->circs[y].n_eff; });
    const size_t pool_bytes = size_t(slot) * amp_bytes(dtype);
    auto fail = [&](hipError_t e, const char *what) {
        qsim_batch_free(b);
        return hip_error(e, what);
    };
    hipError_t e;
    if ((e = hipMalloc(&b->pool, pool_bytes)) != hipSuccess) return fail(e, "batch: state pool");
    if ((e = hipMalloc(&b->d_circs, sizeof(BatchCirc) * count)) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_order, sizeof(int) * count)) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_passes, sizeof(SPass) * passes.size())) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_stages, sizeof(SStage) * std::max<size_t>(1, stages.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_rounds, sizeof(SRound) * std::max<size_t>(1, rounds.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_ops, sizeof(SOp) * std::max<size_t>(1, ops.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_tclaim, sizeof(uint64_t) * count)) != hipSuccess) return fail(e, "batch: timestamps");
    if ((e = hipMalloc(&b->d_tdone, sizeof(uint64_t) * count)) != hipSuccess) return fail(e, "batch: timestamps");
    if ((e = hipMemcpy(b->d_circs, b->circs.data(), sizeof(BatchCirc) * count, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "batch: upload");
    if ((e = hipMemcpy(b->d_order, b->order.data(), sizeof(int) * count, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "batch: upload");
    if ((e = hipMemcpy(b->d_passes, passes.data(), sizeof(SPass) * passes.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "batch: upload");
    if (!stages.empty() && (e = hipMemcpy(b->d_stages, stages.data(), sizeof(SStage) * stages.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "batch: upload");
    if (!rounds.empty() && (e = hipMemcpy(b->d_rounds, rounds.data(), sizeof(SRound) * rounds.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "batch: upload");
    if (!ops.empty()) {
        if ((e = hipMemcpy(b->d_ops, ops.data(), sizeof(SOp) * ops.size(), hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "batch: upload");
        hipLaunchKernelGGL(k_op_angles, dim3(unsigned((ops.size() + 255) / 256)), dim3(256), 0, nullptr, b->d_ops, int(ops.size()));
        if ((e = hipGetLastError()) != hipSuccess) return fail(e, "batch: angles");
        if ((e = hipDeviceSynchronize()) != hipSuccess) return fail(e, "batch: angles");
    }
    int dev = 0, khz = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return fail(e, "hipGetDevice");
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return fail(e, "wall clock rate");
    b->wall_khz = double(khz);
    if (int rc = dispatch_grid(b)) {
        qsim_batch_free(b);
        return rc;
    }
    *out = b;
    return QSIM_OK;
}

int qsim_batch_run(qsim_batch *b, qsim_batch_stats *stats)
{
    if (!b) return set_error(QSIM_EINVAL, "null batch");
    hipEvent_t e0, e1;
    QSIM_HIP(hipEventCreate(&e0));
    QSIM_HIP(hipEventCreate(&e1));
    QSIM_HIP(hipEventRecord(e0, b->stream));
    int rc = QSIM_OK;
    if (b->use_graph) {
        if (!b->graph_exec) {
            QSIM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            rc = dispatch_launch(b);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(b->stream, &g);
            if (rc) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (ec != hipSuccess) return hip_error(ec, "batch: hipStreamEndCapture");
            b->graph = g;
            QSIM_HIP(hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
        }
        QSIM_HIP(hipGraphLaunch(b->graph_exec, b->stream));
    } else {
        rc = dispatch_launch(b);
    }
    if (rc) return rc;
    QSIM_HIP(hipEventRecord(e1, b->stream));
    QSIM_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    QSIM_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (stats) {
        stats->launch_ms = ms;
        stats->circuits = b->count;
        stats->gates = b->total_gates;
    }
    return QSIM_OK;
}

int qsim_batch_latencies(qsim_batch *b, double *out_us)
{
    if (!b || !out_us) return set_error(QSIM_EINVAL, "null argument");
    std::vector<uint64_t> t0(b->count), t1(b->count);
    QSIM_HIP(hipMemcpy(t0.data(), b->d_tclaim, sizeof(uint64_t) * b->count, hipMemcpyDeviceToHost));
    QSIM_HIP(hipMemcpy(t1.data(), b->d_tdone, sizeof(uint64_t) * b->count, hipMemcpyDeviceToHost));
    for (int c = 0; c < b->count; ++c) out_us[c] = double(t1[c] - t0[c]) / b->wall_khz * 1e3;
    return QSIM_OK;
}

int qsim_batch_download(qsim_batch *b, int c, void *host, size_t bytes)
{
    if (!b || !host) return set_error(QSIM_EINVAL, "null argument");
    if (c < 0 || c >= b->count) return set_error(QSIM_EINVAL, "batch: circuit index out of range");
    const BatchCirc &bc = b->circs[c];
    const size_t nb = (size_t(1) << bc.n) * amp_bytes(b->dtype);
    if (bytes != nb) return set_error(QSIM_EINVAL, "batch: byte count != 2^n * amplitude size");
    QSIM_HIP(hipMemcpy(host, static_cast<unsigned char *>(b->pool) + bc.slot * amp_bytes(b->dtype), nb, hipMemcpyDeviceToHost));
    return QSIM_OK;
}

int qsim_batch_free(qsim_batch *b)
{
    if (!b) return QSIM_OK;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    free_dev(b->pool);
    free_dev(b->d_circs);
    free_dev(b->d_order);
    free_dev(b->d_passes);
    free_dev(b->d_stages);
    free_dev(b->d_rounds);
    free_dev(b->d_ops);
    free_dev(b->d_tclaim);
    free_dev(b->d_tdone);
    delete b;
    return QSIM_OK;
}

}  // extern "C"
