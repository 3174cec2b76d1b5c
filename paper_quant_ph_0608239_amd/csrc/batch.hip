// Many independent small circuits in one launch sequence.
//
// Every circuit gets its own LDS-staged schedule (the passes of staged.hip) and its own slot in a
// device state pool. A circuit whose state holds at least kSplitBlocks LDS blocks is split: its pass p
// runs as chunks of blocks that any workgroup may take, in launch step p, so that the largest circuits
// spread over the whole device instead of running their passes block by block on one workgroup (the
// blocks of one pass are independent; launch order on the stream orders pass p before pass p + 1).
// The smaller circuits run whole, all passes on one workgroup, in step 0. Within a step, workgroups of
// a persistent grid walk a fixed list of items in a static cyclic order (workgroup w takes items w,
// w + G, w + 2G, ...), the whole circuits first, largest first. A split pass runs on the wave-split,
// half-buffer or full-buffer kernel that its round trips allow, as in a single staged pass. Pass 0
// generates |0...0> inside its loads instead of reading the pool. A circuit smaller than one LDS block
// runs padded to the block size: its extra high qubits are never touched by a gate and stay |0>, so
// the first 2^n amplitudes of the slot are its state. Device wall-clock stamps give per-circuit
// latency: the first start of any of its pass-0 items to the last end of its last pass.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "qsim_internal.h"
#include "staged_device.h"

using namespace qsim;
using namespace qsim::staged;

namespace {

constexpr uint64_t kSplitBlocks = 8;  // circuits with at least this many LDS blocks per pass are split
constexpr uint64_t kChunkBlocks = 4;  // blocks per item of a split pass

struct BatchCirc {
    int32_t n;          // qubits of the circuit
    int32_t n_eff;      // qubits simulated (>= block size)
    int32_t pass_begin, pass_end;
    uint64_t slot;      // offset of the state in the pool, in amplitudes
};

// One item of a launch step: blocks [b0, b1) of pass `pass` of circuit `circ`, or, with pass < 0, every
// pass of the circuit. first / last: the pass is the circuit's first / last.
struct BatchItem {
    int32_t circ;
    int32_t pass;
    uint32_t b0, b1;
    int32_t first, last;
};

enum Form { kFull = 0, kHalf = 1, kWave = 2 };

// one block of a pass in the kernel form FORM; afterwards every thread has finished its LDS reads, so
// the workgroup may start another block
template <typename T, int LOG_E, int LOG_T, int FORM>
__device__ __forceinline__ void item_block(T *__restrict__ a, const SPass &pass, uint64_t b, cptr<SStage> stages,
                                           cptr<SRound> rounds, cptr<SOp> ops, cptr<SBlk> blks, typename Vec<T>::C *lds,
                                           bool init)
{
    if constexpr (FORM == kWave) {
        run_block_wave<T, LOG_E, LOG_T>(a, pass, b, stages, rounds, ops, blks, lds, init, SEdge{nullptr, nullptr});
        __syncthreads();
    } else if constexpr (FORM == kHalf) {
        run_block_half<T, LOG_E, LOG_T>(a, pass, b, stages, rounds, ops, blks, lds, init, SEdge{nullptr, nullptr});
        __syncthreads();
    } else {
        run_block<T, LOG_E, LOG_T>(a, pass, b, stages, rounds, ops, blks, lds, init, SEdge{nullptr, nullptr});  // ends with a barrier
    }
}

template <typename T, int LOG_E, int LOG_T, int MINW, int FORM>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_batch(T *__restrict__ pool, const BatchCirc *__restrict__ circs,
                                                            const BatchItem *__restrict__ items, int nitems,
                                                            const SPass *__restrict__ passes, const SStage *__restrict__ stages,
                                                            const SRound *__restrict__ rounds, const SOp *__restrict__ ops,
                                                            const SBlk *__restrict__ blks, uint64_t *__restrict__ t_claim,
                                                            uint64_t *__restrict__ t_done)
{
    using C = typename Vec<T>::C;
    constexpr int M = LOG_E + LOG_T;
    __shared__ C lds[lds_slots<T>(FORM == kFull ? M : M - 1)];
    // items in a fixed cyclic order: the loop bounds are kernel constants, so every barrier below sits in
    // uniform control flow
    for (int i = blockIdx.x; i < nitems; i += gridDim.x) {
        const BatchItem it = items[i];
        const BatchCirc bc = circs[it.circ];
        const uint64_t t0 = wall_clock64();
        T *a = pool + 2 * bc.slot;
        if constexpr (FORM == kFull) {
            if (it.pass < 0) {
                const uint64_t nblocks = uint64_t(1) << (bc.n_eff - M);
                for (int p = bc.pass_begin; p < bc.pass_end; ++p) {
                    const SPass pass = ldc<SPass>(as_const(passes) + p);
                    for (uint64_t b = 0; b < nblocks; ++b)
                        item_block<T, LOG_E, LOG_T, FORM>(a, pass, b, as_const(stages), as_const(rounds), as_const(ops), as_const(blks), lds,
                                                          p == bc.pass_begin);
                    // the next pass reads, from other threads of this workgroup, what this one wrote:
                    // a workgroup-scope barrier (release/acquire) orders it; all threads share the CU's L1
                    __syncthreads();
                }
            }
        }
        if (it.pass >= 0) {
            const SPass pass = ldc<SPass>(as_const(passes) + it.pass);
            for (uint64_t b = it.b0; b < it.b1; ++b)
                item_block<T, LOG_E, LOG_T, FORM>(a, pass, b, as_const(stages), as_const(rounds), as_const(ops), as_const(blks), lds,
                                                  it.first != 0);
        }
        if (threadIdx.x == 0) {
            if (it.first) atomicMin(reinterpret_cast<unsigned long long *>(t_claim + it.circ), (unsigned long long)t0);
            if (it.last) atomicMax(reinterpret_cast<unsigned long long *>(t_done + it.circ), (unsigned long long)wall_clock64());
        }
    }
}

// per-circuit stamps of a run start empty: first start = max, last end = 0
__global__ void k_batch_reset(uint64_t *__restrict__ t_claim, uint64_t *__restrict__ t_done, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        t_claim[i] = ~uint64_t(0);
        t_done[i] = 0;
    }
}

// a kernel launch of the run: the items [begin, begin + count) in kernel form `form` on `grid` workgroups
struct BatchLaunch {
    int form, begin, count, grid;
};

}  // namespace

struct qsim_batch {
    int count = 0, dtype = 0, m = 0, log_e = 0, log_t = 0;
    bool use_graph = false;
    hipStream_t stream = nullptr;
    std::vector<BatchCirc> circs;
    std::vector<BatchLaunch> launches;
    int steps = 0, split = 0;
    int64_t total_gates = 0;
    void *pool = nullptr;
    BatchCirc *d_circs = nullptr;
    BatchItem *d_items = nullptr;
    SPass *d_passes = nullptr;
    SStage *d_stages = nullptr;
    SRound *d_rounds = nullptr;
    SOp *d_ops = nullptr;
    SBlk *d_blks = nullptr;
    uint64_t *d_tclaim = nullptr, *d_tdone = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double wall_khz = 0.0;
    int grid[3] = {0, 0, 0};  // persistent grid of each kernel form (0: no kernel of that form)
};

namespace {

template <typename T, int LE, int LT, int MW, int FORM> int form_grid(int *grid)
{
    int per_cu = 0, dev = 0, cus = 0;
    QSIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<T, LE, LT, MW, FORM>, 1 << LT, 0));
    QSIM_HIP(hipGetDevice(&dev));
    QSIM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *grid = std::max(1, per_cu) * cus;
    return QSIM_OK;
}

template <typename T, int LE, int LT, int MW, int FORM> int form_launch(qsim_batch *b, const BatchLaunch &l)
{
    hipLaunchKernelGGL((k_batch<T, LE, LT, MW, FORM>), dim3(l.grid), dim3(1 << LT), 0, b->stream, static_cast<T *>(b->pool),
                       b->d_circs, b->d_items + l.begin, l.count, b->d_passes, b->d_stages, b->d_rounds, b->d_ops, b->d_blks,
                       b->d_tclaim, b->d_tdone);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

// The block shapes a batch can use, with the occupancy of each kernel form: the full-buffer kernel for
// every shape, the half-buffer and wave-split kernels for the shapes that the single staged pass has
// them for. op: 0 = fill b->grid, 1 = launch l.
template <typename T, int LE, int LT, int MWF, int MWH, int MWW, bool HW>
int variant_op(qsim_batch *b, int op, const BatchLaunch *l)
{
    if (op == 0) {
        if (int rc = form_grid<T, LE, LT, MWF, kFull>(&b->grid[kFull])) return rc;
        if constexpr (HW) {
            if (int rc = form_grid<T, LE, LT, MWH, kHalf>(&b->grid[kHalf])) return rc;
            if (int rc = form_grid<T, LE, LT, MWW, kWave>(&b->grid[kWave])) return rc;
        }
        return QSIM_OK;
    }
    if (l->form == kFull) return form_launch<T, LE, LT, MWF, kFull>(b, *l);
    if constexpr (HW) {
        if (l->form == kHalf) return form_launch<T, LE, LT, MWH, kHalf>(b, *l);
        return form_launch<T, LE, LT, MWW, kWave>(b, *l);
    }
    return set_error(QSIM_EINVAL, "batch: no kernel of that form for this block shape");
}

int dispatch(qsim_batch *b, int op, const BatchLaunch *l)
{
    const int v = b->log_e * 16 + b->log_t;
    if (b->dtype == QSIM_C128) {
        switch (v) {
        case 3 * 16 + 8: return variant_op<double, 3, 8, 4, 4, 4, false>(b, op, l);
        case 4 * 16 + 7: return variant_op<double, 4, 7, 2, 3, 4, true>(b, op, l);
        default: return variant_op<double, 4, 8, 2, 3, 4, true>(b, op, l);
        }
    }
    switch (v) {
    case 4 * 16 + 7: return variant_op<float, 4, 7, 3, 3, 3, false>(b, op, l);
    case 5 * 16 + 8: return variant_op<float, 5, 8, 1, 3, 4, true>(b, op, l);
    default: return variant_op<float, 4, 8, 3, 3, 3, false>(b, op, l);
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

// the kernel form that runs a pass (as for a single staged pass), given the forms the shape has
int pass_form(const SPass &ps, const qsim_batch *b)
{
    if (b->grid[kWave] && (ps.direct & 12) == 12) return kWave;
    if (b->grid[kHalf] && (ps.direct & 4)) return kHalf;
    return kFull;
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
    if (int rc = dispatch(b, 0, nullptr)) {
        delete b;
        return rc;
    }
    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SRound> rounds;
    std::vector<SOp> ops;
    std::vector<SBlk> blks;
    uint64_t slot = 0;
    for (int c = 0; c < count; ++c) {
        BatchCirc bc{};
        bc.n = nqubits[c];
        bc.n_eff = std::max(bc.n, m);
        std::vector<qsim_gate> gl(gates + offsets[c], gates + offsets[c + 1]);
        for (const qsim_gate &g : gl) {
            if (int rc = validate_gate(g, bc.n)) {
                delete b;
                return rc;
            }
            if (g.op == QSIM_OP_RENORM) {
                delete b;
                return set_error(QSIM_EINVAL, "batch: renormalisation points run only inside plans");
            }
        }
        b->total_gates += int64_t(gl.size());
        bc.pass_begin = int(passes.size());
        if (int rc = staged_schedule(bc.n_eff, dtype, m, log_e, gl, passes, stages, rounds, ops, blks)) {
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
    // launch steps: step p holds pass p of every split circuit, as chunks of blocks per kernel form;
    // step 0 also holds the whole circuits, largest first
    std::vector<std::vector<BatchItem>> by[3];
    auto at = [&](int form, int step) -> std::vector<BatchItem> & {
        if (int(by[form].size()) <= step) by[form].resize(size_t(step) + 1);
        return by[form][size_t(step)];
    };
    std::vector<int> whole;
    for (int c = 0; c < count; ++c) {
        const BatchCirc &bc = b->circs[size_t(c)];
        const uint64_t nblocks = uint64_t(1) << (bc.n_eff - m);
        if (nblocks < kSplitBlocks) {
            whole.push_back(c);
            continue;
        }
        ++b->split;
        for (int p = bc.pass_begin; p < bc.pass_end; ++p) {
            const int step = p - bc.pass_begin;
            std::vector<BatchItem> &dst = at(pass_form(passes[size_t(p)], b), step);
            for (uint64_t b0 = 0; b0 < nblocks; b0 += kChunkBlocks)
                dst.push_back(BatchItem{c, p, uint32_t(b0), uint32_t(std::min(nblocks, b0 + kChunkBlocks)),
                                        p == bc.pass_begin, p == bc.pass_end - 1});
        }
    }
    auto cost = [&](int c) {
        const BatchCirc &bc = b->circs[size_t(c)];
        return uint64_t(bc.pass_end - bc.pass_begin) << (bc.n_eff - m);
    };
    std::stable_sort(whole.begin(), whole.end(), [&](int x, int y) { return cost(x) > cost(y); });
    {
        std::vector<BatchItem> w;
        for (int c : whole) w.push_back(BatchItem{c, -1, 0, 0, 1, 1});
        std::vector<BatchItem> &dst = at(kFull, 0);
        dst.insert(dst.begin(), w.begin(), w.end());
    }
    std::vector<BatchItem> items;
    int nsteps = 0;
    for (int f = 0; f < 3; ++f) nsteps = std::max(nsteps, int(by[f].size()));
    for (int s = 0; s < nsteps; ++s)
        for (int f = 0; f < 3; ++f) {
            if (s >= int(by[f].size()) || by[f][size_t(s)].empty()) continue;
            const std::vector<BatchItem> &v = by[f][size_t(s)];
            b->launches.push_back(BatchLaunch{f, int(items.size()), int(v.size()), std::min(b->grid[f], int(v.size()))});
            items.insert(items.end(), v.begin(), v.end());
        }
    b->steps = nsteps;
    const size_t pool_bytes = size_t(slot) * amp_bytes(dtype);
    auto fail = [&](hipError_t e, const char *what) {
        qsim_batch_free(b);
        return hip_error(e, what);
    };
    hipError_t e;
    if ((e = hipMalloc(&b->pool, pool_bytes)) != hipSuccess) return fail(e, "batch: state pool");
    if ((e = hipMalloc(&b->d_circs, sizeof(BatchCirc) * count)) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_items, sizeof(BatchItem) * std::max<size_t>(1, items.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_passes, sizeof(SPass) * passes.size())) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_stages, sizeof(SStage) * std::max<size_t>(1, stages.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_rounds, sizeof(SRound) * std::max<size_t>(1, rounds.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_ops, sizeof(SOp) * std::max<size_t>(1, ops.size()))) != hipSuccess) return fail(e, "batch: tables");
    if ((e = hipMalloc(&b->d_blks, sizeof(SBlk) * std::max<size_t>(1, blks.size()))) != hipSuccess) return fail(e, "batch: tables");
    if (!blks.empty() && (e = hipMemcpy(b->d_blks, blks.data(), sizeof(SBlk) * blks.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "batch: upload");
    if ((e = hipMalloc(&b->d_tclaim, sizeof(uint64_t) * count)) != hipSuccess) return fail(e, "batch: timestamps");
    if ((e = hipMalloc(&b->d_tdone, sizeof(uint64_t) * count)) != hipSuccess) return fail(e, "batch: timestamps");
    if ((e = hipMemcpy(b->d_circs, b->circs.data(), sizeof(BatchCirc) * count, hipMemcpyHostToDevice)) != hipSuccess) return fail(e, "batch: upload");
    if (!items.empty() && (e = hipMemcpy(b->d_items, items.data(), sizeof(BatchItem) * items.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e, "batch: upload");
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
    *out = b;
    return QSIM_OK;
}

// the launch sequence of one run: clear the stamps, then every step's kernels in order
static int batch_launch_all(qsim_batch *b)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(unsigned((b->count + 255) / 256)), dim3(256), 0, b->stream, b->d_tclaim, b->d_tdone,
                       b->count);
    QSIM_HIP(hipGetLastError());
    for (const BatchLaunch &l : b->launches)
        if (int rc = dispatch(b, 1, &l)) return rc;
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
            rc = batch_launch_all(b);
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
        rc = batch_launch_all(b);
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

int qsim_batch_get_info(const qsim_batch *b, qsim_batch_info *info)
{
    if (!b || !info) return set_error(QSIM_EINVAL, "null argument");
    info->circuits = b->count;
    info->gates = b->total_gates;
    info->split_circuits = b->split;
    info->steps = b->steps;
    info->launches = int64_t(b->launches.size()) + 1;
    info->lds_qubits = b->m;
    info->lds_regs = b->log_e;
    return QSIM_OK;
}

int qsim_batch_download(qsim_batch *b, int c, void *host, size_t bytes)
{
    if (!b || !host) return set_error(QSIM_EINVAL, "null argument");
    if (c < 0 || c >= b->count) return set_error(QSIM_EINVAL, "batch: circuit index out of range");
    const BatchCirc &bc = b->circs[size_t(c)];
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
    free_dev(b->d_items);
    free_dev(b->d_passes);
    free_dev(b->d_stages);
    free_dev(b->d_rounds);
    free_dev(b->d_ops);
    free_dev(b->d_blks);
    free_dev(b->d_tclaim);
    free_dev(b->d_tdone);
    delete b;
    return QSIM_OK;
}

}  // extern "C"
