// LDS-staged passes: several gates per read and write of the state.
//
// The paper distributes the state over processors and calls the qubits held in one processor's
// memory "local": gates on local qubits need no communication (Sec. III.B). Here the same idea is
// applied to one workgroup's LDS. A pass picks m resident qubits R (always the lowest L index bits,
// so that every block is a set of contiguous runs of >= 256 bytes, plus the targets of the next
// pending gates). Block b of the pass holds the 2^m amplitudes whose index bits outside R equal b.
// A workgroup loads its block into LDS, applies, in circuit order, every pending gate whose target
// is resident and that no skipped earlier gate blocks (controls and diagonal gates may sit on any
// qubit: outside R they are constants of the block), then writes the block back once.
//
// Inside a block, gates run in stages. In a stage each thread holds E = 2^LOG_E amplitudes in
// registers: the amplitudes whose local index has the thread's bits at the "thread bits" TB and
// any value at the stage's "register bits" RB (|RB| = LOG_E). Gates whose target is a register
// bit are register-only (no LDS, no barrier); diagonal gates run in any stage. Between stages the
// block goes through LDS once to change RB. LDS slots are padded (one slot per 2^P) so that the
// usual RB/TB splits are free of bank conflicts.
#include <algorithm>
#include <cmath>

#include "qsim_internal.h"

#include "staged_device.h"

namespace qsim {

using namespace staged;

namespace {

template <typename T, int LOG_E, int LOG_T, int MINW>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_staged(T *__restrict__ a, const SPass *__restrict__ passp,
                                                             const SStage *__restrict__ stages, const SOp *__restrict__ ops)
{
    using C = typename Vec<T>::C;
    __shared__ C lds[lds_slots<T>(LOG_E + LOG_T)];
    const SPass pass = *passp;
    run_block<T, LOG_E, LOG_T>(a, pass, blockIdx.x, stages, ops, lds, false);
}

}  // namespace

namespace staged {
// phase factors of angle-defined operations, evaluated once per plan in FP64 on the device
__global__ void k_op_angles(SOp *ops, int nops)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nops) return;
    SOp &op = ops[i];
    if (op.angles == 1) {
        sincos(op.theta[0], &op.m[1], &op.m[0]);
    } else if (op.angles == 2) {
        sincos(op.theta[0], &op.m[1], &op.m[0]);
        sincos(op.theta[1], &op.m[3], &op.m[2]);
    }
}
}  // namespace staged

// ------------------------------------------------------------------------------------------------
// host side: scheduling
// ------------------------------------------------------------------------------------------------
struct StagedPlan;
void staged_free(StagedPlan *p);

struct StagedPlan {
    int n = 0, dtype = 0, m = 0, log_e = 0, log_t = 0;
    std::vector<SPass> passes;
    SPass *d_passes = nullptr;
    SStage *d_stages = nullptr;
    SOp *d_ops = nullptr;
};

namespace {

enum GKind { G_DENSE, G_X, G_PHASE, G_DIAG, G_SWAP };

struct GInfo {
    GKind kind;
    int target, target2;
    uint64_t controls;
    uint64_t qmask;   // every qubit the gate touches
    double m[8];
    double theta[2];
    int angles;
};

GInfo describe(const qsim_gate &g)
{
    GInfo d{};
    d.target = g.target;
    d.target2 = g.op == QSIM_OP_SWAP ? g.target2 : -1;
    d.controls = g.controls;
    d.qmask = g.controls | (uint64_t(1) << g.target) | (g.op == QSIM_OP_SWAP ? (uint64_t(1) << g.target2) : 0);
    if (g.op == QSIM_OP_SWAP) {
        d.kind = G_SWAP;
        return d;
    }
    if (g.op == QSIM_OP_PHASE) {
        d.kind = G_PHASE;
        d.angles = 1;
        d.theta[0] = g.theta;
        return d;
    }
    if (g.op == QSIM_OP_RZ) {
        d.kind = G_DIAG;
        d.angles = 2;
        d.theta[0] = -0.5 * g.theta;
        d.theta[1] = 0.5 * g.theta;
        return d;
    }
    double u[8];
    gate_matrix(g, u);
    switch (classify(u)) {
    case Kind::Phase1: d.kind = G_PHASE; d.m[0] = u[6]; d.m[1] = u[7]; break;
    case Kind::Diag: d.kind = G_DIAG; d.m[0] = u[0]; d.m[1] = u[1]; d.m[2] = u[6]; d.m[3] = u[7]; break;
    case Kind::Swap: d.kind = G_X; memcpy(d.m, u, sizeof(u)); break;
    default: d.kind = G_DENSE; memcpy(d.m, u, sizeof(u)); break;
    }
    return d;
}

inline bool diagonal(const GInfo &g) { return g.kind == G_PHASE || g.kind == G_DIAG; }

}  // namespace

// kernel variants: (amplitudes per thread, threads) per dtype; see launch_pass
bool staged::staged_variant_ok(int dtype, int log_e, int log_t)
{
    if (log_t < 6 || log_t > 9) return false;
    if (dtype == QSIM_C128) return (log_e == 3 && log_t >= 7) || (log_e == 4 && log_t <= 8);
    return (log_e == 4 && log_t >= 7) || (log_e == 5 && log_t <= 8);
}

// Schedule `gates` for an n-qubit state into passes of m resident qubits with 2^log_e amplitudes per
// thread; passes, stages and ops are appended to the given tables (indices are absolute).
int staged::staged_schedule(int n, int dtype, int m, int log_e, const std::vector<qsim_gate> &gates,
                            std::vector<SPass> &passes, std::vector<SStage> &stages, std::vector<SOp> &ops)
{
    const int L = dtype == QSIM_C128 ? 4 : 5;  // low run: 2^L amplitudes = 256 bytes
    const size_t G = gates.size();
    std::vector<GInfo> gi(G);
    for (size_t i = 0; i < G; ++i) gi[i] = describe(gates[i]);
    std::vector<char> done(G, 0);
    size_t ndone = 0;


    while (ndone < G) {
        // --- resident set: the low run, then the targets of the earliest pending non-diagonal gates
        uint64_t R = (uint64_t(1) << L) - 1;
        int cnt = L;
        for (size_t i = 0; i < G && cnt < m; ++i) {
            if (done[i] || diagonal(gi[i])) continue;
            const int tg[2] = {gi[i].target, gi[i].target2};
            const int need = (gi[i].kind == G_SWAP) ? 2 : 1;
            int missing = 0;
            for (int k = 0; k < need; ++k)
                if (!((R >> tg[k]) & 1)) ++missing;
            if (cnt + missing > m) break;
            for (int k = 0; k < need; ++k)
                if (!((R >> tg[k]) & 1)) {
                    R |= uint64_t(1) << tg[k];
                    ++cnt;
                }
        }
        for (int q = 0; q < n && cnt < m; ++q)
            if (!((R >> q) & 1)) {
                R |= uint64_t(1) << q;
                ++cnt;
            }
        SPass ps{};
        ps.m = m;
        int localof[64];
        for (int q = 0, s = 0; q < n; ++q) {
            localof[q] = -1;
            if ((R >> q) & 1) {
                ps.R[s] = uint8_t(q);
                localof[q] = s++;
            }
        }
        auto local_mask = [&](uint64_t phys) {
            uint32_t lm = 0;
            for (int q = 0; q < n; ++q)
                if (((phys >> q) & 1) && localof[q] >= 0) lm |= 1u << localof[q];
            return lm;
        };
        // --- executable gates, in circuit order
        std::vector<size_t> take;
        uint64_t blocked = 0;
        for (size_t i = 0; i < G; ++i) {
            if (done[i]) continue;
            const GInfo &g = gi[i];
            if (g.qmask & blocked) {
                blocked |= g.qmask;
                continue;
            }
            bool ok = diagonal(g) || ((R >> g.target) & 1);
            if (g.kind == G_SWAP) ok = ((R >> g.target) & 1) && ((R >> g.target2) & 1);
            if (ok) take.push_back(i);
            else blocked |= g.qmask;
        }
        // --- stages
        ps.stage_begin = int(stages.size());
        SStage cur{};
        uint32_t rbset = 0;
        int nrb = 0;
        cur.op_begin = int(ops.size());
        cur.swap_p = cur.swap_q = -1;
        auto close_stage = [&]() {
            // fill the register bits from the top local bits so the thread bits keep the low ones
            for (int s = m - 1; s >= 0 && nrb < log_e; --s)
                if (!((rbset >> s) & 1)) {
                    rbset |= 1u << s;
                    ++nrb;
                }
            int j = 0, jt = 0;
            for (int s = 0; s < m; ++s) {
                if ((rbset >> s) & 1) cur.rb[j++] = uint8_t(s);
                else cur.tbits[jt++] = uint8_t(s);
            }
            cur.op_end = int(ops.size());
            stages.push_back(cur);
            cur = SStage{};
            cur.op_begin = int(ops.size());
            cur.swap_p = cur.swap_q = -1;
            rbset = 0;
            nrb = 0;
        };
        auto rbit_of = [&](uint32_t lb) {
            // index of local bit lb among the stage's register bits (fixed at close: ascending)
            return lb;
        };
        (void)rbit_of;
        std::vector<std::pair<size_t, int>> pending_rbit;  // op index -> local target bit (fixed up at close)
        auto rank_of = [&](int lb) {  // register-bit index of local bit lb (rank among the sorted RB)
            int rank = 0;
            for (int s = 0; s < lb; ++s)
                if ((rbset >> s) & 1) ++rank;
            return rank;
        };
        auto fix_rbits = [&]() {
            for (auto &pr : pending_rbit) ops[pr.first].rbit = rank_of(pr.second);
            pending_rbit.clear();
            // split every condition of the stage into its register part (as a mask over the
            // register index r) and its thread part
            for (size_t oi = size_t(cur.op_begin); oi < ops.size(); ++oi) {
                SOp &o = ops[oi];
                o.rsel = 0;
                for (int s = 0; s < m; ++s)
                    if (((o.lcm >> s) & 1) && ((rbset >> s) & 1)) o.rsel |= 1u << rank_of(s);
                o.lcm_t = o.lcm & ~rbset;
                if (o.type == 3) o.rbit = (o.lt >= 0 && ((rbset >> o.lt) & 1)) ? rank_of(o.lt) : -1;
            }
        };
        for (size_t i : take) {
            const GInfo &g = gi[i];
            SOp op{};
            op.gcm = g.controls & ~R;
            op.lcm = local_mask(g.controls);
            op.lt = -1;
            if (g.kind == G_SWAP) {
                // ends the current stage as an LDS permutation
                cur.swap_p = localof[g.target];
                cur.swap_q = localof[g.target2];
                cur.swap_lcm = local_mask(g.controls);
                cur.swap_gcm = g.controls & ~R;
                // fill RB and close (before fix_rbits uses the final set)
                for (int s = m - 1; s >= 0 && nrb < log_e; --s)
                    if (!((rbset >> s) & 1)) {
                        rbset |= 1u << s;
                        ++nrb;
                    }
                fix_rbits();
                close_stage();
                continue;
            }
            if (diagonal(g)) {
                if (g.kind == G_PHASE) {
                    op.type = 2;
                    // condition: controls and the target bit are 1
                    const uint64_t cond = g.controls | (uint64_t(1) << g.target);
                    op.gcm = cond & ~R;
                    op.lcm = local_mask(cond);
                    op.m[0] = g.m[0];
                    op.m[1] = g.m[1];
                } else {
                    op.type = 3;
                    if ((R >> g.target) & 1) {
                        op.lt = localof[g.target];
                    } else {
                        op.lt = -1;
                        op.gtb = uint64_t(1) << g.target;
                    }
                    memcpy(op.m, g.m, sizeof(op.m));
                }
                op.angles = g.angles;
                op.theta[0] = g.theta[0];
                op.theta[1] = g.theta[1];
                ops.push_back(op);
                continue;
            }
            // dense or X on a resident target
            const int lb = localof[g.target];
            if (!((rbset >> lb) & 1)) {
                if (nrb == log_e) {
                    fix_rbits();
                    close_stage();
                }
                rbset |= 1u << lb;
                ++nrb;
            }
            op.type = 0;  // X runs as the 2x2 [[0,1],[1,0]]: products with exact 0/1 coefficients
            memcpy(op.m, g.m, sizeof(op.m));
            pending_rbit.push_back({ops.size(), lb});
            ops.push_back(op);
        }
        if (int(ops.size()) > cur.op_begin || int(stages.size()) == ps.stage_begin) {
            for (int s = m - 1; s >= 0 && nrb < log_e; --s)
                if (!((rbset >> s) & 1)) {
                    rbset |= 1u << s;
                    ++nrb;
                }
            fix_rbits();
            close_stage();
        }
        ps.stage_end = int(stages.size());
        passes.push_back(ps);
        for (size_t i : take) done[i] = 1;
        ndone += take.size();
        if (take.empty()) return set_error(QSIM_EINVAL, "staged: scheduler made no progress");
    }

    return QSIM_OK;
}

int staged_build(int n, int dtype, const std::vector<qsim_gate> &gates, int lds_qubits, int lds_regs, StagedPlan **out,
                 qsim_plan_info *info)
{
    *out = nullptr;
    // defaults measured on the 30-qubit brickwork: 4096 amplitudes per block, 16 per thread
    const int log_e = lds_regs ? lds_regs : 4;
    int m = lds_qubits ? lds_qubits : 12;
    if (!staged_variant_ok(dtype, log_e, m - log_e))
        return set_error(QSIM_EINVAL, "staged: lds_qubits / lds_regs combination not available for this dtype");
    if (n < m) return set_error(QSIM_EUNSUPPORTED, "staged: the state is smaller than one LDS block");
    const int log_t = m - log_e;

    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SOp> ops;
    if (int rc = staged_schedule(n, dtype, m, log_e, gates, passes, stages, ops)) return rc;
    StagedPlan *p = new StagedPlan();
    p->n = n;
    p->dtype = dtype;
    p->m = m;
    p->log_e = log_e;
    p->log_t = log_t;
    p->passes = passes;
    // one device copy of each pass record, of the stage table and of the op table
    hipError_t e = hipMalloc(&p->d_passes, sizeof(SPass) * passes.size());
    if (e == hipSuccess) e = hipMalloc(&p->d_stages, sizeof(SStage) * std::max<size_t>(1, stages.size()));
    if (e == hipSuccess) e = hipMalloc(&p->d_ops, sizeof(SOp) * std::max<size_t>(1, ops.size()));
    if (e == hipSuccess) e = hipMemcpy(p->d_passes, passes.data(), sizeof(SPass) * passes.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !stages.empty())
        e = hipMemcpy(p->d_stages, stages.data(), sizeof(SStage) * stages.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ops.empty()) e = hipMemcpy(p->d_ops, ops.data(), sizeof(SOp) * ops.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !ops.empty()) {
        hipLaunchKernelGGL(k_op_angles, dim3(unsigned((ops.size() + 255) / 256)), dim3(256), 0, nullptr, p->d_ops, int(ops.size()));
        e = hipGetLastError();
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        staged_free(p);
        return hip_error(e, "staged plan upload");
    }
    info->method = QSIM_PLAN_STAGED;
    info->lds_qubits = m;
    info->lds_regs = log_e;
    info->launches = int64_t(passes.size());
    info->passes = int64_t(passes.size());
    info->alg_bytes = double(passes.size()) * 2.0 * std::ldexp(1.0, n) * amp_bytes(dtype);
    info->alg_flops = 0.0;
    *out = p;
    return QSIM_OK;
}

static int launch_pass(StagedPlan *p, qsim_state *s, size_t i)
{
    const unsigned blocks = unsigned(dim(p->n - p->m));
    const SPass *dp = p->d_passes + i;
#define QSIM_STAGED_LAUNCH(T, LE, LT, MW)                                                                  \
    hipLaunchKernelGGL((k_staged<T, LE, LT, MW>), dim3(blocks), dim3(1 << LT), 0, s->stream, static_cast<T *>(s->data), dp, \
                       p->d_stages, p->d_ops)
    const int v = p->log_e * 16 + p->log_t;
    if (p->dtype == QSIM_C128) {
        switch (v) {
        case 3 * 16 + 7: QSIM_STAGED_LAUNCH(double, 3, 7, 4); break;
        case 3 * 16 + 8: QSIM_STAGED_LAUNCH(double, 3, 8, 4); break;
        case 3 * 16 + 9: QSIM_STAGED_LAUNCH(double, 3, 9, 3); break;
        case 4 * 16 + 6: QSIM_STAGED_LAUNCH(double, 4, 6, 2); break;
        case 4 * 16 + 7: QSIM_STAGED_LAUNCH(double, 4, 7, 2); break;
        default: QSIM_STAGED_LAUNCH(double, 4, 8, 2); break;
        }
    } else {
        switch (v) {
        case 4 * 16 + 7: QSIM_STAGED_LAUNCH(float, 4, 7, 3); break;
        case 4 * 16 + 8: QSIM_STAGED_LAUNCH(float, 4, 8, 3); break;
        case 4 * 16 + 9: QSIM_STAGED_LAUNCH(float, 4, 9, 2); break;
        case 5 * 16 + 6: QSIM_STAGED_LAUNCH(float, 5, 6, 1); break;
        case 5 * 16 + 7: QSIM_STAGED_LAUNCH(float, 5, 7, 1); break;
        default: QSIM_STAGED_LAUNCH(float, 5, 8, 1); break;
        }
    }
#undef QSIM_STAGED_LAUNCH
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int staged_execute(StagedPlan *p, qsim_state *s)
{
    for (size_t i = 0; i < p->passes.size(); ++i)
        if (int rc = launch_pass(p, s, i)) return rc;
    return QSIM_OK;
}

int staged_execute_timed(StagedPlan *p, qsim_state *s, double *ms, int32_t *kind, int32_t *fk)
{
    const size_t L = p->passes.size();
    std::vector<hipEvent_t> ev(2 * L, nullptr);
    for (auto &e : ev) QSIM_HIP(hipEventCreate(&e));
    int rc = QSIM_OK;
    for (size_t i = 0; i < L && !rc; ++i) {
        QSIM_HIP(hipEventRecord(ev[2 * i], s->stream));
        rc = launch_pass(p, s, i);
        QSIM_HIP(hipEventRecord(ev[2 * i + 1], s->stream));
    }
    if (!rc) {
        QSIM_HIP(hipStreamSynchronize(s->stream));
        for (size_t i = 0; i < L; ++i) {
            float tms = 0.f;
            QSIM_HIP(hipEventElapsedTime(&tms, ev[2 * i], ev[2 * i + 1]));
            if (ms) ms[i] = tms;
            if (kind) kind[i] = QSIM_KERNEL_STAGED;
            if (fk) fk[i] = 0;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return rc;
}

void staged_free(StagedPlan *p)
{
    if (!p) return;
    if (p->d_passes) (void)hipFree(p->d_passes);
    if (p->d_stages) (void)hipFree(p->d_stages);
    if (p->d_ops) (void)hipFree(p->d_ops);
    delete p;
}

}  // namespace qsim
