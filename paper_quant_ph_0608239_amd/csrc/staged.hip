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

namespace qsim {

namespace {

constexpr int kMaxM = 14;

struct SOp {
    int32_t type;      // 0 dense 2x2, 1 X (swap pairs), 2 conditional phase, 3 diag(d0, d1)
    int32_t rbit;      // dense / X: register-bit index of the target; diag: register-bit index of
                       // the target if it is a register bit, else -1
    int32_t lt;        // diag: local bit of the target, or -1 if the target is outside R
    uint32_t lcm;      // local condition mask (local index bits that must be 1)
    uint32_t rsel;     // the part of lcm on register bits, as a mask over the register index r
    uint32_t lcm_t;    // the part of lcm on thread bits (local bit positions)
    int32_t run;       // at the first op of a run: number of consecutive ops of the same class
    int32_t fast;      // 1: uncontrolled 2x2 on a register bit (no resident condition)
    uint64_t gcm;      // condition mask on the block's non-resident index bits (must be 1)
    uint64_t gtb;      // diag with a non-resident target: that bit of the index
    double m[8];       // dense: 2x2; phase: m[0], m[1]; diag: d0 = m[0..1], d1 = m[2..3]
    double theta[2];   // angle inputs, turned into m[] on the device when angles != 0
    int32_t angles;    // 1: phase e^{i theta0}; 2: diag (e^{i theta0}, e^{i theta1})
    int32_t pad;
};

struct SStage {
    int32_t op_begin, op_end;
    uint8_t rb[8];      // register bits (local bit indices), LOG_E of them, ascending
    uint8_t tbits[8];   // thread bits (the other local bits), LOG_T of them, ascending
    int32_t swap_p;     // stage-end local swap (quantum swap of two resident qubits), -1 if none
    int32_t swap_q;
    uint32_t swap_lcm;  // its local condition
    uint32_t pad;
    uint64_t swap_gcm;  // its condition on non-resident bits
};

struct SPass {
    int32_t m;
    int32_t stage_begin, stage_end;
    int32_t pad;
    uint8_t R[16];      // physical bit of local bit s, ascending
};

template <typename T> struct Vec;
template <> struct Vec<double> { using C = double2; };
template <> struct Vec<float> { using C = float2; };

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <typename C> __device__ __forceinline__ C ld_nt(const C *p)
{
    using V = typename std::conditional<sizeof(C) == 16, u32x4, u32x2>::type;
    V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    C c;
    __builtin_memcpy(&c, &v, sizeof(C));
    return c;
}
template <typename C> __device__ __forceinline__ void st_nt(C *p, const C &c)
{
    using V = typename std::conditional<sizeof(C) == 16, u32x4, u32x2>::type;
    V v;
    __builtin_memcpy(&v, &c, sizeof(C));
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
}

// LDS slot of local index e: one padding slot per 2^P slots (P = 4 for 16-byte, 5 for 8-byte
// amplitudes, i.e. one per 256 bytes)
template <typename T> __device__ __forceinline__ int slot(int e) { return sizeof(T) == 8 ? e + (e >> 4) : e + (e >> 5); }
template <typename T> constexpr int lds_slots(int m) { return (1 << m) + ((1 << m) >> (sizeof(T) == 8 ? 4 : 5)); }

template <typename T>
__device__ __forceinline__ void cmul(typename Vec<T>::C &x, T fr, T fi)
{
    const T r = fr * x.x - fi * x.y;
    const T i = fr * x.y + fi * x.x;
    x.x = r;
    x.y = i;
}

// Element r of a thread in a stage has local index et | er[r]: et (the thread's bits, per lane) and
// er[r] (the register bits, the same for every lane) occupy disjoint bits. A condition mask lcm
// therefore splits into a per-lane test on et and a wave-uniform test on er[r], and the padded LDS
// slot is additive: slot(et | er) = slot(et) + slot(er).

// register-bit ops with a compile-time register bit so that every register index is static.
// The lane-dependent part of a condition is folded into the coefficients once per op (identity
// or a phase of 1 on lanes where it fails); the register part (uniform) selects elements with
// scalar branches, so no element is updated through per-lane selects.
template <typename T> struct U2 {
    T r[4], i[4];
};

template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense(typename Vec<T>::C *x, const uint32_t *er, uint32_t lcm_r, const U2<T> &u)
{
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((r >> RB) & 1) continue;
        if ((er[r] & lcm_r) != lcm_r) continue;  // uniform
        const int r1 = r | (1 << RB);
        const auto a = x[r], b = x[r1];
        x[r].x = u.r[0] * a.x - u.i[0] * a.y + u.r[1] * b.x - u.i[1] * b.y;
        x[r].y = u.r[0] * a.y + u.i[0] * a.x + u.r[1] * b.y + u.i[1] * b.x;
        x[r1].x = u.r[2] * a.x - u.i[2] * a.y + u.r[3] * b.x - u.i[3] * b.y;
        x[r1].y = u.r[2] * a.y + u.i[2] * a.x + u.r[3] * b.y + u.i[3] * b.x;
    }
}

template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense_all(typename Vec<T>::C *x, const U2<T> &u)
{
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((r >> RB) & 1) continue;
        const int r1 = r | (1 << RB);
        const auto a = x[r], b = x[r1];
        x[r].x = u.r[0] * a.x - u.i[0] * a.y + u.r[1] * b.x - u.i[1] * b.y;
        x[r].y = u.r[0] * a.y + u.i[0] * a.x + u.r[1] * b.y + u.i[1] * b.x;
        x[r1].x = u.r[2] * a.x - u.i[2] * a.y + u.r[3] * b.x - u.i[3] * b.y;
        x[r1].y = u.r[2] * a.y + u.i[2] * a.x + u.r[3] * b.y + u.i[3] * b.x;
    }
}

// phase factor on the elements whose register index r has every bit of SEL set (compile time)
template <typename T, int E, int SEL>
__device__ __forceinline__ void op_phase_sel(typename Vec<T>::C *x, T fr, T fi, bool flip)
{
    if (flip) {
#pragma unroll
        for (int r = 0; r < E; ++r)
            if ((r & SEL) == SEL) {
                x[r].x *= fr;
                x[r].y *= fr;
            }
    } else {
#pragma unroll
        for (int r = 0; r < E; ++r)
            if ((r & SEL) == SEL) {
                const T re = fr * x[r].x - fi * x[r].y;
                const T im = fr * x[r].y + fi * x[r].x;
                x[r].x = re;
                x[r].y = im;
            }
    }
}

template <typename T, int E>
__device__ __forceinline__ void phase_dispatch(int sel, typename Vec<T>::C *x, T fr, T fi, bool flip)
{
#define QSIM_SEL(k) \
    case k: if constexpr (k < E) op_phase_sel<T, E, (k < E ? k : 0)>(x, fr, fi, flip); break;
    switch (sel) {
        QSIM_SEL(0) QSIM_SEL(1) QSIM_SEL(2) QSIM_SEL(3) QSIM_SEL(4) QSIM_SEL(5) QSIM_SEL(6) QSIM_SEL(7)
        QSIM_SEL(8) QSIM_SEL(9) QSIM_SEL(10) QSIM_SEL(11) QSIM_SEL(12) QSIM_SEL(13) QSIM_SEL(14) QSIM_SEL(15)
        QSIM_SEL(16) QSIM_SEL(17) QSIM_SEL(18) QSIM_SEL(19) QSIM_SEL(20) QSIM_SEL(21) QSIM_SEL(22) QSIM_SEL(23)
        QSIM_SEL(24) QSIM_SEL(25) QSIM_SEL(26) QSIM_SEL(27) QSIM_SEL(28) QSIM_SEL(29) QSIM_SEL(30) QSIM_SEL(31)
    default: break;
    }
#undef QSIM_SEL
}

template <typename T, int E, int RB>
__device__ __forceinline__ void op_xswap(typename Vec<T>::C *x, const uint32_t *er, uint32_t lcm_r, bool lane_ok)
{
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((r >> RB) & 1) continue;
        if ((er[r] & lcm_r) != lcm_r) continue;  // uniform
        const int r1 = r | (1 << RB);
        const auto a = x[r], b = x[r1];
        x[r].x = lane_ok ? b.x : a.x;
        x[r].y = lane_ok ? b.y : a.y;
        x[r1].x = lane_ok ? a.x : b.x;
        x[r1].y = lane_ok ? a.y : b.y;
    }
}

template <typename T, int LOG_E, int LOG_T, int MINW>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_staged(T *__restrict__ a, const SPass *__restrict__ passp,
                                                       const SStage *__restrict__ stages, const SOp *__restrict__ ops)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    constexpr int NT = 1 << LOG_T;
    constexpr int M = LOG_E + LOG_T;
    constexpr int NS = lds_slots<T>(M);
    __shared__ C lds[NS];

    const SPass pass = *passp;
    const int t = threadIdx.x;
    // block base: insert a zero bit at every resident position (uniform)
    uint64_t base = blockIdx.x;
#pragma unroll
    for (int s = 0; s < M; ++s) {
        const int p = pass.R[s];
        const uint64_t lo = base & ((uint64_t(1) << p) - 1);
        base = lo | ((base ^ lo) << 1);
    }
    // global index of local index k * NT + t = base | dep(t) | dep(k << LOG_T): the lane part is
    // computed once, the k part is uniform
    uint64_t dt = 0;
#pragma unroll
    for (int s = 0; s < LOG_T; ++s)
        if ((t >> s) & 1) dt |= uint64_t(1) << pass.R[s];
    const C *ag = reinterpret_cast<const C *>(a) + (base | dt);
    C *agw = reinterpret_cast<C *>(a) + (base | dt);
    auto dk = [&](int k) {  // uniform
        uint64_t v = 0;
#pragma unroll
        for (int j = 0; j < LOG_E; ++j)
            if ((k >> j) & 1) v |= uint64_t(1) << pass.R[LOG_T + j];
        return v;
    };
    // load: consecutive threads take consecutive local indices (contiguous runs in memory)
    {
        C v[E];
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = ld_nt(ag + dk(k));
#pragma unroll
        for (int k = 0; k < E; ++k) lds[slot<T>(k * NT + t)] = v[k];
    }
    __syncthreads();

    for (int si = pass.stage_begin; si < pass.stage_end; ++si) {
        const SStage st = stages[si];
        uint32_t rbm = 0;
#pragma unroll
        for (int j = 0; j < LOG_E; ++j) rbm |= 1u << st.rb[j];
        // thread bits: the local bits that are not register bits, in ascending order
        uint32_t et = 0;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j) et |= uint32_t((t >> j) & 1) << st.tbits[j];
        uint32_t er[E];
#pragma unroll
        for (int r = 0; r < E; ++r) {
            uint32_t v = 0;
#pragma unroll
            for (int j = 0; j < LOG_E; ++j)
                if ((r >> j) & 1) v |= 1u << st.rb[j];
            er[r] = v;
        }
        const int ls = slot<T>(et);
        C x[E];
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = lds[ls + slot<T>(er[r])];
        for (int oi = st.op_begin; oi < st.op_end; ++oi) {
            const SOp op = ops[oi];  // one wide scalar load of the whole record
            if ((base & op.gcm) != op.gcm) continue;  // a control outside R is 0 in this block
            const uint32_t lcm_r = op.lcm & rbm;
            const bool lane_ok = (et & op.lcm_t) == op.lcm_t;
            switch (op.type) {
            case 0: {
                U2<T> u;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool dg = (k == 0 || k == 3);
                    u.r[k] = lane_ok ? T(op.m[2 * k]) : (dg ? T(1) : T(0));
                    u.i[k] = lane_ok ? T(op.m[2 * k + 1]) : T(0);
                }
                if (op.rsel == 0) {
                    switch (op.rbit) {
                    case 0: op_dense_all<T, E, 0>(x, u); break;
                    case 1: op_dense_all<T, E, 1>(x, u); break;
                    case 2: op_dense_all<T, E, 2>(x, u); break;
                    case 3: op_dense_all<T, E, 3>(x, u); break;
                    default: if constexpr (LOG_E > 4) op_dense_all<T, E, (LOG_E > 4 ? 4 : 0)>(x, u); break;
                    }
                    break;
                }
                switch (op.rbit) {
                case 0: op_dense<T, E, 0>(x, er, lcm_r, u); break;
                case 1: op_dense<T, E, 1>(x, er, lcm_r, u); break;
                case 2: op_dense<T, E, 2>(x, er, lcm_r, u); break;
                case 3: op_dense<T, E, 3>(x, er, lcm_r, u); break;
                default: if constexpr (LOG_E > 4) op_dense<T, E, (LOG_E > 4 ? 4 : 0)>(x, er, lcm_r, u); break;
                }
                break;
            }
            case 2: {
                const bool flip = op.m[1] == 0.0 && op.m[0] == -1.0;  // Z, CZ: multiply by -1, exact
                const T fr = lane_ok ? T(op.m[0]) : T(1), fi = lane_ok ? T(op.m[1]) : T(0);
                phase_dispatch<T, E>(int(op.rsel), x, fr, fi, flip);
                break;
            }
            case 3: {
                // diag(d0, d1): elements with target bit 0 get d0, with 1 get d1 (conditions as above)
                T f0r = T(op.m[0]), f0i = T(op.m[1]), f1r = T(op.m[2]), f1i = T(op.m[3]);
                if (op.rbit < 0) {  // target on a thread bit or outside R: one factor per lane
                    const bool one = op.lt >= 0 ? ((et >> op.lt) & 1) != 0 : (base & op.gtb) != 0;
                    const T fr = lane_ok ? (one ? f1r : f0r) : T(1), fi = lane_ok ? (one ? f1i : f0i) : T(0);
                    phase_dispatch<T, E>(int(op.rsel), x, fr, fi, false);
                } else {  // target on register bit j: two selections
                    if (!lane_ok) {
                        f0r = f1r = T(1);
                        f0i = f1i = T(0);
                    }
                    const int j = op.rbit;
#pragma unroll
                    for (int r = 0; r < E; ++r)
                        if ((er[r] & lcm_r) == lcm_r) {
                            const bool one = (r >> j) & 1;
                            cmul<T>(x[r], one ? f1r : f0r, one ? f1i : f0i);
                        }
                }
                break;
            }
            default: break;
            }
        }
        __syncthreads();  // every thread has read this stage's inputs before anyone overwrites LDS
        if (st.swap_p >= 0 && (base & st.swap_gcm) == st.swap_gcm) {
            // stage-end quantum swap of two resident qubits: a permutation of the LDS slots
#pragma unroll
            for (int r = 0; r < E; ++r) {
                uint32_t d = et | er[r];
                if ((d & st.swap_lcm) == st.swap_lcm) {
                    const uint32_t bp = (d >> st.swap_p) & 1, bq = (d >> st.swap_q) & 1;
                    if (bp != bq) d ^= (1u << st.swap_p) | (1u << st.swap_q);
                }
                lds[slot<T>(d)] = x[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) lds[ls + slot<T>(er[r])] = x[r];
        }
        __syncthreads();
    }
    // store: the same contiguous order as the load
    {
        C v[E];
#pragma unroll
        for (int k = 0; k < E; ++k) v[k] = lds[slot<T>(k * NT + t)];
#pragma unroll
        for (int k = 0; k < E; ++k) st_nt(agw + dk(k), v[k]);
    }
}

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

}  // namespace

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
static bool staged_variant_ok(int dtype, int log_e, int log_t)
{
    if (log_t < 6 || log_t > 9) return false;
    if (dtype == QSIM_C128) return (log_e == 3 && log_t >= 7) || (log_e == 4 && log_t <= 8);
    return (log_e == 4 && log_t >= 7) || (log_e == 5 && log_t <= 8);
}

int staged_build(int n, int dtype, const std::vector<qsim_gate> &gates, int lds_qubits, int lds_regs, StagedPlan **out,
                 qsim_plan_info *info)
{
    *out = nullptr;
    // defaults measured on the 30-qubit brickwork: 4096 amplitudes per block, 16 per thread
    const int log_e = lds_regs ? lds_regs : 4;
    const int L = dtype == QSIM_C128 ? 4 : 5;  // low run: 2^L amplitudes = 256 bytes
    int m = lds_qubits ? lds_qubits : 12;
    if (!staged_variant_ok(dtype, log_e, m - log_e))
        return set_error(QSIM_EINVAL, "staged: lds_qubits / lds_regs combination not available for this dtype");
    if (n < m) return set_error(QSIM_EUNSUPPORTED, "staged: the state is smaller than one LDS block");
    const int log_t = m - log_e;

    const size_t G = gates.size();
    std::vector<GInfo> gi(G);
    for (size_t i = 0; i < G; ++i) gi[i] = describe(gates[i]);
    std::vector<char> done(G, 0);
    size_t ndone = 0;

    std::vector<SPass> passes;
    std::vector<SStage> stages;
    std::vector<SOp> ops;

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
                o.fast = (o.type == 0 && o.lcm == 0) ? 1 : 0;
            }
            for (size_t oi = size_t(cur.op_begin); oi < ops.size();) {
                size_t oe = oi + 1;
                while (oe < ops.size() && ops[oe].fast == ops[oi].fast) ++oe;
                ops[oi].run = int32_t(oe - oi);
                oi = oe;
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
