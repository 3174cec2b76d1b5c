// Device side of the LDS-staged passes: records shared by the scheduler and the kernels, the
// register-bit operations and the block processor (used by the per-pass kernel and by the
// persistent batch kernel).
#pragma once

#include "qsim_internal.h"

namespace qsim {
namespace staged {

constexpr int kMaxM = 14;

struct SOp {
    int32_t type;      // 0 dense 2x2, 1 X (swap pairs), 2 conditional phase, 3 diag(d0, d1)
    int32_t rbit;      // dense / X: register-bit index of the target; diag: register-bit index of
                       // the target if it is a register bit, else -1
    int32_t lt;        // diag: local bit of the target, or -1 if the target is outside R
    uint32_t lcm;      // local condition mask (local index bits that must be 1)
    uint32_t rsel;     // the part of lcm on register bits, as a mask over the register index r
    uint32_t lcm_t;    // the part of lcm on thread bits (local bit positions)
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
template <typename T> __host__ __device__ constexpr int lds_slots(int m) { return (1 << m) + ((1 << m) >> (sizeof(T) == 8 ? 4 : 5)); }

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

// Process block `blk` of a pass: load it (or generate |0...0> when init_zero is set), run the
// stages, store it. Called by every thread of a workgroup of 2^LOG_T threads; `lds` holds
// lds_slots<T>(LOG_E + LOG_T) amplitudes.
template <typename T, int LOG_E, int LOG_T>
__device__ __forceinline__ void run_block(T *__restrict__ a, const SPass &pass, uint64_t blk, const SStage *__restrict__ stages,
                                          const SOp *__restrict__ ops, typename Vec<T>::C *lds, bool init_zero)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    constexpr int NT = 1 << LOG_T;
    constexpr int M = LOG_E + LOG_T;
    const int t = threadIdx.x;
    // block base: insert a zero bit at every resident position (uniform)
    uint64_t base = blk;
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
    if (init_zero) {
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const bool one = base == 0 && k == 0 && t == 0;
            lds[slot<T>(k * NT + t)] = C{one ? T(1) : T(0), T(0)};
        }
    } else {
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
    // a caller that runs the next block in this workgroup overwrites LDS: every thread must have
    // read its last values first
    __syncthreads();
}


// host: append the schedule of one circuit (see staged.hip)
int staged_schedule(int n, int dtype, int m, int log_e, const std::vector<qsim_gate> &gates, std::vector<SPass> &passes,
                    std::vector<SStage> &stages, std::vector<SOp> &ops);
bool staged_variant_ok(int dtype, int log_e, int log_t);
__global__ void k_op_angles(SOp *ops, int nops);

}  // namespace staged
}  // namespace qsim
