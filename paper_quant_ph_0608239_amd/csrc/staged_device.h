// Device side of the LDS-staged passes: records shared by the scheduler and the kernels, the
// register-bit operations and the block processor (used by the per-pass kernel and by the
// persistent batch kernel).
#pragma once

#include "qsim_internal.h"

namespace qsim {
namespace staged {

constexpr int kMaxM = 14;
constexpr int kMaxLogE = 5;
constexpr int kMaxLogT = 10;  // threads per workgroup: at most 2^10

// One operation of a stage. Dense ops act on one register bit (the list they sit in says which);
// diagonal ops multiply register elements by per-lane factors.
struct SOp {
    uint32_t pmask;    // dense: pairs p of the register bit that the register part of the condition admits
    uint32_t lcm_t;    // condition on thread bits: local bit positions that must be 1
    uint64_t gcm;      // condition on non-resident index bits (must all be 1)
    uint64_t gtb;      // diag: the target's index bit when the target is not resident, else 0
    uint32_t m0, m1;   // diag: register elements r that take factor d0 / d1
    int32_t lt;        // diag: local bit of the target when it is a thread bit, else -1
    int32_t angles;    // 0: m[] given; 1: d0 = 1, d1 = e^{i theta0}; 2: d0 = e^{i theta0}, d1 = e^{i theta1};
                       // 3: d0 = 1, d1 = e^{i theta0 2 pi / 2^theta1} (theta0 = +-1, theta1 = k)
    double m[8];       // dense: 2x2 row-major (re, im); diag: d0 = m[0..1], d1 = m[2..3]
    double theta[2];   // angle inputs of the angles != 0 forms
    float mf[8];       // m rounded to FP32 (complex64 kernels), filled on the device
    // dense: a sign flip fused into the op (Z on the target, conditioned on one other qubit). Where
    // the condition holds (pairs in amask, lanes meeting alt_lcm, blocks meeting galt), the op
    // applies its 2x2 with row 1 negated (the flip follows the op) or, with alt_col, column 1
    // negated (the flip precedes it)
    uint64_t galt;
    uint32_t amask;
    uint32_t alt_lcm;
    uint32_t alt_col;
    int32_t alt_rank;  // flip chosen per pair: the rank of the other qubit's register bit, else -1
};

// A round of a stage. For register bit j, eight lists of dense ops [seg[8j + l], seg[8j + l + 1]): l = 0
// without condition; l = 1 with a sign flip fused per block; l = 2 + i with a flip fused per pair, by
// the i-th other register bit (i < LOG_E - 1); l = 6 with a flip fused per lane; l = 7 with a
// condition. The first seven hold 2x2s with a real first column only. Then the sign flips (diagonal
// ops whose only factor is -1) [seg[8 LOG_E], seg[8 LOG_E + 1]) and the other diagonal ops
// [seg[8 LOG_E + 1], seg[8 LOG_E + 2]). Dense ops of one round on different bits commute, diagonal ops
// commute with each other, and every diagonal op of the round runs after its dense ops, so this order
// equals circuit order.
constexpr int kLists = 8;
constexpr int kListBlockFlip = 1, kListPairFlip = 2, kListLaneFlip = 6, kListCond = 7;
// After the register-bit lists, a round runs one list of two-qubit blocks per pair of register bits
// (ja < jb, numbered ja-major: (0,1), (0,2), ..., (1,2), ...): [pseg[p], pseg[p + 1]) in the block
// table. Then come the sign flips and the other diagonal ops of the op table.
constexpr int kMaxPairs = kMaxLogE * (kMaxLogE - 1) / 2;
constexpr int npairs(int log_e) { return log_e * (log_e - 1) / 2; }
constexpr int pair_index(int log_e, int ja, int jb) { return ja * (2 * log_e - ja - 1) / 2 + (jb - ja - 1); }
struct SRound {
    int32_t seg[kLists * kMaxLogE + 4];
    int32_t pseg[kMaxPairs + 1];
};

// A two-qubit block: a run of a stage's ops that act only on two register bits ja < jb, multiplied into
// one 4x4 unitary (row-major complex, index p = bit ja + 2 bit jb) applied to each group of four
// register elements. A 4x4 costs 16 multiply-adds per amplitude where the four or more single-qubit
// 2x2s it replaces cost 6 each.
struct SBlk {
    double m[32];
    float mf[32];  // m rounded to FP32 (complex64 kernels), filled by the scheduler
};

struct SStage {
    int32_t round_begin, round_end;
    uint8_t rb[8];                // register bits (local bit indices), LOG_E of them, ascending
    uint8_t tbits[kMaxLogT + 6];  // thread bits (the other local bits), LOG_T of them, lowest lane first
    int32_t swap_p;               // stage-end local swap (quantum swap of two resident qubits), -1 if none
    int32_t swap_q;
    uint32_t swap_lcm;            // its local condition
    // half-buffer passes: the LDS round trip into this stage (from the previous stage, or from the
    // load layout) and the one out of it (to the next stage, or to the store layout) each run in two
    // halves split by local bit hb_* at thread position hj_* of both layouts
    uint8_t hb_in, hj_in, hb_out, hj_out;
    uint64_t swap_gcm;            // its condition on non-resident bits
    uint8_t prb[8];               // index bit (physical qubit) of each register bit
    uint8_t ptb[kMaxLogT + 6];    // index bit of each thread bit, lowest lane first
};
static_assert(sizeof(SStage) == 80, "stage record layout");

struct SPass {
    int32_t m;
    int32_t stage_begin, stage_end;
    int32_t direct;     // bit 0: the first stage loads its registers straight from memory; bit 1: the
                        // last stage stores them straight to memory (no LDS round trip). Set when the
                        // stage's register bits avoid the low run, so that its thread bits keep
                        // consecutive lanes on consecutive amplitudes. Bit 2: every LDS round trip of
                        // the pass has a split bit, and it runs with a half-size LDS buffer. Bit 3: all
                        // those split bits sit at wave positions (whole wavefronts per half)
    uint8_t R[16];      // physical bit of local bit s, ascending
};

// Plan tables are read-only while a pass runs: they are read through constant-address-space
// pointers, so wave-uniform reads of them become scalar loads whatever the kernel stores elsewhere.
template <typename T> using cptr = const T __attribute__((address_space(4))) *;
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }
// copy of a table record (word by word, so the compiler can merge the reads into wide scalar loads)
template <typename S> __device__ __forceinline__ S ldc(cptr<S> p)
{
    static_assert(sizeof(S) % 4 == 0, "records are whole words");
    S v;
    uint32_t *d = reinterpret_cast<uint32_t *>(&v);
    const cptr<uint32_t> w = (cptr<uint32_t>)p;
#pragma unroll
    for (int i = 0; i < int(sizeof(S) / 4); ++i) d[i] = w[i];
    return v;
}

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
// amplitudes, i.e. one per 256 bytes). Additive over index parts without common bits:
// slot(a | b) = slot(a) + slot(b).
template <typename T> __device__ __forceinline__ int slot(int e) { return sizeof(T) == 8 ? e + (e >> 4) : e + (e >> 5); }
template <typename T> __host__ __device__ constexpr int lds_slots(int m) { return (1 << m) + ((1 << m) >> (sizeof(T) == 8 ? 4 : 5)); }

// In-place complex updates. Every output is an accumulation chain whose last step consumes one input
// that no other chain still needs; that step writes its result into the input's own register
// (fma_into). The amplitudes then stay in fixed registers across the op loops, and the compiler
// has no reason to copy the register array between ops. S: the coefficient is wave-uniform and
// may sit in a scalar register.
template <bool S> __device__ __forceinline__ void fma_into(double &x, double c, double t)
{
    if constexpr (S) asm("v_fma_f64 %0, %1, %0, %2" : "+v"(x) : "s"(c), "v"(t));
    else asm("v_fma_f64 %0, %1, %0, %2" : "+v"(x) : "v"(c), "v"(t));
}
template <bool S> __device__ __forceinline__ void fma_into(float &x, float c, float t)
{
    if constexpr (S) asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x) : "s"(c), "v"(t));
    else asm("v_fma_f32 %0, %1, %0, %2" : "+v"(x) : "v"(c), "v"(t));
}

// fused multiply-add in the type's own precision (__builtin_fma is the double one)
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// x <- (fr + i fi) x
template <typename T>
__device__ __forceinline__ void cmul(typename Vec<T>::C &x, T fr, T fi)
{
    const T ti = fi * x.x;
    const T tr = -(fi * x.y);
    fma_into<false>(x.x, fr, tr);
    fma_into<false>(x.y, fr, ti);
}

template <typename T> struct U2 {
    T r[4], i[4];
};

// (a, b) <- (u00 a + u01 b, u10 a + u11 b), in place
template <typename T, bool S>
__device__ __forceinline__ void pair2x2(typename Vec<T>::C &a, typename Vec<T>::C &b, const U2<T> &u)
{
    T t0 = u.r[1] * b.x;
    T t1 = u.i[0] * a.x;
    T t2 = u.r[2] * a.x;
    T t3 = u.r[2] * a.y;
    t0 = fmat(-u.i[1], b.y, t0);
    t1 = fmat(u.r[1], b.y, t1);
    t2 = fmat(-u.i[2], a.y, t2);
    t3 = fmat(u.i[2], a.x, t3);
    t0 = fmat(-u.i[0], a.y, t0);
    t1 = fmat(u.i[1], b.x, t1);
    t2 = fmat(-u.i[3], b.y, t2);
    t3 = fmat(u.i[3], b.x, t3);
    fma_into<S>(a.x, u.r[0], t0);
    fma_into<S>(a.y, u.r[0], t1);
    fma_into<S>(b.x, u.r[3], t2);
    fma_into<S>(b.y, u.r[3], t3);
}

// The same for a 2x2 whose first column is real (u00 and u10 have no imaginary part; u.i[0] and
// u.i[2] are not read): 12 multiply-adds instead of 16.
template <typename T, bool S>
__device__ __forceinline__ void pair2x2_rc(typename Vec<T>::C &a, typename Vec<T>::C &b, const U2<T> &u)
{
    T s2 = u.r[2] * a.x;
    T s3 = u.r[2] * a.y;
    T s0 = u.r[1] * b.x;
    T s1 = u.r[1] * b.y;
    s2 = fmat(-u.i[3], b.y, s2);
    s3 = fmat(u.i[3], b.x, s3);
    s0 = fmat(-u.i[1], b.y, s0);
    s1 = fmat(u.i[1], b.x, s1);
    fma_into<S>(a.x, u.r[0], s0);
    fma_into<S>(a.y, u.r[0], s1);
    fma_into<S>(b.x, u.r[3], s2);
    fma_into<S>(b.y, u.r[3], s3);
}

template <typename T> __device__ __forceinline__ const T *coef(const SOp &op);
template <> __device__ __forceinline__ const double *coef<double>(const SOp &op) { return op.m; }
template <> __device__ __forceinline__ const float *coef<float>(const SOp &op) { return op.mf; }

// A dense op with no condition on register bit RB: every pair, wave-uniform coefficients.
template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense_all(typename Vec<T>::C *x, const SOp &op)
{
    const T *c = coef<T>(op);
    U2<T> u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u.r[k] = c[2 * k];
        u.i[k] = c[2 * k + 1];
    }
#pragma unroll
    for (int r = 0; r < E; ++r)
        if (!((r >> RB) & 1)) pair2x2_rc<T, true>(x[r], x[r | (1 << RB)], u);
}

// sign toggle by an integer xor of the sign bit (exact); t is 0 or 0x80000000
__device__ __forceinline__ void xor_sign(double &v, uint32_t t)
{
    uint2 w = __builtin_bit_cast(uint2, v);
    w.y ^= t;
    v = __builtin_bit_cast(double, w);
}
__device__ __forceinline__ void xor_sign(float &v, uint32_t t) { v = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ t); }

// Dense ops with a fused flip chosen per pair (register bits) or per block: in the pairs that take it,
// the second amplitude changes sign before the 2x2 (column flip) or after it (row flip). Those pairs
// use the 2x2 with column 1 or row 1 negated instead, which gives the same bits as negating the data
// (rounding is sign-symmetric). Per block, the coefficient set is chosen once per op; per pair, the
// pairs that flip are those with register bit K set, and each list holds one K, so every pair's set
// is fixed at compile time. Either way the op costs the same FMAs as an unconditional one.
template <typename T>
__device__ __forceinline__ void flip_coefs(const SOp &op, U2<T> &u, U2<T> &v)
{
    const T *c = coef<T>(op);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u.r[k] = c[2 * k];
        u.i[k] = c[2 * k + 1];
    }
    const bool col = op.alt_col != 0;
    v = u;
    v.r[1] = col ? -u.r[1] : u.r[1];
    v.i[1] = col ? -u.i[1] : u.i[1];
    v.r[2] = col ? u.r[2] : -u.r[2];
    v.r[3] = -u.r[3];
    v.i[3] = -u.i[3];
}
template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense_flip_block(typename Vec<T>::C *x, const SOp &op, uint64_t base)
{
    U2<T> u, v, w;
    flip_coefs<T>(op, u, v);
    const bool neg = (base & op.galt) == op.galt;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w.r[q] = neg ? v.r[q] : u.r[q];
        w.i[q] = neg ? v.i[q] : u.i[q];
    }
#pragma unroll
    for (int r = 0; r < E; ++r)
        if (!((r >> RB) & 1)) pair2x2_rc<T, true>(x[r], x[r | (1 << RB)], w);
}
template <typename T, int E, int RB, int K>
__device__ __forceinline__ void op_dense_flip_pair(typename Vec<T>::C *x, const SOp &op)
{
    U2<T> u, v;
    flip_coefs<T>(op, u, v);
#pragma unroll
    for (int r = 0; r < E; ++r)
        if (!((r >> RB) & 1)) pair2x2_rc<T, true>(x[r], x[r | (1 << RB)], ((r >> K) & 1) ? v : u);
}

// A dense op with a fused flip chosen per lane (a thread bit): every pair of the lanes that take it
// uses the 2x2 with row 1 (or column 1) negated. (A sign xor of the data instead needs the flip on
// one side of the 2x2 or the other; a branch on that side made the compiler copy the amplitudes.)
// the coefficient with its sign bit xor-ed with t (0 or the sign bit): an exact negation where t is set
__device__ __forceinline__ double xsign(double c, uint32_t t)
{
    uint2 w = __builtin_bit_cast(uint2, c);
    w.y ^= t;
    return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ float xsign(float c, uint32_t t) { return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, c) ^ t); }

// c where keep is all ones, 0 where it is 0 (bitwise: exact)
__device__ __forceinline__ double bmask(double c, uint32_t keep)
{
    uint2 w = __builtin_bit_cast(uint2, c);
    w.x &= keep;
    w.y &= keep;
    return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ float bmask(float c, uint32_t keep) { return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, c) & keep); }
// c where keep is all ones, 1 where it is 0 (bitwise: exact)
__device__ __forceinline__ double bsel_one(double c, uint32_t keep)
{
    uint2 w = __builtin_bit_cast(uint2, c);
    w.x &= keep;
    w.y = (w.y & keep) | (0x3ff00000u & ~keep);
    return __builtin_bit_cast(double, w);
}
__device__ __forceinline__ float bsel_one(float c, uint32_t keep)
{
    return __builtin_bit_cast(float, (__builtin_bit_cast(uint32_t, c) & keep) | (0x3f800000u & ~keep));
}

template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense_alt_lane(typename Vec<T>::C *x, const SOp &op, uint32_t et, uint64_t base)
{
    const T *c = coef<T>(op);
    // the lane's sign mask, applied to column 1 (column flip) or row 1 (row flip) and to u11
    const uint32_t t = ((base & op.galt) == op.galt && (et & op.alt_lcm) == op.alt_lcm) ? 0x80000000u : 0u;
    const uint32_t col = op.alt_col ? ~0u : 0u;
    const uint32_t t1 = t & col, t2 = t & ~col;
    U2<T> w;
    w.r[0] = c[0];
    w.i[0] = c[1];
    w.r[1] = xsign(c[2], t1);
    w.i[1] = xsign(c[3], t1);
    w.r[2] = xsign(c[4], t2);
    w.i[2] = xsign(c[5], t2);
    w.r[3] = xsign(c[6], t);
    w.i[3] = xsign(c[7], t);
#pragma unroll
    for (int r = 0; r < E; ++r)
        if (!((r >> RB) & 1)) pair2x2_rc<T, false>(x[r], x[r | (1 << RB)], w);
}

// A dense op with a condition: lanes that fail its thread part keep the identity, pairs outside
// its register part (pmask, wave-uniform) are skipped.
template <typename T, int E, int RB>
__device__ __forceinline__ void op_dense_cond(typename Vec<T>::C *x, const SOp &op, bool lane_ok)
{
    const T *c = coef<T>(op);
    // lanes that fail the condition take the identity: the coefficients' bits are masked (off-diagonal
    // and imaginary parts to 0) and the diagonal's real parts bit-selected against 1
    const uint32_t keep = lane_ok ? ~0u : 0u;
    U2<T> u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool dg = (k == 0 || k == 3);
        u.r[k] = dg ? bsel_one(c[2 * k], keep) : bmask(c[2 * k], keep);
        u.i[k] = bmask(c[2 * k + 1], keep);
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((r >> RB) & 1) continue;
        const int p = (r & ((1 << RB) - 1)) | ((r >> (RB + 1)) << RB);
        if ((op.pmask >> p) & 1) pair2x2<T, false>(x[r], x[r | (1 << RB)], u);
    }
}

// A diagonal op: elements r in m1 take factor f1, those in m0 take f0; with a thread-bit or
// non-resident target, f1 is chosen per lane (or block) from d0 and d1.
template <typename T, int E>
__device__ __forceinline__ void op_diag(typename Vec<T>::C *x, const SOp &op, uint32_t et, uint64_t base)
{
    const T *c = coef<T>(op);
    const bool lane_ok = (et & op.lcm_t) == op.lcm_t;
    T f0r = c[0], f0i = c[1], f1r = c[2], f1i = c[3];
    if (op.lt >= 0 || op.gtb) {
        const bool one = op.lt >= 0 ? ((et >> op.lt) & 1) != 0 : (base & op.gtb) != 0;
        f1r = one ? f1r : f0r;
        f1i = one ? f1i : f0i;
    }
    f0r = lane_ok ? f0r : T(1);
    f0i = lane_ok ? f0i : T(0);
    f1r = lane_ok ? f1r : T(1);
    f1i = lane_ok ? f1i : T(0);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        if ((op.m1 >> r) & 1) cmul<T>(x[r], f1r, f1i);
        if ((op.m0 >> r) & 1) cmul<T>(x[r], f0r, f0i);
    }
}

// A sign flip: elements r in m1 change sign on lanes that meet the condition. The sign bit is
// toggled with an integer xor (exact, no rounding), the per-element choice is made in scalar
// registers, so the op runs without branches.
__device__ __forceinline__ void flip_sign(double &v, uint32_t t)
{
    uint2 h = __builtin_bit_cast(uint2, v);
    h.y ^= t;
    v = __builtin_bit_cast(double, h);
}
__device__ __forceinline__ void flip_sign(float &v, uint32_t t) { v = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) ^ t); }

template <typename T, int E>
__device__ __forceinline__ void op_flip(typename Vec<T>::C *x, const SOp &op, uint32_t et)
{
    const uint32_t lane_sign = (et & op.lcm_t) == op.lcm_t ? 0x80000000u : 0u;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const uint32_t t = ((op.m1 >> r) & 1) ? lane_sign : 0u;
        flip_sign(x[r].x, t);
        flip_sign(x[r].y, t);
    }
}

// the i-th register bit other than J
constexpr int other_bit(int J, int i) { return i < J ? i : i + 1; }

template <typename T> __device__ __forceinline__ const T *coefb(const SBlk &b);
template <> __device__ __forceinline__ const double *coefb<double>(const SBlk &b) { return b.m; }
template <> __device__ __forceinline__ const float *coefb<float>(const SBlk &b) { return b.mf; }

// A two-qubit block on register bits JA < JB, in place: for each group of four elements, every output
// is first summed over the three inputs other than its own (P_r), then its own input's term is added
// into that input's registers (the input is no longer needed by any other output). 16 multiply-adds
// per amplitude, no register copies; the 4x4 is wave-uniform.
template <typename T, int E, int JA, int JB>
__device__ __forceinline__ void op_pair(typename Vec<T>::C *x, const SBlk &b)
{
    const T *c = coefb<T>(b);
    T mr[16], mi[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        mr[k] = c[2 * k];
        mi[k] = c[2 * k + 1];
    }
#pragma unroll
    for (int g = 0; g < E / 4; ++g) {
        // element index of group g: g's bits with zeros inserted at JA and JB
        const int lo = g & ((1 << JA) - 1);
        const int mid = (g >> JA) & ((1 << (JB - JA - 1)) - 1);
        const int hi = g >> (JB - 1);
        const int r0 = lo | (mid << (JA + 1)) | (hi << (JB + 1));
        const int id[4] = {r0, r0 | (1 << JA), r0 | (1 << JB), r0 | (1 << JA) | (1 << JB)};
        T pr[4], pi[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bool first = true;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q == r) continue;
                const T ar = mr[4 * r + q], ai = mi[4 * r + q];
                const T xr = x[id[q]].x, xi = x[id[q]].y;
                if (first) {
                    pr[r] = ar * xr;
                    pi[r] = ar * xi;
                    pr[r] = fmat(-ai, xi, pr[r]);
                    pi[r] = fmat(ai, xr, pi[r]);
                    first = false;
                } else {
                    pr[r] = fmat(ar, xr, pr[r]);
                    pi[r] = fmat(ar, xi, pi[r]);
                    pr[r] = fmat(-ai, xi, pr[r]);
                    pi[r] = fmat(ai, xr, pi[r]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const T dr = mr[5 * r], di = mi[5 * r];
            typename Vec<T>::C &v = x[id[r]];
            const T sre = fmat(-di, v.y, pr[r]);
            const T sim = fmat(di, v.x, pi[r]);
            fma_into<true>(v.y, dr, sim);
            fma_into<true>(v.x, dr, sre);
        }
    }
}

// the pair list of register bits (JA, JB), if the stage has that pair
template <typename T, int E, int LOG_E, int JA, int JB>
__device__ __forceinline__ void pair_list(typename Vec<T>::C *x, const SRound &rd, cptr<SBlk> blks)
{
    if constexpr (JB < LOG_E) {
        constexpr int s = pair_index(LOG_E, JA, JB);
        for (int bi = rd.pseg[s]; bi < rd.pseg[s + 1]; ++bi) {
            const SBlk b = ldc<SBlk>(blks + bi);
            op_pair<T, E, JA, JB>(x, b);
        }
    }
}

// the per-pair flip list i of register bit J (flips by register bit other_bit(J, i))
template <typename T, int E, int J, int I>
__device__ __forceinline__ void pair_flip_list(typename Vec<T>::C *x, const SRound &rd, cptr<SOp> ops)
{
    if constexpr ((1 << (I + 1)) < E) {
        for (int oi = rd.seg[kLists * J + kListPairFlip + I]; oi < rd.seg[kLists * J + kListPairFlip + I + 1]; ++oi) {
            const SOp op = ldc<SOp>(ops + oi);
            op_dense_flip_pair<T, E, J, other_bit(J, I)>(x, op);
        }
    }
}

// the ops of one round on register bit J
template <typename T, int E, int J>
__device__ __forceinline__ void round_bit(typename Vec<T>::C *x, const SRound &rd, cptr<SOp> ops, uint32_t et,
                                          uint64_t base)
{
    // one test skips all lists of a bit without dense ops in this round, one more the flip lists
    if (rd.seg[kLists * J] == rd.seg[kLists * J + kLists]) return;
    for (int oi = rd.seg[kLists * J]; oi < rd.seg[kLists * J + 1]; ++oi) {
        const SOp op = ldc<SOp>(ops + oi);
        op_dense_all<T, E, J>(x, op);
    }
    if (rd.seg[kLists * J + kListBlockFlip] != rd.seg[kLists * J + kListLaneFlip]) {
        for (int oi = rd.seg[kLists * J + kListBlockFlip]; oi < rd.seg[kLists * J + kListBlockFlip + 1]; ++oi) {
            const SOp op = ldc<SOp>(ops + oi);
            op_dense_flip_block<T, E, J>(x, op, base);
        }
        pair_flip_list<T, E, J, 0>(x, rd, ops);
        pair_flip_list<T, E, J, 1>(x, rd, ops);
        pair_flip_list<T, E, J, 2>(x, rd, ops);
        pair_flip_list<T, E, J, 3>(x, rd, ops);
    }
    for (int oi = rd.seg[kLists * J + kListLaneFlip]; oi < rd.seg[kLists * J + kListLaneFlip + 1]; ++oi) {
        const SOp op = ldc<SOp>(ops + oi);
        op_dense_alt_lane<T, E, J>(x, op, et, base);
    }
    for (int oi = rd.seg[kLists * J + kListCond]; oi < rd.seg[kLists * J + kListCond + 1]; ++oi) {
        const SOp op = ldc<SOp>(ops + oi);
        if ((base & op.gcm) != op.gcm) continue;  // a control outside R is 0 in this block
        op_dense_cond<T, E, J>(x, op, (et & op.lcm_t) == op.lcm_t);
    }
}

// all rounds of a stage on the registers x (in the stage's layout; et: the thread's local index part)
template <typename T, int LOG_E>
__device__ __forceinline__ void run_rounds(typename Vec<T>::C *x, const SStage &st, cptr<SRound> rounds, cptr<SOp> ops,
                                           cptr<SBlk> blks, uint32_t et, uint64_t base)
{
    constexpr int E = 1 << LOG_E;
    for (int ri = st.round_begin; ri < st.round_end; ++ri) {
        const SRound rd = ldc<SRound>(rounds + ri);
        round_bit<T, E, 0>(x, rd, ops, et, base);
        round_bit<T, E, 1>(x, rd, ops, et, base);
        round_bit<T, E, 2>(x, rd, ops, et, base);
        if constexpr (LOG_E > 3) round_bit<T, E, (LOG_E > 3 ? 3 : 0)>(x, rd, ops, et, base);
        if constexpr (LOG_E > 4) round_bit<T, E, (LOG_E > 4 ? 4 : 0)>(x, rd, ops, et, base);
        // the two-qubit blocks: one test skips all pair lists of a round without blocks
        if (rd.pseg[0] != rd.pseg[npairs(LOG_E)]) {
            pair_list<T, E, LOG_E, 0, 1>(x, rd, blks);
            pair_list<T, E, LOG_E, 0, 2>(x, rd, blks);
            pair_list<T, E, LOG_E, 0, 3>(x, rd, blks);
            pair_list<T, E, LOG_E, 0, 4>(x, rd, blks);
            pair_list<T, E, LOG_E, 1, 2>(x, rd, blks);
            pair_list<T, E, LOG_E, 1, 3>(x, rd, blks);
            pair_list<T, E, LOG_E, 1, 4>(x, rd, blks);
            pair_list<T, E, LOG_E, 2, 3>(x, rd, blks);
            pair_list<T, E, LOG_E, 2, 4>(x, rd, blks);
            pair_list<T, E, LOG_E, 3, 4>(x, rd, blks);
        }
        for (int oi = rd.seg[kLists * LOG_E]; oi < rd.seg[kLists * LOG_E + 1]; ++oi) {
            const SOp op = ldc<SOp>(ops + oi);
            if ((base & op.gcm) != op.gcm) continue;
            op_flip<T, E>(x, op, et);
        }
        for (int oi = rd.seg[kLists * LOG_E + 1]; oi < rd.seg[kLists * LOG_E + 2]; ++oi) {
            const SOp op = ldc<SOp>(ops + oi);
            if ((base & op.gcm) != op.gcm) continue;
            op_diag<T, E>(x, op, et, base);
        }
    }
}

// Renormalisation folded into a pass (Eq. STAT1). `scale` (NULL: none) points at the FP64 squared
// norm that the previous pass left: every amplitude the pass loads is multiplied by 1/sqrt of it (by 1
// when it is not positive), exactly as a separate rescaling sweep would. `norm` (NULL: none) receives one
// FP64 partial sum of |a|^2 per block, over the amplitudes the pass stores; the partials are summed
// afterwards in a fixed order.
// The block runners take it only when instantiated with EDGE = true, so the passes that need neither
// are compiled without it.
struct SEdge {
    const double *scale;
    double *norm;
};

template <typename T, int E>
__device__ __forceinline__ void edge_scale(typename Vec<T>::C *x, const double *scale)
{
    const double s = *scale;
    const T f = static_cast<T>(s > 0.0 ? 1.0 / sqrt(s) : 1.0);
#pragma unroll
    for (int r = 0; r < E; ++r) {
        x[r].x *= f;
        x[r].y *= f;
    }
}

template <typename T, int E>
__device__ __forceinline__ double sq_sum(const typename Vec<T>::C *x)
{
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < E; ++r) {
        const double re = double(x[r].x), im = double(x[r].y);
        acc += re * re + im * im;
    }
    return acc;
}

// One partial sum per block: a butterfly over each wavefront, then the wavefronts' sums in order.
// Called by every thread of the workgroup after its last LDS access of the block; leaves LDS free.
__device__ __forceinline__ void edge_norm_out(double acc, double *norm, uint64_t blk, void *lds)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o);
    double *w = static_cast<double *>(lds);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (unsigned i = 0; i < blockDim.x / 64; ++i) s += w[i];
        norm[blk] = s;
    }
    __syncthreads();
}

// Addressing of a block: block `blk` of a pass holds the 2^M amplitudes whose index bits outside the
// resident set R equal the bits of blk. In the load/store layout, thread t and element k hold local
// index k * NT + t, so consecutive threads take consecutive local indices (contiguous runs).
template <int M>
__device__ __forceinline__ uint64_t block_base(const SPass &pass, uint64_t blk)
{
    uint64_t base = blk;  // insert a zero bit at every resident position (uniform)
#pragma unroll
    for (int s = 0; s < M; ++s) {
        const int p = pass.R[s];
        const uint64_t lo = base & ((uint64_t(1) << p) - 1);
        base = lo | ((base ^ lo) << 1);
    }
    return base;
}
template <int LOG_T>
__device__ __forceinline__ uint64_t lane_part(const SPass &pass, int t)
{
    uint64_t dt = 0;
#pragma unroll
    for (int s = 0; s < LOG_T; ++s)
        if ((t >> s) & 1) dt |= uint64_t(1) << pass.R[s];
    return dt;
}
template <int LOG_E, int LOG_T>
__device__ __forceinline__ uint64_t elem_part(const SPass &pass, int k)  // uniform
{
    uint64_t v = 0;
#pragma unroll
    for (int j = 0; j < LOG_E; ++j)
        if ((k >> j) & 1) v |= uint64_t(1) << pass.R[LOG_T + j];
    return v;
}

template <typename T, int LOG_E, int LOG_T>
__device__ __forceinline__ void load_block(const T *__restrict__ a, const SPass &pass, uint64_t base, uint64_t dt,
                                           typename Vec<T>::C *v)
{
    using C = typename Vec<T>::C;
    const C *ag = reinterpret_cast<const C *>(a) + (base | dt);
#pragma unroll
    for (int k = 0; k < (1 << LOG_E); ++k) v[k] = ld_nt(ag + elem_part<LOG_E, LOG_T>(pass, k));
}

template <typename T, int LOG_E, int LOG_T>
__device__ __forceinline__ void regs_to_lds(const typename Vec<T>::C *v, typename Vec<T>::C *lds)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < (1 << LOG_E); ++k) lds[slot<T>(k * (1 << LOG_T) + t)] = v[k];
}

template <typename T, int LOG_E, int LOG_T>
__device__ __forceinline__ double store_block(T *__restrict__ a, const SPass &pass, uint64_t base, uint64_t dt,
                                              const typename Vec<T>::C *lds, bool want_norm)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    const int t = threadIdx.x;
    C *agw = reinterpret_cast<C *>(a) + (base | dt);
    C v[E];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = lds[slot<T>(k * (1 << LOG_T) + t)];
#pragma unroll
    for (int k = 0; k < E; ++k) st_nt(agw + elem_part<LOG_E, LOG_T>(pass, k), v[k]);
    return want_norm ? sq_sum<T, E>(v) : 0.0;
}

// Run the stages of a pass on the block held in LDS (load/store layout in, load/store layout out).
// Every stage reads the block into registers in its own layout, applies its rounds, and writes it
// back (permuted by the stage-end quantum swap, if any).
template <typename T, int LOG_E, int LOG_T, bool EDGE = false>
__device__ __forceinline__ void run_stages(T *__restrict__ a, const SPass &pass, uint64_t base, cptr<SStage> stages,
                                           cptr<SRound> rounds, cptr<SOp> ops, cptr<SBlk> blks,
                                           typename Vec<T>::C *lds, bool init_zero, SEdge edge, double &nacc)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    const int t = threadIdx.x;
    C x[E];
    for (int si = pass.stage_begin; si < pass.stage_end; ++si) {
        const SStage st = ldc<SStage>(stages + si);
        // thread bits: the local bits that are not register bits, in the stage's lane order
        uint32_t et = 0;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j) et |= uint32_t((t >> j) & 1) << st.tbits[j];
        int so[E];  // LDS slot offsets of the register elements (slots are additive over disjoint bits)
        {
            int sj[LOG_E];
#pragma unroll
            for (int j = 0; j < LOG_E; ++j) sj[j] = slot<T>(int(1u << st.rb[j]));
            so[0] = 0;
#pragma unroll
            for (int r = 1; r < E; ++r) so[r] = so[r & (r - 1)] + sj[__builtin_ctz(r)];
        }
        const int ls = slot<T>(et);
        const bool first = si == pass.stage_begin, last = si == pass.stage_end - 1;
        const bool in_mem = first && (pass.direct & 1), out_mem = last && (pass.direct & 2);
        // memory address of element (t, r) in this stage's layout: base | index bits of et | index bits of r's register bits
        uint64_t gt = 0;
        if (in_mem) {
#pragma unroll
            for (int j = 0; j < LOG_T; ++j)
                if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
            gt |= base;
        }
        auto gr = [&](int r) {  // uniform
            uint64_t v = 0;
#pragma unroll
            for (int j = 0; j < LOG_E; ++j)
                if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
            return v;
        };
        if (in_mem) {
            const C *ag = reinterpret_cast<const C *>(a) + gt;
            if (init_zero) {
#pragma unroll
                for (int r = 0; r < E; ++r) x[r] = C{(gt | gr(r)) == 0 ? T(1) : T(0), T(0)};
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) x[r] = ld_nt(ag + gr(r));
                if (EDGE && edge.scale) edge_scale<T, E>(x, edge.scale);
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) x[r] = lds[ls + so[r]];
        }
        run_rounds<T, LOG_E>(x, st, rounds, ops, blks, et, base);
        if (out_mem) break;  // stored below, after the loop
        __syncthreads();  // every thread has read this stage's inputs before anyone overwrites LDS
        if (st.swap_p >= 0 && (base & st.swap_gcm) == st.swap_gcm) {
            // stage-end quantum swap of two resident qubits: a permutation of the LDS slots
#pragma unroll
            for (int r = 0; r < E; ++r) {
                uint32_t d = et;
#pragma unroll
                for (int j = 0; j < LOG_E; ++j)
                    if ((r >> j) & 1) d |= 1u << st.rb[j];
                if ((d & st.swap_lcm) == st.swap_lcm) {
                    const uint32_t bp = (d >> st.swap_p) & 1, bq = (d >> st.swap_q) & 1;
                    if (bp != bq) d ^= (1u << st.swap_p) | (1u << st.swap_q);
                }
                lds[slot<T>(d)] = x[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) lds[ls + so[r]] = x[r];
        }
        __syncthreads();
    }
    if (pass.direct & 2) {
        // the last stage's registers go straight to memory; storing after the stage loop keeps every
        // load of the op tables ahead of the first store to the state (scalar loads stay legal)
        const SStage st = ldc<SStage>(stages + (pass.stage_end - 1));
        uint64_t gt = base;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j)
            if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
        C *agw = reinterpret_cast<C *>(a) + gt;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            uint64_t v = 0;
#pragma unroll
            for (int j = 0; j < LOG_E; ++j)
                if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
            st_nt(agw + v, x[r]);
        }
        if (EDGE && edge.norm) nacc += sq_sum<T, E>(x);
    }
}

// Process block `blk` of a pass: load it (or generate |0...0> when init_zero is set), run the
// stages, store it. Called by every thread of a workgroup of 2^LOG_T threads; `lds` holds
// lds_slots<T>(LOG_E + LOG_T) amplitudes.
template <typename T, int LOG_E, int LOG_T, bool EDGE = false>
__device__ __forceinline__ void run_block(T *__restrict__ a, const SPass &pass, uint64_t blk, cptr<SStage> stages,
                                          cptr<SRound> rounds, cptr<SOp> ops, cptr<SBlk> blks,
                                          typename Vec<T>::C *lds, bool init_zero, SEdge edge)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    constexpr int NT = 1 << LOG_T;
    const int t = threadIdx.x;
    const uint64_t base = block_base<LOG_E + LOG_T>(pass, blk);
    const uint64_t dt = lane_part<LOG_T>(pass, t);
    if (!(pass.direct & 1)) {
        if (init_zero) {
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const bool one = base == 0 && k == 0 && t == 0;
                lds[slot<T>(k * NT + t)] = C{one ? T(1) : T(0), T(0)};
            }
        } else {
            C v[E];
            load_block<T, LOG_E, LOG_T>(a, pass, base, dt, v);
            if (EDGE && edge.scale) edge_scale<T, E>(v, edge.scale);
            regs_to_lds<T, LOG_E, LOG_T>(v, lds);
        }
        __syncthreads();
    }
    double nacc = 0.0;
    run_stages<T, LOG_E, LOG_T, EDGE>(a, pass, base, stages, rounds, ops, blks, lds, init_zero, edge, nacc);
    if (!(pass.direct & 2)) nacc += store_block<T, LOG_E, LOG_T>(a, pass, base, dt, lds, EDGE && edge.norm != nullptr);
    if (EDGE && edge.norm) edge_norm_out(nacc, edge.norm, blk, lds);
    // a caller that runs the next block in this workgroup overwrites LDS: every thread must have
    // read its last values first
    __syncthreads();
}


// ---- half-buffer passes ----------------------------------------------------------------------------
// Local index v with bit b removed (the bits above b move down one place): the slot of an element in
// a buffer that holds one half of the block, the half with a fixed value of bit b.
__device__ __forceinline__ uint32_t squeeze(uint32_t v, uint32_t b)
{
    const uint32_t low = (1u << b) - 1;
    return (v & low) | ((v >> 1) & ~low);
}

// Slot offsets of a stage's register elements in the half buffer split by local bit b (a thread bit,
// so never one of the register bits rb[]): slots are additive over disjoint bits, so so[r] is the sum
// of the offsets of r's bits, one addition per element.
template <typename T, int LOG_E>
__device__ __forceinline__ void half_slots(const uint8_t *rb, uint32_t b, int *so)
{
    int sj[LOG_E];
#pragma unroll
    for (int j = 0; j < LOG_E; ++j) {
        const uint32_t p = rb[j];
        sj[j] = slot<T>(int(1u << (p - (p > b ? 1u : 0u))));
    }
    so[0] = 0;
#pragma unroll
    for (int r = 1; r < (1 << LOG_E); ++r) so[r] = so[r & (r - 1)] + sj[__builtin_ctz(r)];
}

// One LDS round trip of a half-buffer pass: registers x move from layout A (thread slot wls, register
// slots wso[r]) to layout B (rls, rso[r]) through a buffer of half the block, split by a local bit that
// sits at thread position j in both layouts: all elements of a thread lie in the half of its own bit j.
// The threads with bit j = 0 exchange first, then the others. pre: start with a barrier (the buffer
// may still be being read).
template <typename T, int E>
__device__ __forceinline__ void exchange_half(typename Vec<T>::C *x, typename Vec<T>::C *lds, int wls, const int *wso,
                                              int rls, const int *rso, uint32_t j, bool pre)
{
    const uint32_t mine = (uint32_t(threadIdx.x) >> j) & 1;
#pragma unroll
    for (uint32_t p = 0; p < 2; ++p) {
        if (pre || p) __syncthreads();
        if (mine == p) {
#pragma unroll
            for (int r = 0; r < E; ++r) lds[wls + wso[r]] = x[r];
        }
        __syncthreads();
        if (mine == p) {
#pragma unroll
            for (int r = 0; r < E; ++r) x[r] = lds[rls + rso[r]];
        }
    }
}

// Process block `blk` of a half-buffer pass (SPass::direct bit 2): as run_block, with every LDS round
// trip split in two by the stages' split bits. `lds` holds lds_slots<T>(LOG_E + LOG_T - 1) amplitudes.
template <typename T, int LOG_E, int LOG_T, bool EDGE = false>
__device__ __forceinline__ void run_block_half(T *__restrict__ a, const SPass &pass, uint64_t blk, cptr<SStage> stages,
                                               cptr<SRound> rounds, cptr<SOp> ops, cptr<SBlk> blks, typename Vec<T>::C *lds,
                                               bool init_zero, SEdge edge)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    const int t = threadIdx.x;
    const uint64_t base = block_base<LOG_E + LOG_T>(pass, blk);
    // load/store layout: thread t, element k at local index k * 2^LOG_T + t; its split bit is a thread
    // bit, so the element parts move down one place in the half buffer
    int lso[E];
#pragma unroll
    for (int k = 0; k < E; ++k) lso[k] = slot<T>(k << (LOG_T - 1));
    C x[E];
    SStage st = ldc<SStage>(stages + pass.stage_begin);
    uint32_t et = 0;
#pragma unroll
    for (int j = 0; j < LOG_T; ++j) et |= uint32_t((t >> j) & 1) << st.tbits[j];
    if (pass.direct & 1) {
        uint64_t gt = base;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j)
            if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
        if (init_zero) {  // |0...0>: only element 0 of thread 0 of block 0 is 1
#pragma unroll
            for (int r = 0; r < E; ++r) x[r] = C{(gt == 0 && r == 0) ? T(1) : T(0), T(0)};
        } else {
            const C *ag = reinterpret_cast<const C *>(a) + gt;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                uint64_t v = 0;
#pragma unroll
                for (int j = 0; j < LOG_E; ++j)
                    if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
                x[r] = ld_nt(ag + v);
            }
            if (EDGE && edge.scale) edge_scale<T, E>(x, edge.scale);
        }
    } else {
        const uint64_t g0 = base | lane_part<LOG_T>(pass, t);
        if (init_zero) {
#pragma unroll
            for (int k = 0; k < E; ++k) x[k] = C{(g0 == 0 && k == 0) ? T(1) : T(0), T(0)};
        } else {
            const C *ag = reinterpret_cast<const C *>(a) + g0;
#pragma unroll
            for (int k = 0; k < E; ++k) x[k] = ld_nt(ag + elem_part<LOG_E, LOG_T>(pass, k));
            if (EDGE && edge.scale) edge_scale<T, E>(x, edge.scale);
        }
        int so[E];
        half_slots<T, LOG_E>(st.rb, st.hb_in, so);
        exchange_half<T, E>(x, lds, slot<T>(int(squeeze(uint32_t(t), st.hb_in))), lso,
                            slot<T>(int(squeeze(et, st.hb_in))), so, st.hj_in, false);
    }
    for (int si = pass.stage_begin;;) {
        run_rounds<T, LOG_E>(x, st, rounds, ops, blks, et, base);
        if (++si == pass.stage_end) break;
        const SStage nx = ldc<SStage>(stages + si);
        uint32_t nt = 0;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j) nt |= uint32_t((t >> j) & 1) << nx.tbits[j];
        int wso[E], rso[E];
        half_slots<T, LOG_E>(st.rb, st.hb_out, wso);
        half_slots<T, LOG_E>(nx.rb, st.hb_out, rso);
        exchange_half<T, E>(x, lds, slot<T>(int(squeeze(et, st.hb_out))), wso, slot<T>(int(squeeze(nt, st.hb_out))), rso,
                            st.hj_out, true);
        st = nx;
        et = nt;
    }
    double nacc = 0.0;
    if (pass.direct & 2) {
        uint64_t gt = base;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j)
            if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
        C *agw = reinterpret_cast<C *>(a) + gt;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            uint64_t v = 0;
#pragma unroll
            for (int j = 0; j < LOG_E; ++j)
                if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
            st_nt(agw + v, x[r]);
        }
        if (EDGE && edge.norm) nacc = sq_sum<T, E>(x);
    } else {
        int so[E];
        half_slots<T, LOG_E>(st.rb, st.hb_out, so);
        exchange_half<T, E>(x, lds, slot<T>(int(squeeze(et, st.hb_out))), so, slot<T>(int(squeeze(uint32_t(t), st.hb_out))),
                            lso, st.hj_out, true);
        C *agw = reinterpret_cast<C *>(a) + (base | lane_part<LOG_T>(pass, t));
#pragma unroll
        for (int k = 0; k < E; ++k) st_nt(agw + elem_part<LOG_E, LOG_T>(pass, k), x[k]);
        if (EDGE && edge.norm) nacc = sq_sum<T, E>(x);
    }
    if (EDGE && edge.norm) edge_norm_out(nacc, edge.norm, blk, lds);
}

// ---- wave-split half-buffer passes ----------------------------------------------------------------
// The same round trips when every split position is a wave bit (j >= 6): each wavefront lies wholly in
// one half, so the branches are uniform and each arm is straight-line code:
//   first half:   [B0] write B1 read B2 B3
//   second half:  [B0] B1 B2 write B3 read
// The write half ends a stage and the read half starts the next, so the amplitudes are not live across
// the stage loop; together with recomputing addresses and thread bits where they are used, the block
// fits in 128 VGPRs (four 256-thread workgroups per CU).
//
// Barrier invariant. The barriers sit in branches that are uniform per wavefront (j >= 6 is a wave bit)
// but differ between the halves. This is correct because s_barrier counts one arrival per wavefront:
// the k-th barrier a wavefront executes is the same barrier instance for every wavefront, whichever
// branch issued it. Every wavefront executes pre + 3 barriers per round trip (first half: pre, B1
// after its write, B2 and B3 after its read; second half: pre, B1, B2 before its write, B3 after it),
// and all wavefronts run the same round trips in the same order (they depend only on the uniform pass
// and stage records). So B1 orders the first half's writes before its reads, B2 its reads before the
// second half's writes, B3 those writes before the second half's reads, and the next round trip's
// pre barrier orders the second half's reads before any new write. tests/staged_model.py follows this
// control flow wavefront by wavefront and checks the counts and these orderings on real schedules.
template <typename T, int E>
__device__ __forceinline__ void wave_out(const typename Vec<T>::C *x, typename Vec<T>::C *lds, int wls, const int *wso,
                                         uint32_t j, bool pre)
{
    const uint32_t second = __builtin_amdgcn_readfirstlane((uint32_t(threadIdx.x) >> j) & 1);
    if (pre) __syncthreads();
    if (second) {
        __syncthreads();
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < E; ++r) lds[wls + wso[r]] = x[r];
    __syncthreads();
}
template <typename T, int E>
__device__ __forceinline__ void wave_in(typename Vec<T>::C *x, const typename Vec<T>::C *lds, int rls, const int *rso,
                                        uint32_t j)
{
    const uint32_t second = __builtin_amdgcn_readfirstlane((uint32_t(threadIdx.x) >> j) & 1);
#pragma unroll
    for (int r = 0; r < E; ++r) x[r] = lds[rls + rso[r]];
    if (!second) {
        __syncthreads();  // the other half may overwrite the buffer after this
        __syncthreads();
    }
}

// Process block `blk` of a wave-split pass (SPass::direct bits 2 and 3). `lds` holds
// lds_slots<T>(LOG_E + LOG_T - 1) amplitudes.
template <typename T, int LOG_E, int LOG_T, bool EDGE = false>
__device__ __forceinline__ void run_block_wave(T *__restrict__ a, const SPass &pass, uint64_t blk, cptr<SStage> stages,
                                               cptr<SRound> rounds, cptr<SOp> ops, cptr<SBlk> blks, typename Vec<T>::C *lds,
                                               bool init_zero, SEdge edge)
{
    using C = typename Vec<T>::C;
    constexpr int E = 1 << LOG_E;
    const int t = threadIdx.x;
    const uint64_t base = block_base<LOG_E + LOG_T>(pass, blk);
    int lso[E];  // load/store layout: element k at local index k * 2^LOG_T + t, one place lower in the half
#pragma unroll
    for (int k = 0; k < E; ++k) lso[k] = slot<T>(k << (LOG_T - 1));
    C x[E];
    for (int si = pass.stage_begin; si < pass.stage_end; ++si) {
        const SStage st = ldc<SStage>(stages + si);
        const bool first = si == pass.stage_begin, last = si == pass.stage_end - 1;
        int tt = t;
        asm volatile("" : "+v"(tt));  // recompute the thread bits per stage rather than keep them live
        uint32_t et = 0;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j) et |= uint32_t((tt >> j) & 1) << st.tbits[j];
        if (first && (pass.direct & 1)) {
            uint64_t gt = base;
#pragma unroll
            for (int j = 0; j < LOG_T; ++j)
                if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
            if (init_zero) {  // |0...0>: only element 0 of thread 0 of block 0 is 1
#pragma unroll
                for (int r = 0; r < E; ++r) x[r] = C{(gt == 0 && r == 0) ? T(1) : T(0), T(0)};
            } else {
                const C *ag = reinterpret_cast<const C *>(a) + gt;
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    uint64_t v = 0;
#pragma unroll
                    for (int j = 0; j < LOG_E; ++j)
                        if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
                    x[r] = ld_nt(ag + v);
                }
                if (EDGE && edge.scale) edge_scale<T, E>(x, edge.scale);
            }
        } else {
            if (first) {
                uint64_t g0 = base | lane_part<LOG_T>(pass, t);
                asm volatile("" : "+v"(g0));  // not kept alive until the store
                if (init_zero) {
#pragma unroll
                    for (int k = 0; k < E; ++k) x[k] = C{(g0 == 0 && k == 0) ? T(1) : T(0), T(0)};
                } else {
                    const C *ag = reinterpret_cast<const C *>(a) + g0;
#pragma unroll
                    for (int k = 0; k < E; ++k) x[k] = ld_nt(ag + elem_part<LOG_E, LOG_T>(pass, k));
                    if (EDGE && edge.scale) edge_scale<T, E>(x, edge.scale);
                }
                wave_out<T, E>(x, lds, slot<T>(int(squeeze(uint32_t(t), st.hb_in))), lso, st.hj_in, false);
            }
            int so[E];
            half_slots<T, LOG_E>(st.rb, st.hb_in, so);
            wave_in<T, E>(x, lds, slot<T>(int(squeeze(et, st.hb_in))), so, st.hj_in);
        }
        run_rounds<T, LOG_E>(x, st, rounds, ops, blks, et, base);
        if (last) break;  // stored below, after the loop
        int so[E];
        half_slots<T, LOG_E>(st.rb, st.hb_out, so);
        wave_out<T, E>(x, lds, slot<T>(int(squeeze(et, st.hb_out))), so, st.hj_out, true);
    }
    // storing after the stage loop keeps every load of the op tables ahead of the first store to the
    // state (scalar loads stay legal)
    const SStage st = ldc<SStage>(stages + (pass.stage_end - 1));
    double nacc = 0.0;
    if (pass.direct & 2) {
        uint64_t gt = base;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j)
            if ((t >> j) & 1) gt |= uint64_t(1) << st.ptb[j];
        C *agw = reinterpret_cast<C *>(a) + gt;
#pragma unroll
        for (int r = 0; r < E; ++r) {
            uint64_t v = 0;
#pragma unroll
            for (int j = 0; j < LOG_E; ++j)
                if ((r >> j) & 1) v |= uint64_t(1) << st.prb[j];
            st_nt(agw + v, x[r]);
        }
        if (EDGE && edge.norm) nacc = sq_sum<T, E>(x);
    } else {
        uint32_t et = 0;
#pragma unroll
        for (int j = 0; j < LOG_T; ++j) et |= uint32_t((t >> j) & 1) << st.tbits[j];
        int so[E];
        half_slots<T, LOG_E>(st.rb, st.hb_out, so);
        wave_out<T, E>(x, lds, slot<T>(int(squeeze(et, st.hb_out))), so, st.hj_out, true);
        wave_in<T, E>(x, lds, slot<T>(int(squeeze(uint32_t(t), st.hb_out))), lso, st.hj_out);
        uint64_t g0 = base | lane_part<LOG_T>(pass, t);
        asm volatile("" : "+v"(g0));
        C *agw = reinterpret_cast<C *>(a) + g0;
#pragma unroll
        for (int k = 0; k < E; ++k) st_nt(agw + elem_part<LOG_E, LOG_T>(pass, k), x[k]);
        if (EDGE && edge.norm) nacc = sq_sum<T, E>(x);
    }
    // every wavefront reaches this point after the same number of barriers, so the ones below pair up
    if (EDGE && edge.norm) edge_norm_out(nacc, edge.norm, blk, lds);
}

// One launch of a staged pass: its tables, the optional renormalisation edge (see SEdge) and the kernel
// mode (0: reads the state; 1: folds a renormalisation point; 2: first pass of a run from |0...0>).
struct PassLaunch {
    void *data;
    const SPass *pass;
    const SStage *stages;
    const SRound *rounds;
    const SOp *ops;
    const SBlk *blks;
    const double *scale;
    double *norm;
    unsigned grid;
    hipStream_t stream;
    int mode;
};
// launch the pass kernel of a block shape (2^log_e amplitudes per thread, 2^log_t threads) in the
// given form (QSIM_STAGED_FULL or QSIM_STAGED_HALF; the wave form through launch_wave_*); EINVAL if the
// shape has no such kernel
int launch_pass_c128(int form, int log_e, int log_t, const PassLaunch &a);
int launch_pass_c64(int form, int log_e, int log_t, const PassLaunch &a);
int launch_wave_c128(int log_e, int log_t, const PassLaunch &a);
int launch_wave_c64(int log_e, int log_t, const PassLaunch &a);

// host: append the schedule of one circuit (see staged.hip). search_width > 1: resident sets from a
// bounded beam search of that width where it needs fewer passes than the greedy rule (plans use
// kPassSearchWidth)
constexpr int kPassSearchWidth = 32;
int staged_schedule(int n, int dtype, int m, int log_e, const std::vector<qsim_gate> &gates, std::vector<SPass> &passes,
                    std::vector<SStage> &stages, std::vector<SRound> &rounds, std::vector<SOp> &ops,
                    std::vector<SBlk> &blks, int search_width = 1);
bool staged_variant_ok(int dtype, int log_e, int log_t);
__global__ void k_op_angles(SOp *ops, int nops);

}  // namespace staged
}  // namespace qsim
