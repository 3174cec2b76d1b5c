// Per-gate sweep kernels for gfx950: one in-place pass over the amplitudes a gate touches.
//
// A gate on target t with control set C updates the pairs (a(..0_t..), a(..1_t..)) whose control
// bits are all 1 (the common form of Eqs. NUM2-NUM8). The pair index j in [0, 2^(n-|C|-1)) is
// turned into the base index by inserting a zero bit at every position of sorted(C u {t}) and
// OR-ing the control bits, so consecutive lanes touch consecutive addresses except across the
// inserted bits: for a high target the two halves of a pair are two fully coalesced runs.
//
// Layout choices for HBM3E:
//   * complex128: 16 B per amplitude = one dwordx4 per lane per half;
//   * complex64: when bit 0 is not an inserted position, a lane owns two neighbouring pairs and
//     moves 16 B per half (VEC = 2), otherwise 8 B (VEC = 1);
//   * every thread keeps ITEMS independent items in flight (all loads issued before any store);
//   * grid-stride outer loop with a capped grid, so any n fits the 32-bit work-item limit.
#include "qsim_internal.h"

namespace qsim {

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kMaxGrid = 1u << 20;

template <typename T> struct Vec;
template <> struct Vec<double> { using C = double2; using C2 = double4; };
template <> struct Vec<float> { using C = float2; using C2 = float4; };

// 16-byte and 8-byte words moved with or without the nontemporal (streaming) hint. Streaming
// loads and stores pay off when every lane's word belongs to a run of at least 256 contiguous
// bytes; for shorter runs the partial lines are better served by the caches.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <bool NT, typename W> __device__ __forceinline__ W ldw(const void *p)
{
    static_assert(sizeof(W) == 16 || sizeof(W) == 8, "8- or 16-byte words only");
    using V = typename std::conditional<sizeof(W) == 16, u32x4, u32x2>::type;
    V v;
    if constexpr (NT) v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
    else v = *reinterpret_cast<const V *>(p);
    W w;
    __builtin_memcpy(&w, &v, sizeof(W));
    return w;
}
template <bool NT, typename W> __device__ __forceinline__ void stw(void *p, const W &w)
{
    static_assert(sizeof(W) == 16 || sizeof(W) == 8, "8- or 16-byte words only");
    using V = typename std::conditional<sizeof(W) == 16, u32x4, u32x2>::type;
    V v;
    __builtin_memcpy(&v, &w, sizeof(W));
    if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
    else *reinterpret_cast<V *>(p) = v;
}


template <typename T> struct CMat {
    T r[4], i[4];
    __device__ __forceinline__ void load(const Mat2 &u)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            r[k] = static_cast<T>(u.m[2 * k]);
            i[k] = static_cast<T>(u.m[2 * k + 1]);
        }
    }
};

template <typename C, typename T>
__device__ __forceinline__ void mix(const CMat<T> &u, C &x0, C &x1)
{
    const T y0r = u.r[0] * x0.x - u.i[0] * x0.y + u.r[1] * x1.x - u.i[1] * x1.y;
    const T y0i = u.r[0] * x0.y + u.i[0] * x0.x + u.r[1] * x1.y + u.i[1] * x1.x;
    const T y1r = u.r[2] * x0.x - u.i[2] * x0.y + u.r[3] * x1.x - u.i[3] * x1.y;
    const T y1i = u.r[2] * x0.y + u.i[2] * x0.x + u.r[3] * x1.y + u.i[3] * x1.x;
    x0.x = y0r;
    x0.y = y0i;
    x1.x = y1r;
    x1.y = y1i;
}

template <typename T>
__device__ __forceinline__ void cmul(T &xr, T &xi, T fr, T fi)
{
    const T r = fr * xr - fi * xi;
    const T i = fr * xi + fi * xr;
    xr = r;
    xi = i;
}

// Sweep bodies come in two forms. FAST: every chunk of kBlock * ITEMS items is full and at most three
// bits are inserted, so the items need no range checks and their indices come from fixed steps; the
// loads of all items issue back to back. Otherwise every item is range-checked and its index is
// built by the general walk.
template <bool FAST> __device__ __forceinline__ uint64_t index_of(uint64_t j, const IndexMap &m)
{
    if constexpr (FAST) return insert_zeros3(j, m);
    else return insert_zeros(j, m);
}
template <bool FAST> __device__ __forceinline__ bool in_range(uint64_t j, uint64_t items)
{
    if constexpr (FAST) return true;
    else return j < items;
}
template <int ITEMS> __device__ __forceinline__ bool fast_form(uint64_t items, const IndexMap &m)
{
    return m.npos <= 3 && items % (uint64_t(kBlock) * ITEMS) == 0;
}

// ---- general 2x2 on pairs ----------------------------------------------------------------------
template <typename T, int VEC, int ITEMS, bool NT, bool FAST>
__device__ __forceinline__ void k_general_body(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t tbit,
                                                   Mat2 um)
{
    using C = typename Vec<T>::C;
    using C2 = typename Vec<T>::C2;
    CMat<T> u;
    u.load(um);
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < items; base += uint64_t(gridDim.x) * chunk) {
        uint64_t i0[ITEMS];
        C x0[ITEMS][VEC], x1[ITEMS][VEC];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
                i0[k] = index_of<FAST>(j * VEC, map);
                if constexpr (VEC == 2) {
                    const C2 p = ldw<NT, C2>(a + 2 * i0[k]);
                    const C2 q = ldw<NT, C2>(a + 2 * (i0[k] | tbit));
                    x0[k][0] = C{p.x, p.y};
                    x0[k][1] = C{p.z, p.w};
                    x1[k][0] = C{q.x, q.y};
                    x1[k][1] = C{q.z, q.w};
                } else {
                    x0[k][0] = ldw<NT, C>(a + 2 * i0[k]);
                    x1[k][0] = ldw<NT, C>(a + 2 * (i0[k] | tbit));
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) mix(u, x0[k][v], x1[k][v]);
                if constexpr (VEC == 2) {
                    stw<NT>(a + 2 * i0[k], C2{x0[k][0].x, x0[k][0].y, x0[k][1].x, x0[k][1].y});
                    stw<NT>(a + 2 * (i0[k] | tbit), C2{x1[k][0].x, x1[k][0].y, x1[k][1].x, x1[k][1].y});
                } else {
                    stw<NT>(a + 2 * i0[k], x0[k][0]);
                    stw<NT>(a + 2 * (i0[k] | tbit), x1[k][0]);
                }
            }
        }
    }
}

template <typename T, int VEC, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_general(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t tbit,
                                                   Mat2 um)
{
    if (fast_form<ITEMS>(items, map)) k_general_body<T, VEC, ITEMS, NT, true>(a, items, map, tbit, um);
    else k_general_body<T, VEC, ITEMS, NT, false>(a, items, map, tbit, um);
}


// ---- low target: partners inside one wave's 64 consecutive amplitude slots --------------------
// Every lane loads whole contiguous words (64 lanes x 16 B = 1 KiB per load instruction) and takes
// the partner amplitude of its pair from lane l ^ 2^tl through a cross-lane permute, so the pair
// update needs no strided access. complex128: lane l holds amplitude base + l (tl = t, t < 6).
// complex64: lane l holds amplitudes base + 2l and base + 2l + 1 (t = 0 is inside the lane;
// otherwise tl = t - 1 < 6). Control bits are tested per amplitude.
template <typename T> __device__ __forceinline__ T xshfl(T v, int m) { return __shfl_xor(v, m, 64); }

template <typename T, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_general_wave(T *__restrict__ a, uint64_t nslots, int t, uint64_t cmask, Mat2 um)
{
    using C = typename Vec<T>::C;
    using C2 = typename Vec<T>::C2;
    CMat<T> u;
    u.load(um);
    constexpr int APL = sizeof(T) == 8 ? 1 : 2;  // amplitudes per lane
    const int lane = threadIdx.x & 63;
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    const int tl = APL == 1 ? t : t - 1;         // lane bit that holds the target (if t >= APL - 1)
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < nslots; base += uint64_t(gridDim.x) * chunk) {
        C x[ITEMS][APL];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t slot = base + uint64_t(k) * kBlock;  // lane-contiguous within a wave
            if (slot < nslots) {
                if constexpr (APL == 1) {
                    x[k][0] = ldw<true, C>(a + 2 * slot);
                } else {
                    const C2 p = ldw<true, C2>(a + 4 * slot);
                    x[k][0] = C{p.x, p.y};
                    x[k][1] = C{p.z, p.w};
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t slot = base + uint64_t(k) * kBlock;
            // every lane of the wave takes part in the permutes (slot < nslots is wave-uniform
            // because nslots is a multiple of 64)
            if (slot < nslots) {
                C orig[APL];
#pragma unroll
                for (int v = 0; v < APL; ++v) orig[v] = x[k][v];
#pragma unroll
                for (int v = 0; v < APL; ++v) {
                    const uint64_t i = slot * APL + v;
                    C self = orig[v], other;
                    if (APL == 2 && t == 0) {
                        other = orig[v ^ 1];
                    } else {
                        other.x = xshfl(self.x, 1 << tl);
                        other.y = xshfl(self.y, 1 << tl);
                    }
                    const bool one = (i >> t) & 1;
                    C lo = one ? other : self, hi = one ? self : other;
                    mix(u, lo, hi);
                    const C y = one ? hi : lo;
                    x[k][v] = ((i & cmask) == cmask) ? y : self;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t slot = base + uint64_t(k) * kBlock;
            if (slot < nslots) {
                if constexpr (APL == 1)
                    stw<true>(a + 2 * slot, x[k][0]);
                else
                    stw<true>(a + 4 * slot, C2{x[k][0].x, x[k][0].y, x[k][1].x, x[k][1].y});
            }
        }
    }
}

// ---- one phase factor on the selected amplitudes ---------------------------------------------
template <typename T, int VEC, int ITEMS, bool NT, bool FAST>
__device__ __forceinline__ void k_phase_body(T *__restrict__ a, uint64_t items, IndexMap map, double c0, double c1,
                                                 int angle_mode)
{
    using C = typename Vec<T>::C;
    using C2 = typename Vec<T>::C2;
    double fr64 = c0, fi64 = c1;
    if (angle_mode == int(DiagMode::Pow2)) c0 = c0 * ldexp(kTwoPi, -int(c1));  // theta = s 2 pi / 2^k, FP64
    if (angle_mode) sincos(c0, &fi64, &fr64);  // FP64 phase factor e^{i theta}
    const T fr = static_cast<T>(fr64), fi = static_cast<T>(fi64);
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < items; base += uint64_t(gridDim.x) * chunk) {
        uint64_t idx[ITEMS];
        C x[ITEMS][VEC];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
                idx[k] = index_of<FAST>(j * VEC, map);
                if constexpr (VEC == 2) {
                    const C2 p = ldw<NT, C2>(a + 2 * idx[k]);
                    x[k][0] = C{p.x, p.y};
                    x[k][1] = C{p.z, p.w};
                } else {
                    x[k][0] = ldw<NT, C>(a + 2 * idx[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) cmul(x[k][v].x, x[k][v].y, fr, fi);
                if constexpr (VEC == 2)
                    stw<NT>(a + 2 * idx[k], C2{x[k][0].x, x[k][0].y, x[k][1].x, x[k][1].y});
                else
                    stw<NT>(a + 2 * idx[k], x[k][0]);
            }
        }
    }
}

template <typename T, int VEC, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_phase(T *__restrict__ a, uint64_t items, IndexMap map, double c0, double c1,
                                                 int angle_mode)
{
    if (fast_form<ITEMS>(items, map)) k_phase_body<T, VEC, ITEMS, NT, true>(a, items, map, c0, c1, angle_mode);
    else k_phase_body<T, VEC, ITEMS, NT, false>(a, items, map, c0, c1, angle_mode);
}

// ---- diag(d0, d1) on the target, controlled ----------------------------------------------------
template <typename T, int VEC, int ITEMS, bool NT, bool FAST>
__device__ __forceinline__ void k_diag_body(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t tbit,
                                                double d0r, double d0i, double d1r, double d1i, int angle_mode)
{
    using C = typename Vec<T>::C;
    using C2 = typename Vec<T>::C2;
    if (angle_mode) {  // d0 = e^{i d0r}, d1 = e^{i d1r}, evaluated in FP64
        sincos(d0r, &d0i, &d0r);
        sincos(d1r, &d1i, &d1r);
    }
    const T f0r = static_cast<T>(d0r), f0i = static_cast<T>(d0i);
    const T f1r = static_cast<T>(d1r), f1i = static_cast<T>(d1i);
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < items; base += uint64_t(gridDim.x) * chunk) {
        uint64_t idx[ITEMS];
        C x[ITEMS][VEC];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
                idx[k] = index_of<FAST>(j * VEC, map);
                if constexpr (VEC == 2) {
                    const C2 p = ldw<NT, C2>(a + 2 * idx[k]);
                    x[k][0] = C{p.x, p.y};
                    x[k][1] = C{p.z, p.w};
                } else {
                    x[k][0] = ldw<NT, C>(a + 2 * idx[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const bool one = ((idx[k] + v) & tbit) != 0;
                    cmul(x[k][v].x, x[k][v].y, one ? f1r : f0r, one ? f1i : f0i);
                }
                if constexpr (VEC == 2)
                    stw<NT>(a + 2 * idx[k], C2{x[k][0].x, x[k][0].y, x[k][1].x, x[k][1].y});
                else
                    stw<NT>(a + 2 * idx[k], x[k][0]);
            }
        }
    }
}

template <typename T, int VEC, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_diag(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t tbit,
                                                double d0r, double d0i, double d1r, double d1i, int angle_mode)
{
    if (fast_form<ITEMS>(items, map)) k_diag_body<T, VEC, ITEMS, NT, true>(a, items, map, tbit, d0r, d0i, d1r, d1i, angle_mode);
    else k_diag_body<T, VEC, ITEMS, NT, false>(a, items, map, tbit, d0r, d0i, d1r, d1i, angle_mode);
}

// ---- permutation: swap a(i) <-> a(i ^ flip), no arithmetic (bit-exact) -------------------------
template <typename T, int VEC, int ITEMS, bool NT, bool FAST>
__device__ __forceinline__ void k_swap_body(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t flip)
{
    // moved as raw 8/16-byte words: no floating-point operation touches the data
    using W = typename std::conditional<sizeof(T) * 2 * VEC == 16, uint4, uint2>::type;
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < items; base += uint64_t(gridDim.x) * chunk) {
        uint64_t i0[ITEMS];
        W x0[ITEMS], x1[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
                i0[k] = index_of<FAST>(j * VEC, map);
                x0[k] = ldw<NT, W>(a + 2 * i0[k]);
                x1[k] = ldw<NT, W>(a + 2 * (i0[k] ^ flip));
            }
        }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const uint64_t j = base + uint64_t(k) * kBlock;
            if (in_range<FAST>(j, items)) {
                stw<NT>(a + 2 * i0[k], x1[k]);
                stw<NT>(a + 2 * (i0[k] ^ flip), x0[k]);
            }
        }
    }
}

template <typename T, int VEC, int ITEMS, bool NT>
__global__ __launch_bounds__(kBlock) void k_swap(T *__restrict__ a, uint64_t items, IndexMap map, uint64_t flip)
{
    if (fast_form<ITEMS>(items, map)) k_swap_body<T, VEC, ITEMS, NT, true>(a, items, map, flip);
    else k_swap_body<T, VEC, ITEMS, NT, false>(a, items, map, flip);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_set_basis(T *__restrict__ a, uint64_t namps, uint64_t x)
{
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < namps; i += uint64_t(gridDim.x) * kBlock) {
        a[2 * i] = (i == x) ? T(1) : T(0);
        a[2 * i + 1] = T(0);
    }
}

// Powers f(x) = y^x mod G for x < count by square and multiply (G < 2^32, so every product of two
// residues fits 64 bits).
// Powers y^(x * stride) mod G for x < count (square and multiply; G < 2^32, so every product of two
// residues fits in 64 bits).
__global__ __launch_bounds__(kBlock) void k_powmod_table(uint32_t *__restrict__ f, uint64_t count, uint64_t y,
                                                        uint64_t stride, uint64_t G)
{
    for (uint64_t x = uint64_t(blockIdx.x) * kBlock + threadIdx.x; x < count; x += uint64_t(gridDim.x) * kBlock) {
        uint64_t r = 1 % G, b = y % G, e = x * stride;
        while (e) {
            if (e & 1) r = r * b % G;
            b = b * b % G;
            e >>= 1;
        }
        f[x] = uint32_t(r);
    }
}

// a * b mod G for residues a, b < G < 2^32 by Barrett reduction with minv = floor((2^64 - 1) / G):
// the estimated quotient is at most two below the true one, so at most two corrections follow
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, uint64_t G, uint64_t minv)
{
    const uint64_t p = a * b;
    uint64_t r = p - __umul64hi(p, minv) * G;
    if (r >= G) r -= G;
    if (r >= G) r -= G;
    return r;
}

// |x>|z> -> |x>|z XOR f(x)>, f(x) = y^x mod G = lo[x mod 2^h] * hi[x >> h] mod G: a permutation of
// basis states made of disjoint exchanges; the thread of the smaller index of each exchanged pair moves
// both amplitudes (no arithmetic on them, bit-exact).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_xor_permute(T *__restrict__ a, uint64_t namps, const uint32_t *__restrict__ lo,
                                                        const uint32_t *__restrict__ hi, int x_first, uint64_t xmask, int h,
                                                        int f_first, uint64_t G, uint64_t minv)
{
    using C = typename Vec<T>::C;
    C *ac = reinterpret_cast<C *>(a);
    const uint64_t lomask = (uint64_t(1) << h) - 1;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < namps; i += uint64_t(gridDim.x) * kBlock) {
        const uint64_t x = (i >> x_first) & xmask;
        const uint64_t v = mulmod(lo[x & lomask], hi[x >> h], G, minv);
        const uint64_t j = i ^ (v << f_first);
        if (j <= i) continue;
        const C ai = ac[i], aj = ac[j];
        ac[i] = aj;
        ac[j] = ai;
    }
}

inline unsigned grid_for(uint64_t items, uint64_t per_block)
{
    uint64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > kMaxGrid) g = kMaxGrid;
    return unsigned(g);
}

// VEC = 2 (two neighbouring amplitudes per lane) is legal when bit 0 is not an inserted position
// and there is an even number of items
inline bool can_vec2(const IndexMap &m, uint64_t items) { return m.p0 > 0 && (items % 2 == 0); }

constexpr int kItems = 4;

// contiguous run (bytes) that every lane's word belongs to: set by the lowest inserted position
template <typename T> inline bool streaming(const IndexMap &m)
{
    const int p0 = m.p0 > 63 ? 63 : m.p0;
    return (uint64_t(2 * sizeof(T)) << (p0 > 40 ? 40 : p0)) >= 256;
}

template <typename T>
int general_t(qsim_state *s, const IndexMap &map, int target, const Mat2 &u)
{
    const uint64_t pairs = dim(s->n) >> map.npos;
    T *a = static_cast<T *>(s->data);
    const uint64_t tbit = uint64_t(1) << target;
    // low target, partner inside the wave's 64 slots: cross-lane exchange on contiguous words
    constexpr int APL = sizeof(T) == 8 ? 1 : 2;
    const uint64_t nslots = dim(s->n) / APL;
    const int tl = target - (APL - 1);
    if (tl < 6 && !streaming<T>(make_index_map(tbit, 0)) && nslots % 64 == 0) {
        uint64_t cmask = map.set;
        const int IT = 4;
        hipLaunchKernelGGL((k_general_wave<T, IT>), dim3(grid_for(nslots, kBlock * IT)), dim3(kBlock), 0, s->stream, a, nslots,
                           target, cmask, u);
        QSIM_HIP(hipGetLastError());
        return QSIM_OK;
    }
    const bool nt = streaming<T>(map);
    // complex64 moves two neighbouring amplitudes per 16-byte word (VEC = 2); complex128 never does
    bool vec2 = false;
    if constexpr (sizeof(T) == 4) {
        vec2 = can_vec2(map, pairs);
        if (vec2) {
            const uint64_t items = pairs / 2;
            if (nt)
                hipLaunchKernelGGL((k_general<T, 2, kItems, true>), dim3(grid_for(items, kBlock * kItems)), dim3(kBlock), 0,
                                   s->stream, a, items, map, tbit, u);
            else
                hipLaunchKernelGGL((k_general<T, 2, kItems, false>), dim3(grid_for(items, kBlock * kItems)), dim3(kBlock), 0,
                                   s->stream, a, items, map, tbit, u);
        }
    }
    if (!vec2) {
        if (nt)
            hipLaunchKernelGGL((k_general<T, 1, kItems, true>), dim3(grid_for(pairs, kBlock * kItems)), dim3(kBlock), 0, s->stream,
                               a, pairs, map, tbit, u);
        else
            hipLaunchKernelGGL((k_general<T, 1, kItems, false>), dim3(grid_for(pairs, kBlock * kItems)), dim3(kBlock), 0,
                               s->stream, a, pairs, map, tbit, u);
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

template <typename T, bool NTV>
int phase_nt(qsim_state *s, const IndexMap &map, const double c[2], DiagMode mode)
{
    const uint64_t items0 = dim(s->n) >> map.npos;
    T *a = static_cast<T *>(s->data);
    bool vec2 = false;  // complex64 only, as in general_t
    if constexpr (sizeof(T) == 4) {
        vec2 = can_vec2(map, items0);
        if (vec2) {
            const uint64_t items = items0 / 2;
            hipLaunchKernelGGL((k_phase<T, 2, kItems, NTV>), dim3(grid_for(items, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                               items, map, c[0], c[1], int(mode));
        }
    }
    if (!vec2) {
        hipLaunchKernelGGL((k_phase<T, 1, kItems, NTV>), dim3(grid_for(items0, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                           items0, map, c[0], c[1], int(mode));
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

template <typename T, bool NTV>
int diag_nt(qsim_state *s, const IndexMap &map, int target, const double d[4], DiagMode mode)
{
    const uint64_t items0 = dim(s->n) >> map.npos;
    T *a = static_cast<T *>(s->data);
    const uint64_t tbit = uint64_t(1) << target;
    bool vec2 = false;  // complex64 only, as in general_t
    if constexpr (sizeof(T) == 4) {
        vec2 = can_vec2(map, items0);
        if (vec2) {
            const uint64_t items = items0 / 2;
            hipLaunchKernelGGL((k_diag<T, 2, kItems, NTV>), dim3(grid_for(items, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                               items, map, tbit, d[0], d[1], d[2], d[3], int(mode));
        }
    }
    if (!vec2) {
        hipLaunchKernelGGL((k_diag<T, 1, kItems, NTV>), dim3(grid_for(items0, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                           items0, map, tbit, d[0], d[1], d[2], d[3], int(mode));
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

template <typename T, bool NTV>
int swap_nt(qsim_state *s, const IndexMap &map, uint64_t flip)
{
    const uint64_t items0 = dim(s->n) >> map.npos;
    T *a = static_cast<T *>(s->data);
    bool vec2 = false;  // complex64 only, as in general_t
    if constexpr (sizeof(T) == 4) {
        vec2 = can_vec2(map, items0);
        if (vec2) {
            const uint64_t items = items0 / 2;
            hipLaunchKernelGGL((k_swap<T, 2, kItems, NTV>), dim3(grid_for(items, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                               items, map, flip);
        }
    }
    if (!vec2) {
        hipLaunchKernelGGL((k_swap<T, 1, kItems, NTV>), dim3(grid_for(items0, kBlock * kItems)), dim3(kBlock), 0, s->stream, a,
                           items0, map, flip);
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

template <typename T>
int phase_t(qsim_state *s, const IndexMap &map, const double c[2], DiagMode mode)
{
    return streaming<T>(map) ? phase_nt<T, true>(s, map, c, mode) : phase_nt<T, false>(s, map, c, mode);
}

template <typename T>
int diag_t(qsim_state *s, const IndexMap &map, int target, const double d[4], DiagMode mode)
{
    return streaming<T>(map) ? diag_nt<T, true>(s, map, target, d, mode) : diag_nt<T, false>(s, map, target, d, mode);
}

template <typename T>
int swap_t(qsim_state *s, const IndexMap &map, uint64_t flip)
{
    // the partner run starts at the lowest flipped bit too
    IndexMap m2 = map;
    return streaming<T>(m2) ? swap_nt<T, true>(s, map, flip) : swap_nt<T, false>(s, map, flip);
}

}  // namespace

IndexMap make_index_map(uint64_t posmask, uint64_t set)
{
    IndexMap m{};
    m.set = set;
    m.posmask = posmask;
    m.npos = __builtin_popcountll(posmask);
    m.p0 = posmask ? __builtin_ctzll(posmask) : 64;
    uint64_t pm = posmask;
    for (int k = 0; k < 3; ++k) {
        if (pm) {
            m.lo[k] = (uint64_t(1) << __builtin_ctzll(pm)) - 1;
            pm &= pm - 1;
        } else {
            m.lo[k] = ~uint64_t(0);
        }
    }
    return m;
}

int launch_general(qsim_state *s, const IndexMap &map, int target, const Mat2 &u)
{
    return s->dtype == QSIM_C128 ? general_t<double>(s, map, target, u) : general_t<float>(s, map, target, u);
}

int launch_phase(qsim_state *s, const IndexMap &map, const double c[2], DiagMode mode)
{
    return s->dtype == QSIM_C128 ? phase_t<double>(s, map, c, mode) : phase_t<float>(s, map, c, mode);
}

int launch_diag(qsim_state *s, const IndexMap &map, int target, const double d[4], DiagMode mode)
{
    return s->dtype == QSIM_C128 ? diag_t<double>(s, map, target, d, mode) : diag_t<float>(s, map, target, d, mode);
}

int launch_swap(qsim_state *s, const IndexMap &map, uint64_t flip)
{
    return s->dtype == QSIM_C128 ? swap_t<double>(s, map, flip) : swap_t<float>(s, map, flip);
}

int launch_modexp(qsim_state *s, int x_first, int x_qubits, int f_first, uint64_t y, uint64_t G)
{
    // two power tables in the state's scratch buffer: y^xl for the low h bits of x and y^(xh 2^h) for
    // the high ones (at most 2 * 2^15 entries for a 30-qubit x-register); no allocation, no host wait
    const int h = (x_qubits + 1) / 2;
    const uint64_t nlo = uint64_t(1) << h, nhi = uint64_t(1) << (x_qubits - h);
    static_assert(2 * (1 << 15) * sizeof(uint32_t) <= kScratchDoubles * sizeof(double), "power tables fit the scratch");
    uint32_t *lo = reinterpret_cast<uint32_t *>(s->scratch);
    uint32_t *hi = lo + nlo;
    const uint64_t minv = ~uint64_t(0) / G;
    hipLaunchKernelGGL(k_powmod_table, dim3(grid_for(nlo, kBlock)), dim3(kBlock), 0, s->stream, lo, nlo, y, uint64_t(1), G);
    hipLaunchKernelGGL(k_powmod_table, dim3(grid_for(nhi, kBlock)), dim3(kBlock), 0, s->stream, hi, nhi, y, nlo, G);
    QSIM_HIP(hipGetLastError());
    const uint64_t N = dim(s->n);
    const uint64_t xmask = (uint64_t(1) << x_qubits) - 1;
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_xor_permute<double>, dim3(grid_for(N, kBlock * 4)), dim3(kBlock), 0, s->stream,
                           static_cast<double *>(s->data), N, lo, hi, x_first, xmask, h, f_first, G, minv);
    else
        hipLaunchKernelGGL(k_xor_permute<float>, dim3(grid_for(N, kBlock * 4)), dim3(kBlock), 0, s->stream,
                           static_cast<float *>(s->data), N, lo, hi, x_first, xmask, h, f_first, G, minv);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int launch_set_basis(qsim_state *s, uint64_t x)
{
    const uint64_t N = dim(s->n);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_set_basis<double>, dim3(grid_for(N, kBlock * 4)), dim3(kBlock), 0, s->stream,
                           static_cast<double *>(s->data), N, x);
    else
        hipLaunchKernelGGL(k_set_basis<float>, dim3(grid_for(N, kBlock * 4)), dim3(kBlock), 0, s->stream,
                           static_cast<float *>(s->data), N, x);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

}  // namespace qsim
