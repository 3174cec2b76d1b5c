// Dense k-qubit gates (1 <= k <= 5): for every base index b with zero bits at the gate qubits,
// v_r = a(b + off[r]) (off[r] = sum_s bit_s(r) 2^qubits[s]) is replaced by U v.
//
// k >= 4: a dense contraction on the matrix cores. With K = 2^k amplitudes per column, X = Xr + i Xi
// (K x 2^(n-k), split into real and imaginary parts) goes to Y = U X through three real K x K products
// (the three-multiplication form of a complex product): T1 = Ur Xr, T2 = Ui Xi, T3 = (Ur + Ui)(Xr + Xi),
// then Yr = T1 - T2 and Yi = T3 - T1 - T2. That is 3 K^2 multiply-adds per column on the matrix cores
// instead of the 4 K^2 of the real form [[Ur, -Ui], [Ui, Ur]], for 2 K additions per column on the
// vector ALU. One wave computes 16 columns at a time with v_mfma_f64_16x16x4f64 (complex128) or
// v_mfma_f32_16x16x4f32 (complex64, FP32 accumulation): lane l owns column l % 16 and K-row group
// l / 16. A lane loads whole amplitudes (16 B / 8 B), one per K-step, and stores whole amplitudes from
// the accumulators of the same row positions. The three matrices are staged in LDS in fragment order,
// so every A-operand read is one conflict-free ds_read per lane.
//
// k <= 3: one lane per column on the vector ALUs, U in kernel arguments.
#include "qsim_internal.h"

namespace qsim {

namespace {

constexpr int kBlock = 256;

template <typename T> struct Vec;
template <> struct Vec<double> { using C = double2; };
template <> struct Vec<float> { using C = float2; };

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct Acc;
template <> struct Acc<double> { using V = d4_t; };
template <> struct Acc<float> { using V = f4_t; };

__device__ __forceinline__ d4_t mfma16(double a, double b, d4_t c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma16(float a, float b, f4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


struct QubitList {
    int32_t k;
    int32_t q[8];
};

__device__ __forceinline__ uint64_t offset_of(int r, const QubitList &ql)
{
    uint64_t o = 0;
#pragma unroll
    for (int s = 0; s < 5; ++s)
        if (s < ql.k && ((r >> s) & 1)) o |= uint64_t(1) << ql.q[s];
    return o;
}

// Amplitude (within the K of a column) that lane group kq loads for real K-step kk < KS/2, and
// whose result the same lane later stores. It is chosen so that the accumulator layout of the
// MFMA hands every lane back exactly the amplitudes it loaded:
//   v_mfma_f64_16x16x4f64: accumulator register v of lane l holds row (l / 16) + 4 v;
//   v_mfma_f32_16x16x4f32: accumulator register v of lane l holds row 4 (l / 16) + v.
// Store (row block mb, register v) <-> load step kk = 4 mb + v.
template <typename T> __host__ __device__ inline int amp_of(int kk, int kq);
template <> __host__ __device__ inline int amp_of<double>(int kk, int kq) { return 4 * kk + kq; }
template <> __host__ __device__ inline int amp_of<float>(int kk, int kq) { return 16 * (kk >> 2) + 4 * kq + (kk & 3); }

// Fragment order of the three matrices M_0 = Ur, M_1 = Ui, M_2 = Ur + Ui:
// frag[((p * MB + mb) * KS + kk) * 64 + l] = M_p[16 mb + l % 16][amp_of(kk, l / 16)].
template <typename T, int KLOG>
__global__ __launch_bounds__(kBlock) void k_fused_mfma(T *__restrict__ a, uint64_t ntiles, IndexMap map, QubitList ql,
                                                      const T *__restrict__ wfrag)
{
    using C = typename Vec<T>::C;
    using AV = typename Acc<T>::V;
    constexpr int K = 1 << KLOG;   // amplitudes per column
    constexpr int KS = K / 4;      // K-steps of 4 (one amplitude per lane each)
    constexpr int MB = K / 16;     // output row blocks of 16
    constexpr int NA = KS;         // amplitudes per lane per column tile
    constexpr int FR = MB * KS * 64;  // fragment words of one matrix
    __shared__ T W[3 * FR];
    for (int i = threadIdx.x; i < 3 * FR; i += kBlock) W[i] = wfrag[i];
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 15;
    const int kq = lane >> 4;
    // offset of the amplitude a lane loads at K-step kk: the lane-group part (bits of kq) plus a
    // wave-uniform part (bits of kk), which occupy disjoint bits of amp_of
    const uint64_t dq = offset_of(amp_of<T>(0, kq), ql);
    auto off = [&](int kk) { return dq + offset_of(amp_of<T>(kk, 0), ql); };

    const uint64_t wstride = uint64_t(gridDim.x) * (kBlock / 64);
    uint64_t tile = uint64_t(blockIdx.x) * (kBlock / 64) + wave;
    C x[NA];
    if (tile < ntiles) {
        const uint64_t b = insert_zeros(tile * 16 + col, map);
#pragma unroll
        for (int kk = 0; kk < NA; ++kk) x[kk] = *reinterpret_cast<const C *>(a + 2 * (b + off(kk)));
    }
    while (tile < ntiles) {
        // the matrices stay in LDS and are re-read every tile (a compiler barrier keeps them from being
        // hoisted into registers), which leaves room for more resident waves
        asm volatile("" ::: "memory");
        const uint64_t b = insert_zeros(tile * 16 + col, map);
        const uint64_t next = tile + wstride;
        // prefetch the next tile of this wave before the contraction of the current one
        C xn[NA];
        if (next < ntiles) {
            const uint64_t bn = insert_zeros(next * 16 + col, map);
#pragma unroll
            for (int kk = 0; kk < NA; ++kk) xn[kk] = *reinterpret_cast<const C *>(a + 2 * (bn + off(kk)));
        }
        // K-step outer, product and row block inner: the 3 MB accumulator chains are independent, so
        // consecutive matrix-core instructions never wait on each other's results
        AV t1[MB], t2[MB], t3[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            t1[mb] = AV{0, 0, 0, 0};
            t2[mb] = AV{0, 0, 0, 0};
            t3[mb] = AV{0, 0, 0, 0};
        }
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const T xr = x[kk].x, xi = x[kk].y, xs = xr + xi;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int f = (mb * KS + kk) * 64 + lane;
                t1[mb] = mfma16(W[f], xr, t1[mb]);
                t2[mb] = mfma16(W[FR + f], xi, t2[mb]);
                t3[mb] = mfma16(W[2 * FR + f], xs, t3[mb]);
            }
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const T yr = t1[mb][v] - t2[mb][v];
                const T yi = t3[mb][v] - t1[mb][v] - t2[mb][v];
                *reinterpret_cast<C *>(a + 2 * (b + off(4 * mb + v))) = C{yr, yi};
            }
#pragma unroll
        for (int kk = 0; kk < NA; ++kk) x[kk] = xn[kk];
        tile = next;
    }
}

// VALU form for small k: one lane per column, U (complex, row-major) in kernel arguments
struct SmallU {
    double u[2 * 64];
};
// k = 4, 5 on the vector ALUs (only for states too small for the matrix-core tiling): U in global
struct BigU {
    const double *u;
};
__device__ __forceinline__ double uget(const SmallU &m, int i) { return m.u[i]; }
__device__ __forceinline__ double uget(const BigU &m, int i) { return m.u[i]; }

template <typename T, int KLOG, int ITEMS, typename UM>
__global__ __launch_bounds__(kBlock) void k_fused_valu(T *__restrict__ a, uint64_t ncols, IndexMap map, QubitList ql, UM um)
{
    using C = typename Vec<T>::C;
    constexpr int K = 1 << KLOG;
    uint64_t off[K];
#pragma unroll
    for (int r = 0; r < K; ++r) off[r] = offset_of(r, ql);
    const uint64_t chunk = uint64_t(kBlock) * ITEMS;
    for (uint64_t base = uint64_t(blockIdx.x) * chunk + threadIdx.x; base < ncols; base += uint64_t(gridDim.x) * chunk) {
        C x[ITEMS][K];
        uint64_t b[ITEMS];
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint64_t j = base + uint64_t(it) * kBlock;
            if (j < ncols) {
                b[it] = insert_zeros(j, map);
#pragma unroll
                for (int r = 0; r < K; ++r) x[it][r] = *reinterpret_cast<const C *>(a + 2 * (b[it] + off[r]));
            }
        }
#pragma unroll
        for (int it = 0; it < ITEMS; ++it) {
            const uint64_t j = base + uint64_t(it) * kBlock;
            if (j < ncols) {
#pragma unroll
                for (int r = 0; r < K; ++r) {
                    T yr = 0, yi = 0;
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        const T ur = static_cast<T>(uget(um, 2 * (r * K + c))), ui = static_cast<T>(uget(um, 2 * (r * K + c) + 1));
                        yr += ur * x[it][c].x - ui * x[it][c].y;
                        yi += ur * x[it][c].y + ui * x[it][c].x;
                    }
                    *reinterpret_cast<C *>(a + 2 * (b[it] + off[r])) = C{yr, yi};
                }
            }
        }
    }
}

inline unsigned grid_cap(uint64_t g, uint64_t cap)
{
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return unsigned(g);
}

template <typename T>
int fused_valu_t(qsim_state *s, int k, const QubitList &ql, const IndexMap &map, const double *U, const BigU *um4)
{
    SmallU um{};
    const int K = 1 << k;
    if (k <= 3)
        for (int i = 0; i < 2 * K * K; ++i) um.u[i] = U[i];
    const uint64_t ncols = dim(s->n) >> k;
    T *a = static_cast<T *>(s->data);
    constexpr int IT = 2;
    const unsigned g = grid_cap((ncols + kBlock * IT - 1) / (kBlock * IT), 1u << 20);
    switch (k) {
    case 1: hipLaunchKernelGGL((k_fused_valu<T, 1, IT, SmallU>), dim3(g), dim3(kBlock), 0, s->stream, a, ncols, map, ql, um); break;
    case 2: hipLaunchKernelGGL((k_fused_valu<T, 2, IT, SmallU>), dim3(g), dim3(kBlock), 0, s->stream, a, ncols, map, ql, um); break;
    case 3: hipLaunchKernelGGL((k_fused_valu<T, 3, 1, SmallU>), dim3(g), dim3(kBlock), 0, s->stream, a, ncols, map, ql, um); break;
    case 4: hipLaunchKernelGGL((k_fused_valu<T, 4, 1, BigU>), dim3(g), dim3(kBlock), 0, s->stream, a, ncols, map, ql, *um4); break;
    case 5: hipLaunchKernelGGL((k_fused_valu<T, 5, 1, BigU>), dim3(g), dim3(kBlock), 0, s->stream, a, ncols, map, ql, *um4); break;
    default: return set_error(QSIM_EINVAL, "fused: k out of range");
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

}  // namespace

// the three matrices of the MFMA kernel (Ur, Ui, Ur + Ui, sums formed in FP64) in fragment order, in
// the state's precision
template <typename T>
static void build_wfrag(int k, const double *U, std::vector<T> &frag)
{
    const int K = 1 << k, KS = K / 4, MB = K / 16, FR = MB * KS * 64;
    auto M = [&](int p, int r, int c) -> double {
        const double ur = U[2 * (r * K + c)], ui = U[2 * (r * K + c) + 1];
        return p == 0 ? ur : p == 1 ? ui : ur + ui;
    };
    frag.assign(size_t(3) * FR, T(0));
    for (int p = 0; p < 3; ++p)
        for (int mb = 0; mb < MB; ++mb)
            for (int kk = 0; kk < KS; ++kk)
                for (int l = 0; l < 64; ++l)
                    frag[size_t(p) * FR + size_t(mb * KS + kk) * 64 + l] =
                        static_cast<T>(M(p, 16 * mb + l % 16, amp_of<T>(kk, l / 16)));
}

size_t wfrag_bytes(int k, int dtype) { return size_t(3) << (2 * k) << (dtype == QSIM_C128 ? 3 : 2); }

int build_wfrag_host(int k, int dtype, const double *U, void *host_out)
{
    if (dtype == QSIM_C128) {
        std::vector<double> f;
        build_wfrag<double>(k, U, f);
        memcpy(host_out, f.data(), f.size() * sizeof(double));
    } else {
        std::vector<float> f;
        build_wfrag<float>(k, U, f);
        memcpy(host_out, f.data(), f.size() * sizeof(float));
    }
    return QSIM_OK;
}

// launch a fused gate whose W fragments are already in device memory (k = 4, 5)
int launch_fused_mfma(qsim_state *s, int k, const int *qubits, const void *dev_wfrag)
{
    QubitList ql{};
    ql.k = k;
    uint64_t mask = 0;
    for (int i = 0; i < k; ++i) {
        ql.q[i] = qubits[i];
        mask |= uint64_t(1) << qubits[i];
    }
    const IndexMap map = make_index_map(mask, 0);
    const uint64_t ncols = dim(s->n) >> k;
    if (ncols % 16) return set_error(QSIM_EUNSUPPORTED, "fused: the matrix-core form needs n >= k + 4");
    const uint64_t ntiles = ncols / 16;
    // persistent-style grid: each workgroup stages W once and walks many column tiles
    const unsigned g = grid_cap((ntiles + 3) / 4, 256 * 8);
    if (s->dtype == QSIM_C128) {
        double *a = static_cast<double *>(s->data);
        if (k == 4)
            hipLaunchKernelGGL((k_fused_mfma<double, 4>), dim3(g), dim3(kBlock), 0, s->stream, a, ntiles, map, ql,
                               static_cast<const double *>(dev_wfrag));
        else
            hipLaunchKernelGGL((k_fused_mfma<double, 5>), dim3(g), dim3(kBlock), 0, s->stream, a, ntiles, map, ql,
                               static_cast<const double *>(dev_wfrag));
    } else {
        float *a = static_cast<float *>(s->data);
        if (k == 4)
            hipLaunchKernelGGL((k_fused_mfma<float, 4>), dim3(g), dim3(kBlock), 0, s->stream, a, ntiles, map, ql,
                               static_cast<const float *>(dev_wfrag));
        else
            hipLaunchKernelGGL((k_fused_mfma<float, 5>), dim3(g), dim3(kBlock), 0, s->stream, a, ntiles, map, ql,
                               static_cast<const float *>(dev_wfrag));
    }
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

// U: host pointer for k <= 3; for k = 4, 5 a device pointer to 2^(2k+1) doubles
int launch_fused_valu(qsim_state *s, int k, const int *qubits, const double *U)
{
    QubitList ql{};
    ql.k = k;
    uint64_t mask = 0;
    for (int i = 0; i < k; ++i) {
        ql.q[i] = qubits[i];
        mask |= uint64_t(1) << qubits[i];
    }
    const IndexMap map = make_index_map(mask, 0);
    BigU big{U};
    return s->dtype == QSIM_C128 ? fused_valu_t<double>(s, k, ql, map, U, &big) : fused_valu_t<float>(s, k, ql, map, U, &big);
}

// C-ABI entry: matrices staged through the state's small device buffer
int launch_fused(qsim_state *s, int k, const int *qubits, const double *U)
{
    const bool mfma = k >= 4 && s->n >= k + 4;
    if (k <= 3) return launch_fused_valu(s, k, qubits, U);
    // the matrix staging area sits after the reduction partials in the state's scratch buffer;
    // stream order keeps it from being overwritten while an earlier fused launch still reads it
    void *dev = reinterpret_cast<unsigned char *>(s->scratch) + (size_t(kScratchDoubles) * 8 - 64 * 1024);
    if (!mfma) {  // k = 4, 5 on a state too small for the matrix-core tiling
        QSIM_HIP(hipMemcpyAsync(dev, U, sizeof(double) * (size_t(2) << (2 * k)), hipMemcpyHostToDevice, s->stream));
        QSIM_HIP(hipStreamSynchronize(s->stream));
        return launch_fused_valu(s, k, qubits, static_cast<const double *>(dev));
    }
    const size_t bytes = wfrag_bytes(k, s->dtype);
    std::vector<unsigned char> host(bytes);
    build_wfrag_host(k, s->dtype, U, host.data());
    QSIM_HIP(hipMemcpyAsync(dev, host.data(), bytes, hipMemcpyHostToDevice, s->stream));
    // the host copy lives on this stack frame: wait for the copy before returning
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return launch_fused_mfma(s, k, qubits, dev);
}

}  // namespace qsim
