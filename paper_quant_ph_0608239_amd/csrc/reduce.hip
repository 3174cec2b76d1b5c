// FP64 reductions over the state (both dtypes accumulate in FP64):
//   norm sum_i |a_i|^2 (Eq. STAT1), probabilities |a_i|^2 (Sec. II.A), qubit expectation values
//   <Q_q> = sum_k |a_k|^2 bit_q(k) (Eq. Shor7), renormalisation, and inverse-CDF sampling.
// Every reduction uses a grid fixed by the state size and fixed-order tree sums, so results are
// deterministic run to run.
#include <mutex>
#include <type_traits>

#include "qsim_internal.h"

namespace qsim {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
    return v;  // valid in lane 0
}

__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) lds[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
        for (int k = 0; k < kWaves; ++k) r += lds[k];
    }
    __syncthreads();
    return r;  // valid in thread 0
}

template <typename T> __device__ __forceinline__ double sq(T r, T i)
{
    const double x = double(r), y = double(i);
    return x * x + y * y;
}

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
constexpr int kScaleWords = 4;

// grid-stride partial sums of |a|^2; every lane reads 16-byte words (one complex128 amplitude or two
// complex64 ones) with nontemporal loads (a state far larger than the caches is streamed once)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm_partial(const T *__restrict__ a, uint64_t namps, double *__restrict__ partial)
{
    __shared__ double lds[kWaves];
    double acc = 0.0;
    if constexpr (sizeof(T) == 8) {
        for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < namps; i += uint64_t(gridDim.x) * kBlock) {
            const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v *>(a) + i);
            acc += sq(v.x, v.y);
        }
    } else {
        const uint64_t nq = namps / 2;
        for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < nq; i += uint64_t(gridDim.x) * kBlock) {
            const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(a) + i);
            acc += sq(v.x, v.y) + sq(v.z, v.w);
        }
        if (namps % 2 && blockIdx.x == 0 && threadIdx.x == 0) acc += sq(a[2 * (namps - 1)], a[2 * (namps - 1) + 1]);
    }
    const double r = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(kBlock) void k_sum_final(const double *__restrict__ partial, int count, int stride, int nvec,
                                                      double *__restrict__ out)
{
    // out[v] = sum_b partial[b * stride + v], v < nvec, in a fixed order
    __shared__ double lds[kWaves];
    for (int v = 0; v < nvec; ++v) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < count; b += kBlock) acc += partial[size_t(b) * stride + v];
        const double r = block_sum(acc, lds);
        if (threadIdx.x == 0) out[v] = r;
    }
}

// grid-stride partial sums of an FP64 array (the per-block partials of a pass that accumulated the norm)
__global__ __launch_bounds__(kBlock) void k_sum_partial(const double *__restrict__ x, uint64_t count, double *__restrict__ partial)
{
    __shared__ double lds[kWaves];
    double acc = 0.0;
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += uint64_t(gridDim.x) * kBlock) acc += x[i];
    const double r = block_sum(acc, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_probs(const T *__restrict__ a, double *__restrict__ p, uint64_t first,
                                                 uint64_t count)
{
    for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += uint64_t(gridDim.x) * kBlock) {
        const uint64_t g = first + i;
        p[i] = sq(a[2 * g], a[2 * g + 1]);
    }
}

// <Q_q> partial sums. A block walks tiles of kTile consecutive amplitudes; thread t reads
// amplitude tile_base + r * kBlock + t (r < kRows), so the index bits below log2(kBlock) are the
// thread's own bits, the next log2(kRows) bits are r, and all higher bits are the tile's.
constexpr int kRows = 8;
constexpr int kTile = kBlock * kRows;  // 2048 amplitudes, 11 index bits
constexpr int kLowBits = 8, kRowBits = 3, kTileBits = 11;
constexpr int kMaxQ = QSIM_MAX_QUBITS;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_marg_partial(const T *__restrict__ a, int n, uint64_t ntiles,
                                                        double *__restrict__ partial /* [grid][n + 1] */)
{
    __shared__ double lds[kWaves];
    double own = 0.0;                 // sum of every p this thread read -> low bits via threadIdx
    double row[kRows] = {};           // per row r -> bits kLowBits .. kLowBits + kRowBits - 1
    double hi[kMaxQ - kTileBits] = {};  // per high bit, accumulated per tile
    const uint64_t N = dim(n);
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        double tile = 0.0;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
            const uint64_t i = t * kTile + uint64_t(r) * kBlock + threadIdx.x;
            const double p = (i < N) ? sq(a[2 * i], a[2 * i + 1]) : 0.0;
            row[r] += p;
            tile += p;
        }
        own += tile;
#pragma unroll
        for (int q = 0; q < kMaxQ - kTileBits; ++q)
            if ((t >> q) & 1) hi[q] += tile;
    }
    // bit q of the index, by range of q
    for (int q = 0; q < n; ++q) {
        double v;
        if (q < kLowBits)
            v = ((threadIdx.x >> q) & 1) ? own : 0.0;
        else if (q < kTileBits) {
            v = 0.0;
#pragma unroll
            for (int r = 0; r < kRows; ++r)
                if ((r >> (q - kLowBits)) & 1) v += row[r];
        } else {
            v = 0.0;
#pragma unroll
            for (int h = 0; h < kMaxQ - kTileBits; ++h)
                if (h == q - kTileBits) v = hi[h];
        }
        const double r = block_sum(v, lds);
        if (threadIdx.x == 0) partial[size_t(blockIdx.x) * (n + 1) + q] = r;
    }
    const double r = block_sum(own, lds);
    if (threadIdx.x == 0) partial[size_t(blockIdx.x) * (n + 1) + n] = r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_scale(T *__restrict__ a, uint64_t namps, const double *__restrict__ factor_src,
                                                 int mode, double *__restrict__ norm_out)
{
    // mode 0: factor = factor_src[0]; mode 1: factor = 1 / sqrt(factor_src[0]) (FP64); mode 2: the same
    // when factor_src[0] > 0 and 1 (the state is left as it is) otherwise. norm_out (may be NULL)
    // receives factor_src[0]. Lanes move 16-byte words with nontemporal loads and stores.
    const double src = factor_src[0];
    const double f64 = mode == 0 ? src : (mode == 2 && !(src > 0.0)) ? 1.0 : 1.0 / sqrt(src);
    if (norm_out && blockIdx.x == 0 && threadIdx.x == 0) *norm_out = src;
    const T f = static_cast<T>(f64);
    // each lane keeps kScaleWords 16-byte loads in flight before it multiplies and stores them
    using W = typename std::conditional<sizeof(T) == 8, d2v, f4v>::type;
    const uint64_t nw = sizeof(T) == 8 ? namps : namps / 2;
    W *aw = reinterpret_cast<W *>(a);
    const uint64_t step = uint64_t(gridDim.x) * kBlock * kScaleWords;
    for (uint64_t b = uint64_t(blockIdx.x) * kBlock * kScaleWords + threadIdx.x; b < nw; b += step) {
        W v[kScaleWords];
#pragma unroll
        for (int k = 0; k < kScaleWords; ++k)
            if (b + uint64_t(k) * kBlock < nw) v[k] = __builtin_nontemporal_load(aw + b + uint64_t(k) * kBlock);
#pragma unroll
        for (int k = 0; k < kScaleWords; ++k) {
            if (b + uint64_t(k) * kBlock < nw) {
                v[k] *= f;
                __builtin_nontemporal_store(v[k], aw + b + uint64_t(k) * kBlock);
            }
        }
    }
    if constexpr (sizeof(T) == 4) {
        if (namps % 2 && blockIdx.x == 0 && threadIdx.x == 0) {
            a[2 * (namps - 1)] *= f;
            a[2 * (namps - 1) + 1] *= f;
        }
    }
}

// chunk sums of |a|^2 over fixed chunks of 2^c amplitudes (for sampling)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_chunk_sums(const T *__restrict__ a, uint64_t chunk, uint64_t nchunks,
                                                      double *__restrict__ out)
{
    __shared__ double lds[kWaves];
    for (uint64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        double acc = 0.0;
        for (uint64_t i = threadIdx.x; i < chunk; i += kBlock) {
            const uint64_t g = c * chunk + i;
            acc += sq(a[2 * g], a[2 * g + 1]);
        }
        const double r = block_sum(acc, lds);
        if (threadIdx.x == 0) out[c] = r;
    }
}

// one thread per shot: walk the amplitudes of its chunk in index order until the running sum
// passes the target value
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sample_in_chunk(const T *__restrict__ a, uint64_t chunk,
                                                           const uint64_t *__restrict__ shot_chunk,
                                                           const double *__restrict__ shot_rem, int64_t shots,
                                                           uint64_t *__restrict__ out)
{
    const int64_t s = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (s >= shots) return;
    const uint64_t c = shot_chunk[s];
    const double target = shot_rem[s];
    double run = 0.0;
    uint64_t pick = c * chunk;  // rounding can leave target >= run: fall back to the last nonzero
    bool found = false;
    for (uint64_t i = 0; i < chunk && !found; ++i) {
        const uint64_t g = c * chunk + i;
        const double p = sq(a[2 * g], a[2 * g + 1]);
        if (p > 0.0) {
            run += p;
            pick = g;
            found = target < run;
        }
    }
    out[s] = pick;
}

inline unsigned reduce_grid(uint64_t items)
{
    uint64_t g = (items + kBlock * 8 - 1) / (kBlock * 8);
    if (g < 1) g = 1;
    if (g > kReduceMaxGrid) g = kReduceMaxGrid;
    return unsigned(g);
}

}  // namespace

static_assert(kReduceMaxGrid <= kAuxLevel2, "a level-2 buffer holds one partial per reduction workgroup");

int launch_norm_into(qsim_state *s, double *partial, double *out)
{
    const uint64_t N = dim(s->n);
    const unsigned g = reduce_grid(s->dtype == QSIM_C128 ? N : N / 2 + 1);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_norm_partial<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const double *>(s->data), N,
                           partial);
    else
        hipLaunchKernelGGL(k_norm_partial<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const float *>(s->data), N,
                           partial);
    QSIM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s->stream, partial, int(g), 1, 1, out);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

static int norm_to_scratch(qsim_state *s) { return launch_norm_into(s, s->scratch + 8, s->scratch); }

int launch_sum_array(const double *x, uint64_t count, double *level2, double *out, hipStream_t stream)
{
    const unsigned g = reduce_grid(count);
    hipLaunchKernelGGL(k_sum_partial, dim3(g), dim3(kBlock), 0, stream, x, count, level2);
    QSIM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, stream, level2, int(g), 1, 1, out);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int launch_renorm_scale(qsim_state *s, const double *norm)
{
    const uint64_t N = dim(s->n);
    const unsigned g = reduce_grid(N);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<double *>(s->data), N, norm, 2,
                           nullptr);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<float *>(s->data), N, norm, 2,
                           nullptr);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int run_norm(qsim_state *s, double *host_out)
{
    int rc = norm_to_scratch(s);
    if (rc) return rc;
    QSIM_HIP(hipMemcpyAsync(host_out, s->scratch, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

int launch_probs(qsim_state *s, double *dev_out, uint64_t first, uint64_t count)
{
    const unsigned g = reduce_grid(count * 2);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_probs<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const double *>(s->data), dev_out,
                           first, count);
    else
        hipLaunchKernelGGL(k_probs<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const float *>(s->data), dev_out,
                           first, count);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int run_marginals(qsim_state *s, double *host_out)
{
    const int n = s->n;
    const uint64_t ntiles = (dim(n) + kTile - 1) / kTile;
    uint64_t g = ntiles;
    if (g > 2048) g = 2048;
    double *partial = s->scratch + 64;
    if (g * (n + 1) + 64 > uint64_t(kScratchDoubles)) return set_error(QSIM_EINVAL, "marginals: scratch too small");
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_marg_partial<double>, dim3(unsigned(g)), dim3(kBlock), 0, s->stream,
                           static_cast<const double *>(s->data), n, ntiles, partial);
    else
        hipLaunchKernelGGL(k_marg_partial<float>, dim3(unsigned(g)), dim3(kBlock), 0, s->stream,
                           static_cast<const float *>(s->data), n, ntiles, partial);
    QSIM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s->stream, partial, int(g), n + 1, n, s->scratch);
    QSIM_HIP(hipGetLastError());
    QSIM_HIP(hipMemcpyAsync(host_out, s->scratch, sizeof(double) * n, hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

int launch_scale(qsim_state *s, const double *dev_factor)
{
    const uint64_t N = dim(s->n);
    const unsigned g = reduce_grid(N);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<double *>(s->data), N, dev_factor, 0,
                           nullptr);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<float *>(s->data), N, dev_factor, 0,
                           nullptr);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}

int run_renormalize(qsim_state *s, double *norm_before)
{
    int rc = norm_to_scratch(s);
    if (rc) return rc;
    double nrm = 0.0;
    QSIM_HIP(hipMemcpyAsync(&nrm, s->scratch, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    if (!(nrm > 0.0)) return set_error(QSIM_EINVAL, "renormalize: the state has zero norm");
    const uint64_t N = dim(s->n);
    const unsigned g = reduce_grid(N);
    // factor 1/sqrt(norm) evaluated in FP64 on the device from the norm left in scratch[0]
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<double *>(s->data), N, s->scratch, 1,
                           nullptr);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<float *>(s->data), N, s->scratch, 1,
                           nullptr);
    QSIM_HIP(hipGetLastError());
    QSIM_HIP(hipStreamSynchronize(s->stream));
    if (norm_before) *norm_before = nrm;
    return QSIM_OK;
}

namespace {
// device buffers of one sampling call: freed on every return path, after the state's stream has
// drained (a failed call may still have work in flight that reads them)
struct SampleBuffers {
    hipStream_t stream = nullptr;
    double *sums = nullptr, *rem = nullptr;
    uint64_t *chunk = nullptr, *out = nullptr;
    ~SampleBuffers()
    {
        if (sums || rem || chunk || out) (void)hipStreamSynchronize(stream);
        if (sums) (void)hipFree(sums);
        if (rem) (void)hipFree(rem);
        if (chunk) (void)hipFree(chunk);
        if (out) (void)hipFree(out);
    }
};
}  // namespace

int run_sample(qsim_state *s, int64_t shots, const double *uniforms, uint64_t *out)
{
    // two levels: FP64 sums over fixed chunks of 2^c amplitudes (device), a cumulative walk over the
    // chunk sums per shot (host, FP64, in index order), then the walk inside the chosen chunk (device)
    for (int64_t i = 0; i < shots; ++i)
        if (!(uniforms[i] >= 0.0 && uniforms[i] < 1.0)) return set_error(QSIM_EINVAL, "sample: uniforms must lie in [0, 1)");
    const int n = s->n;
    const int c = n > 12 ? 12 : n;
    const uint64_t chunk = uint64_t(1) << c;
    const uint64_t nchunks = dim(n) >> c;
    std::vector<double> sums(nchunks);
    SampleBuffers b;
    b.stream = s->stream;
    QSIM_HIP(hipMalloc((void **)&b.sums, sizeof(double) * nchunks));
    const unsigned g = unsigned(nchunks < 8192 ? nchunks : 8192);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_chunk_sums<double>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const double *>(s->data), chunk,
                           nchunks, b.sums);
    else
        hipLaunchKernelGGL(k_chunk_sums<float>, dim3(g), dim3(kBlock), 0, s->stream, static_cast<const float *>(s->data), chunk,
                           nchunks, b.sums);
    QSIM_HIP(hipGetLastError());
    QSIM_HIP(hipMemcpyAsync(sums.data(), b.sums, sizeof(double) * nchunks, hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    double total = 0.0;
    for (double v : sums) total += v;
    std::vector<double> cum(nchunks);
    double run = 0.0;
    for (uint64_t k = 0; k < nchunks; ++k) {
        run += sums[k];
        cum[k] = run;
    }
    std::vector<uint64_t> sc(shots);
    std::vector<double> rem(shots);
    for (int64_t i = 0; i < shots; ++i) {
        const double target = uniforms[i] * total;
        uint64_t lo = 0, hi = nchunks - 1;  // first chunk with cum > target
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            if (cum[mid] > target) hi = mid; else lo = mid + 1;
        }
        // skip empty chunks at the end of the walk
        while (lo + 1 < nchunks && sums[lo] == 0.0) ++lo;
        sc[i] = lo;
        rem[i] = target - (lo ? cum[lo - 1] : 0.0);
    }
    QSIM_HIP(hipMalloc((void **)&b.chunk, sizeof(uint64_t) * shots));
    QSIM_HIP(hipMalloc((void **)&b.rem, sizeof(double) * shots));
    QSIM_HIP(hipMalloc((void **)&b.out, sizeof(uint64_t) * shots));
    QSIM_HIP(hipMemcpyAsync(b.chunk, sc.data(), sizeof(uint64_t) * shots, hipMemcpyHostToDevice, s->stream));
    QSIM_HIP(hipMemcpyAsync(b.rem, rem.data(), sizeof(double) * shots, hipMemcpyHostToDevice, s->stream));
    const unsigned gs = unsigned((shots + kBlock - 1) / kBlock);
    if (s->dtype == QSIM_C128)
        hipLaunchKernelGGL(k_sample_in_chunk<double>, dim3(gs), dim3(kBlock), 0, s->stream, static_cast<const double *>(s->data),
                           chunk, b.chunk, b.rem, shots, b.out);
    else
        hipLaunchKernelGGL(k_sample_in_chunk<float>, dim3(gs), dim3(kBlock), 0, s->stream, static_cast<const float *>(s->data),
                           chunk, b.chunk, b.rem, shots, b.out);
    QSIM_HIP(hipGetLastError());
    QSIM_HIP(hipMemcpyAsync(out, b.out, sizeof(uint64_t) * shots, hipMemcpyDeviceToHost, s->stream));
    QSIM_HIP(hipStreamSynchronize(s->stream));
    return QSIM_OK;
}

// ---- allocation-free renormalisation ---------------------------------------------------------------
// For callers that cannot allocate device memory, the norm partials (at most one per block of the
// fixed reduction grid, 4096) and the norm live in a file-scope device array instead of the state's
// scratch buffer: one copy per device, held until the process ends. In host code the array's name is
// only a stand-in; its device address is taken once per device with hipGetSymbolAddress and used
// everywhere host code needs the array.
constexpr int kNoAllocPartials = 4096;
constexpr int kNoAllocDoubles = 8 + kNoAllocPartials;
static __device__ __align__(256) double noalloc_scratch[kNoAllocDoubles];

constexpr int kNoAllocMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double *g_noalloc_ptr[kNoAllocMaxDevices] = {};

// the device address of this device's copy of the array (taken on the first call on the device, with
// that device current)
static int noalloc_scratch_ptr(double **out)
{
    int dev = 0;
    QSIM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocMaxDevices) return set_error(QSIM_EUNSUPPORTED, "renormalize_noalloc: device index too large");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        QSIM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
        if (!p) return set_error(QSIM_EDEVICE, "renormalize_noalloc: no device address for the scratch array");
        g_noalloc_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_noalloc_ptr[dev];
    return QSIM_OK;
}

}  // namespace qsim

extern "C" int qsim_renormalize_noalloc(void *dev_amps, int n, int dtype, void *hip_stream, double *dev_norm_before)
{
    using namespace qsim;
    if (!dev_amps) return set_error(QSIM_EINVAL, "renormalize_noalloc: dev_amps is NULL");
    if (reinterpret_cast<uintptr_t>(dev_amps) % 16) return set_error(QSIM_EINVAL, "renormalize_noalloc: dev_amps must be 16-byte aligned");
    if (n < 1 || n > QSIM_MAX_QUBITS) return set_error(QSIM_EINVAL, "renormalize_noalloc: n out of range (1..QSIM_MAX_QUBITS)");
    if (dtype != QSIM_C64 && dtype != QSIM_C128) return set_error(QSIM_EINVAL, "renormalize_noalloc: unknown dtype");
    const uint64_t N = dim(n);
    const unsigned g = reduce_grid(dtype == QSIM_C128 ? N : N / 2 + 1);
    if (g > unsigned(kNoAllocPartials)) return set_error(QSIM_EINVAL, "renormalize_noalloc: more partial sums than the scratch holds");
    double *scr = nullptr;
    if (int rc = noalloc_scratch_ptr(&scr)) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double *partial = scr + 8;
    // the same kernels and grid as qsim_renormalize: the partials are overwritten, nothing needs clearing
    if (dtype == QSIM_C128)
        hipLaunchKernelGGL(k_norm_partial<double>, dim3(g), dim3(kBlock), 0, st, static_cast<const double *>(dev_amps), N, partial);
    else
        hipLaunchKernelGGL(k_norm_partial<float>, dim3(g), dim3(kBlock), 0, st, static_cast<const float *>(dev_amps), N, partial);
    QSIM_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, st, partial, int(g), 1, 1, scr);
    QSIM_HIP(hipGetLastError());
    const unsigned gs = reduce_grid(N);
    if (dtype == QSIM_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(gs), dim3(kBlock), 0, st, static_cast<double *>(dev_amps), N, scr, 2, dev_norm_before);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(gs), dim3(kBlock), 0, st, static_cast<float *>(dev_amps), N, scr, 2, dev_norm_before);
    QSIM_HIP(hipGetLastError());
    return QSIM_OK;
}
