// Internal declarations of libqsim (host and device). Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qsim.h"

namespace qsim {

// ---------------------------------------------------------------------------------------------
// Error handling: thread-local message + return code
// ---------------------------------------------------------------------------------------------
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);

#define QSIM_HIP(call)                                                                                       \
    do {                                                                                                     \
        hipError_t e__ = (call);                                                                             \
        if (e__ != hipSuccess) return ::qsim::hip_error(e__, #call);                                          \
    } while (0)

// ---------------------------------------------------------------------------------------------
// State
// ---------------------------------------------------------------------------------------------
}  // namespace qsim

struct qsim_state {
    int n = 0;
    int dtype = QSIM_C128;
    void *data = nullptr;       // 2^n amplitudes, interleaved
    bool owned = false;
    hipStream_t stream = nullptr;
    int device = 0;
    double *scratch = nullptr;  // small FP64 reduction buffer (owned), QSIM_SCRATCH_DOUBLES
    // per-state HIP graph cache of the last plan executed with use_graph
    const void *graph_plan = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace qsim {

constexpr int kScratchDoubles = 1 << 18;  // 2 MiB of FP64 partials per state

inline size_t amp_bytes(int dtype) { return dtype == QSIM_C128 ? 16 : 8; }
__host__ __device__ inline uint64_t dim(int n) { return uint64_t(1) << n; }

// ---------------------------------------------------------------------------------------------
// Index maps: a gate acting on the qubits P = {p_0 < p_1 < ... < p_{m-1}} (target(s) + controls)
// enumerates j in [0, 2^(n-m)) and forms the base index by inserting a 0 bit at every p_s
// (ascending), then OR-ing `set` (the control bits that must be 1).
// ---------------------------------------------------------------------------------------------
struct IndexMap {
    uint64_t set;       // OR-ed into the base index
    uint64_t posmask;   // positions of the inserted zero bits
    int32_t npos;       // number of inserted zero bits (popcount of posmask)
    int32_t p0;         // lowest inserted position (64 if none)
    uint64_t lo[3];     // npos <= 3: 2^p - 1 for the inserted positions p, ascending; all ones past npos
};

IndexMap make_index_map(uint64_t posmask, uint64_t set);

// Insert a zero bit at every position of m.posmask (ascending) into j, then OR m.set. The positions
// are walked with count-trailing-zeros on the (wave-uniform) mask: no memory access in the loop.
__device__ __forceinline__ uint64_t insert_zeros(uint64_t j, const IndexMap &m)
{
    uint64_t pm = m.posmask;
    while (pm) {
        const int p = __builtin_ctzll(pm);
        pm &= pm - 1;
        const uint64_t lo = j & ((uint64_t(1) << p) - 1);
        j = lo | ((j ^ lo) << 1);
    }
    return j | m.set;
}

// The same for m.npos <= 3 (a target with up to two controls) in three fixed steps, without a loop
// (an all-ones mask leaves j unchanged)
__device__ __forceinline__ uint64_t insert_zeros3(uint64_t j, const IndexMap &m)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint64_t lo = j & m.lo[k];
        j = lo | ((j ^ lo) << 1);
    }
    return j | m.set;
}

// 2x2 complex matrix in kernel arguments (FP64 always; c64 kernels round at use)
struct Mat2 {
    double m[8];
};

// ---------------------------------------------------------------------------------------------
// Kernel launchers (sweep kernels): all asynchronous on `st`
// ---------------------------------------------------------------------------------------------
// Values: the factors are given; Angles: factor e^{i c} for each angle c, sin and cos in FP64 on the
// device; Pow2: a phase factor e^{i s 2 pi / 2^k} with s = c[0] (+1 or -1) and k = c[1], the angle
// itself formed on the device in FP64 (an exact power-of-two scaling of the FP64 value of 2 pi)
enum class DiagMode : int { Values = 0, Angles = 1, Pow2 = 2 };

// the FP64 value of 2 pi (the double nearest to it)
constexpr double kTwoPi = 6.283185307179586;

// ops whose only effect is the phase factor diag(1, e^{i theta}) on the target
inline bool phase_op(int op) { return op == QSIM_OP_PHASE || op == QSIM_OP_RK || op == QSIM_OP_RKDG; }
// theta of a phase op, in FP64 on the host (where gates are multiplied into fused matrices)
double phase_angle(const qsim_gate &g);

// general 2x2 on target (controls in map.set); map positions = sorted(controls U {target})
int launch_general(qsim_state *s, const IndexMap &map, int target, const Mat2 &u);
// multiply the amplitudes selected by map (bits set in map.set are 1) by one factor:
// either the complex value (c[0], c[1]) or e^{i c[0]} evaluated on the device in FP64
int launch_phase(qsim_state *s, const IndexMap &map, const double c[2], DiagMode mode);
// diag(d0, d1) on target for indices whose control bits are 1; map positions = sorted(controls)
int launch_diag(qsim_state *s, const IndexMap &map, int target, const double d[4], DiagMode mode);
// swap a(i) <-> a(i ^ flip) for i = insert(j) | map.set
int launch_swap(qsim_state *s, const IndexMap &map, uint64_t flip);
// fill with |x>
int launch_set_basis(qsim_state *s, uint64_t x);
// |x>|z> -> |x>|z XOR (y^x mod G)> (arguments checked by the caller)
int launch_modexp(qsim_state *s, int x_first, int x_qubits, int f_first, uint64_t y, uint64_t G);
// dense k-qubit gate
int launch_fused(qsim_state *s, int k, const int *qubits, const double *U);

// reductions
int run_norm(qsim_state *s, double *host_out);
int launch_probs(qsim_state *s, double *dev_out, uint64_t first, uint64_t count);
int run_marginals(qsim_state *s, double *host_out);
int launch_scale(qsim_state *s, const double *dev_factor);
// Renormalisation steps of plans (Eq. STAT1), asynchronous on the state's stream. launch_norm_into:
// *out = FP64 sum of |a|^2 over the state, through `partial` (kAuxLevel2 doubles). launch_renorm_scale:
// the state times 1/sqrt(*norm), unchanged when *norm is not positive. launch_sum_array: *out = the sum
// of x[0..count) in a fixed order, through `level2` (kAuxLevel2 doubles).
constexpr int kReduceMaxGrid = 4096;
constexpr int kAuxLevel2 = 4096;
int launch_norm_into(qsim_state *s, double *partial, double *out);
int launch_renorm_scale(qsim_state *s, const double *norm);
int launch_sum_array(const double *x, uint64_t count, double *level2, double *out, hipStream_t stream);
int run_renormalize(qsim_state *s, double *norm_before);
int run_sample(qsim_state *s, int64_t shots, const double *uniforms, uint64_t *out);

// gate validation / classification shared by the C ABI and the planner
enum class Kind : int { General = 0, Diag = 1, Phase1 = 2, Swap = 3 };
Kind classify(const double u[8]);
int gate_matrix(const qsim_gate &g, double u[8]);  // FP64 matrix of a named gate (host)
int apply_gate_record(qsim_state *s, const qsim_gate &g);
int validate_gate(const qsim_gate &g, int n);

}  // namespace qsim
