// The LDS-staged pass kernels (templates) and their launch helpers. Included by the translation units
// that instantiate them (staged_k128.hip, staged_k128w.hip, staged_k64.hip, staged_k64w.hip), which
// the build compiles in parallel.
#pragma once

#include "staged_device.h"

namespace qsim {
namespace staged {
namespace {

// Kernel instantiations per pass (MODE): 0 reads the state and folds no renormalisation; 1 folds a
// renormalisation point (scales its loads and/or sums the norm of its stores); 2 is the first pass of a
// run from |0...0>, which generates the initial state instead of loading it (and may sum the norm).
// Passes of mode 0 thus compile without the code of the other two, which would cost registers.
//
// One pass over the whole state: one workgroup per block of 2^(LOG_E + LOG_T) amplitudes. (A
// persistent grid that prefetches each workgroup's next block into registers while the current one
// is processed measured slower on gfx950: the extra registers and the wait for the previous block's
// stores cost more than the overlap gained.)
template <typename T, int LOG_E, int LOG_T, int MINW, int MODE>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_staged(T *__restrict__ a, const SPass *__restrict__ passp,
                                                             const SStage *__restrict__ stages, const SRound *__restrict__ rounds,
                                                             const SOp *__restrict__ ops, const SBlk *__restrict__ blks,
                                                             const double *scale, double *norm)
{
    using C = typename Vec<T>::C;
    __shared__ C lds[lds_slots<T>(LOG_E + LOG_T)];
    const SPass pass = ldc<SPass>(as_const(passp));
    run_block<T, LOG_E, LOG_T, MODE != 0>(a, pass, blockIdx.x, as_const(stages), as_const(rounds), as_const(ops), as_const(blks), lds,
                               MODE == 2, SEdge{scale, norm});
}

// The same pass with a buffer of half the block (every LDS round trip in two halves): twice the
// workgroups per CU where LDS, not registers, bounds the occupancy.
template <typename T, int LOG_E, int LOG_T, int MINW, int MODE>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_staged_half(T *__restrict__ a, const SPass *__restrict__ passp,
                                                                  const SStage *__restrict__ stages,
                                                                  const SRound *__restrict__ rounds,
                                                                  const SOp *__restrict__ ops, const SBlk *__restrict__ blks,
                                                                  const double *scale, double *norm)
{
    using C = typename Vec<T>::C;
    __shared__ C lds[lds_slots<T>(LOG_E + LOG_T - 1)];
    const SPass pass = ldc<SPass>(as_const(passp));
    run_block_half<T, LOG_E, LOG_T, MODE != 0>(a, pass, blockIdx.x, as_const(stages), as_const(rounds), as_const(ops), as_const(blks), lds,
                                    MODE == 2, SEdge{scale, norm});
}

// The half-buffer pass when every split is at a wave position: uniform split branches, and the block
// fits in 128 VGPRs, so four 256-thread workgroups share a CU.
template <typename T, int LOG_E, int LOG_T, int MINW, int MODE>
__global__ __launch_bounds__(1 << LOG_T, MINW) void k_staged_wave(T *__restrict__ a, const SPass *__restrict__ passp,
                                                                  const SStage *__restrict__ stages,
                                                                  const SRound *__restrict__ rounds,
                                                                  const SOp *__restrict__ ops, const SBlk *__restrict__ blks,
                                                                  const double *scale, double *norm)
{
    using C = typename Vec<T>::C;
    __shared__ C lds[lds_slots<T>(LOG_E + LOG_T - 1)];
    const SPass pass = ldc<SPass>(as_const(passp));
    run_block_wave<T, LOG_E, LOG_T, MODE != 0>(a, pass, blockIdx.x, as_const(stages), as_const(rounds), as_const(ops), as_const(blks), lds,
                                    MODE == 2, SEdge{scale, norm});
}

// One launch of a pass kernel (full, half or wave form) in the mode the launch asks for.
template <typename T, int LE, int LT, int MW> void launch_full(const PassLaunch &a)
{
    const dim3 grid(a.grid), block(1 << LT);
    T *d = static_cast<T *>(a.data);
    if (a.mode == 0)
        hipLaunchKernelGGL((k_staged<T, LE, LT, MW, 0>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops, a.blks,
                           nullptr, nullptr);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_staged<T, LE, LT, MW, 1>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops, a.blks,
                           a.scale, a.norm);
    else
        hipLaunchKernelGGL((k_staged<T, LE, LT, MW, 2>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops, a.blks,
                           a.scale, a.norm);
}
template <typename T, int LE, int LT, int MW> void launch_half(const PassLaunch &a)
{
    const dim3 grid(a.grid), block(1 << LT);
    T *d = static_cast<T *>(a.data);
    if (a.mode == 0)
        hipLaunchKernelGGL((k_staged_half<T, LE, LT, MW, 0>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, nullptr, nullptr);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_staged_half<T, LE, LT, MW, 1>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, a.scale, a.norm);
    else
        hipLaunchKernelGGL((k_staged_half<T, LE, LT, MW, 2>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, a.scale, a.norm);
}
template <typename T, int LE, int LT, int MW> void launch_wave(const PassLaunch &a)
{
    const dim3 grid(a.grid), block(1 << LT);
    T *d = static_cast<T *>(a.data);
    if (a.mode == 0)
        hipLaunchKernelGGL((k_staged_wave<T, LE, LT, MW, 0>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, nullptr, nullptr);
    else if (a.mode == 1)
        hipLaunchKernelGGL((k_staged_wave<T, LE, LT, MW, 1>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, a.scale, a.norm);
    else
        hipLaunchKernelGGL((k_staged_wave<T, LE, LT, MW, 2>), grid, block, 0, a.stream, d, a.pass, a.stages, a.rounds, a.ops,
                           a.blks, a.scale, a.norm);
}

}  // namespace
}  // namespace staged
}  // namespace qsim
