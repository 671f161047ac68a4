// One KDK step of a box class as ONE persistent cooperative launch: the fused particle step
// of every brick, then the three Poisson passes of the next force, separated by grid-wide
// barriers (the dependencies are per box, but a box's passes need all of its bricks and all
// of its planes, so a grid barrier between the phases is the simplest sufficient sync).
// The grid is sized to the number of workgroups that are resident at once (a cooperative
// launch fails rather than oversubscribe), every workgroup walks the logical blocks of each
// phase, and every workgroup reaches every barrier, so no wait can deadlock.  The phases
// call the same device functions as the separate kernels, so results are bitwise those of
// the four-launch step.  This is the batching pattern of one persistent fused launch per
// step; it is offered as a schedule beside the graph-replayed four-launch step, which
// measures faster (the persistent kernel runs every phase at the occupancy the heaviest
// phase allows).
#include <algorithm>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"
#include "particle_step.h"
#include "poisson_passes.h"

namespace scola {

template <typename T>
size_t poisson_lds_bytes(int M, int pass, int ng);

namespace {

// Logical blocks of one phase for this workgroup: with the XCD-aware numbering, the
// workgroups of XCD x (blockIdx mod 8) take the contiguous run x of the logical blocks.
struct Sweep {
  int first, step, end, per, x;
  bool remap;
  __device__ Sweep(const BlockMap& m) {
    remap = m.xcd_remap && (gridDim.x & 7) == 0;
    per = (m.count + 7) >> 3;
    x = blockIdx.x & 7;
    first = remap ? (int)(blockIdx.x >> 3) : (int)blockIdx.x;
    step = remap ? (int)(gridDim.x >> 3) : (int)gridDim.x;
    end = remap ? per : m.count;
  }
  __device__ int logical(int k) const { return remap ? x * per + k : k; }
};

// Grid-wide barrier number `phase` (1, 2, 3) on a counter that the launcher clears: every
// workgroup adds one arrival and waits until all gridDim.x arrivals of this phase are in.
// The launch is cooperative, so all workgroups are resident and the wait ends; it is also
// bounded (about a second of polling), after which the workgroup records a failure in
// counter[1] and goes on, so no wave can spin forever.
__device__ __forceinline__ void grid_barrier(unsigned* counter, unsigned phase) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();                                    // this block's writes, device-wide
    atomicAdd(counter, 1u);
    const unsigned target = phase * gridDim.x;
    unsigned spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1u << 24)) {
        atomicOr(counter + 1, 1u);                      // reported by the launcher's caller
        break;
      }
    }
    __threadfence();
  }
  __syncthreads();
}

// Waves per SIMD the persistent step is compiled for: FP32 boxes up to 64^3 ask for 4, what
// its LDS (the particle window plus the largest pass) allows anyway; without it the
// matrix-core passes inlined here let the register count grow until only 3 fit.
template <typename T, int R>
constexpr int persistent_waves() {
  return std::is_same<T, float>::value && R <= 4 ? 4 : 1;
}

template <typename T, int R>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(persistent_waves<T, R>())))
k_step_persistent(ParticleArgs<T> pa, MeshArgs<T> ma, BlockMap mp, BlockMap m1, BlockMap m2,
                  BlockMap m3, unsigned* barrier) {
  extern __shared__ __align__(16) unsigned char smem[];
  {
    const Sweep w(mp);
    for (int k = w.first; k < w.end; k += w.step) {
      const int L = w.logical(k);
      if (L < mp.count) particles_block<T, kStep>(pa, mp, L);
      __syncthreads();   // the block's LDS is reused by its next logical block
    }
  }
  grid_barrier(barrier, 1);
  {
    const Sweep w(m1);
    for (int k = w.first; k < w.end; k += w.step) {
      const int L = w.logical(k);
      if (L < m1.count) poisson_p1_block<T, R, false>(ma, m1, L, smem);
      __syncthreads();
    }
  }
  grid_barrier(barrier, 2);
  {
    const Sweep w(m2);
    for (int k = w.first; k < w.end; k += w.step) {
      const int L = w.logical(k);
      if (L < m2.count) poisson_p2_block<T, R>(ma, m2, L, smem);
      __syncthreads();
    }
  }
  grid_barrier(barrier, 3);
  {
    const Sweep w(m3);
    for (int k = w.first; k < w.end; k += w.step) {
      const int L = w.logical(k);
      if (L < m3.count) poisson_p3_block<T, R, false>(ma, m3, L, smem);
      __syncthreads();
    }
  }
}

template <typename T, int R>
hipError_t launch_persistent_R(const ParticleArgs<T>& pa, const MeshArgs<T>& ma,
                               const BlockMap& mp, const BlockMap& m1, const BlockMap& m2,
                               const BlockMap& m3, unsigned* barrier, hipStream_t s,
                               int* grid_out) {
  const void* fn = reinterpret_cast<const void*>(k_step_persistent<T, R>);
  size_t lds = 0;
  for (int pass = 1; pass <= 3; ++pass) lds = std::max(lds, poisson_lds_bytes<T>(16 * R, pass, 1));
  hipError_t e;
  if (lds > 65536) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int dev = 0, cus = 0, per_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, lds)) != hipSuccess)
    return e;
  const int most = std::max(std::max(mp.count, m1.count), std::max(m2.count, m3.count));
  int grid = std::min(per_cu * cus, ((most + 7) / 8) * 8);
  grid = std::max(8, grid / 8 * 8);
  if (grid > per_cu * cus) return hipErrorCooperativeLaunchTooLarge;
  if (grid_out) *grid_out = grid;
  if ((e = launch_zero_u32(barrier, 1, s)) != hipSuccess) return e;   // word 1 is sticky
  ParticleArgs<T> a0 = pa;
  MeshArgs<T> a1 = ma;
  BlockMap b0 = mp, b1 = m1, b2 = m2, b3 = m3;
  unsigned* bar = barrier;
  void* args[] = {&a0, &a1, &b0, &b1, &b2, &b3, &bar};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, (unsigned)lds, s);
}

}  // namespace

template <typename T>
hipError_t launch_step_persistent(const ParticleArgs<T>& pa, const MeshArgs<T>& ma, int M,
                                  const BlockMap& mp, const BlockMap& m1, const BlockMap& m2,
                                  const BlockMap& m3, unsigned* barrier, hipStream_t s,
                                  int* grid_out) {
  switch (M) {
    case 16: return launch_persistent_R<T, 1>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 32: return launch_persistent_R<T, 2>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 48: return launch_persistent_R<T, 3>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 64: return launch_persistent_R<T, 4>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 80: return launch_persistent_R<T, 5>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 96: return launch_persistent_R<T, 6>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 112: return launch_persistent_R<T, 7>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    case 128: return launch_persistent_R<T, 8>(pa, ma, mp, m1, m2, m3, barrier, s, grid_out);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_step_persistent<float>(const ParticleArgs<float>&,
                                                  const MeshArgs<float>&, int, const BlockMap&,
                                                  const BlockMap&, const BlockMap&,
                                                  const BlockMap&, unsigned*, hipStream_t, int*);

}  // namespace scola
