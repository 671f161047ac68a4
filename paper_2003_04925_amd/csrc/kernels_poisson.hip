// Dirichlet Poisson solve of every sCOLA box by type-I discrete sine transforms (App. C).
//
// A box of M particles per side has n = M - 1 interior PM nodes per side.  Three passes
// over the (n)^3 mesh of every box, all boxes in one launch each:
//   P1  per x-plane: fixed-point mass -> delta, delta' = delta - Delta Phi_BCs (App. C.1),
//       forward DST-I along z then y, in LDS;
//   P2  per chunk of consecutive x pencils of the box's n^2 (64 in FP32 plans, 32 in FP64):
//       forward DST-I along x, division by the FDA eigenvalue sum times the inverse
//       normalisation 8/M^3 (App. C.2, eq. Poisson_sine_space), inverse DST-I along x;
//   P3  per x-plane: inverse DST-I along y then z, and the potential written to the padded
//       node grid [-g, M+g]^3 with the shell filled from Phi_BCs (Sec. 3.4.2); g = 1, 2, 3
//       ghost layers at finite-difference order 2, 4, 6 (Sec. 3), where delta' also takes
//       the wide stencil's reach into the g Dirichlet layers (App. C.1).
//
// FP32 plans form every DST-I as a product with the sine matrix on the matrix cores
// (dst_mfma.h: split FP16 operands, FP32 accumulation); FP64 plans use the real-data sine
// transform through a half-length complex FFT on a quarter wavefront (poisson_passes.h).
// Within an evolution, P3 leaves each plane's boundary-source perimeter terms in its
// consumed work plane for the next solve's P1 (MeshArgs::bc_handoff).
#include <algorithm>
#include <atomic>
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"
#include "poisson_passes.h"

namespace scola {

namespace {

// Waves per SIMD the FP32 passes are compiled for: their matrix-core transforms leave them
// latency-bound, so boxes up to 64^3 ask for full occupancy (at most 64 registers a lane),
// and boxes of 80^3 for the 4 that their LDS allows (c3: 1.01 -> 0.98 ms per solve); at
// 96^3 that would spill (c5: 4.25 -> 4.68 ms), so larger boxes and FP64 plans take what
// their registers allow.  The 64^3 reverse passes, the 64^3 first pass at orders 4 and 6
// and the 48^3 first pass at order 6 need a few more registers than 64: they take 7 waves
// (72 registers) rather than spill to scratch.
template <typename T, int R, bool ADJ = false, int NG = 1>
constexpr int pass_waves() {
  if (!std::is_same<T, float>::value) return 1;
  if ((R == 4 && (ADJ || NG > 1)) || (R == 3 && NG == 3)) return 7;
  return R <= 4 ? 8 : R == 5 ? 4 : 1;
}

template <typename T, int R, bool ADJ, int NG>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(pass_waves<T, R, ADJ, NG>())))
k_poisson_p1(MeshArgs<T> a, BlockMap m) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = logical_block(m);
  if (L < m.count) poisson_p1_block<T, R, ADJ, NG>(a, m, L, smem);
}

template <typename T, int R>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(pass_waves<T, R>())))
k_poisson_p2(MeshArgs<T> a, BlockMap m) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = logical_block(m);
  if (L < m.count) poisson_p2_block<T, R>(a, m, L, smem);
}

template <typename T, int R, bool ADJ, int NG>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(pass_waves<T, R, ADJ, NG>())))
k_poisson_p3(MeshArgs<T> a, BlockMap m) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int L = logical_block(m);
  if (L < m.count) poisson_p3_block<T, R, ADJ, NG>(a, m, L, smem);
}

}  // namespace

// Dynamic LDS of each pass for boxes of M nodes: FP64 plans the 2M twiddles, then P1 the
// (M-1)^2 plane, P2 the M eigenvalues and an (M-1) x 33 pencil tile, P3 the plane and the
// perimeter terms it hands on; FP32 plans the block-maximum slots, then the plane region
// (the plane or the split lines aliasing it, whose tail beyond the plane holds P3's
// perimeter terms before the transform), P2 the eigenvalues and the chunk's split lines
// aliased by its output tile.  P3 holds the padded plane's border in registers.  Sized per
// M and per pass, so small boxes keep more blocks per CU.
template <typename T>
size_t poisson_lds_bytes(int M, int pass, int ng) {
  (void)ng;
  const size_t n = (size_t)M - 1, tw = 2 * (size_t)M * sizeof(cx<T>);
  // P3: the perimeter terms it hands to the next solve's P1, 8-byte aligned behind the plane
  const size_t terms = 8 + 4 * (n - 1) * sizeof(double);
  if (std::is_same<T, float>::value) {
    // matrix-core transforms: block-maximum slots, then the plane region (the plane or the
    // split lines that alias it); P2: the eigenvalues, then the split lines of the chunk's
    // columns aliased by the output tile
    const int R = M / 16;
    const size_t region = std::max(n * n * sizeof(float), mfma_split_bytes(R));
    if (pass == 1 || pass == 3) return kMfmaHead + region;
    const size_t lines =
        (size_t)kPencilChunkMfma * (32 * ((R + 1) / 2) + 8) * 2 * sizeof(_Float16);
    return kMfmaHead + (size_t)M * sizeof(float) +
           std::max(n * (kPencilChunkMfma + 1) * sizeof(float), lines);
  }
  if (pass == 1) return tw + n * n * sizeof(T);
  if (pass == 2) return tw + ((size_t)M + n * (kPencilChunk + 1)) * sizeof(T);
  return tw + n * n * sizeof(T) + terms;
}

namespace {

template <typename T, int R, bool ADJ, int NG>
hipError_t launch_poisson_R(const MeshArgs<T>& a, const BlockMap& p1, const BlockMap& p2,
                            const BlockMap& p3, hipStream_t s) {
  const size_t l1 = poisson_lds_bytes<T>(16 * R, 1, NG), l2 = poisson_lds_bytes<T>(16 * R, 2, NG),
               l3 = poisson_lds_bytes<T>(16 * R, 3, NG);
  if (l1 > 65536 || l2 > 65536 || l3 > 65536) {
    // allow more than 64 KiB of dynamic LDS (160 KiB on gfx950): a function attribute of
    // each device, set once per device
    static std::atomic<uint64_t> done{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = dev < 64 ? (1ull << dev) : 0ull;
    if (!bit || !(done.load() & bit)) {
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_poisson_p1<T, R, ADJ, NG>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)l1);
      if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_poisson_p2<T, R>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)l2);
      if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_poisson_p3<T, R, ADJ, NG>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)l3);
      if (e != hipSuccess) return e;
      done.fetch_or(bit);
    }
  }
  if (p1.count > 0)
    hipLaunchKernelGGL((k_poisson_p1<T, R, ADJ, NG>), dim3(padded_grid(p1)), dim3(kBlock), l1, s,
                       a, p1);
  if (p2.count > 0)
    hipLaunchKernelGGL((k_poisson_p2<T, R>), dim3(padded_grid(p2)), dim3(kBlock), l2, s, a, p2);
  if (p3.count > 0)
    hipLaunchKernelGGL((k_poisson_p3<T, R, ADJ, NG>), dim3(padded_grid(p3)), dim3(kBlock), l3, s,
                       a, p3);
  return hipGetLastError();
}

template <typename T, int R>
hipError_t launch_poisson_RA(const MeshArgs<T>& a, const BlockMap& p1, const BlockMap& p2,
                             const BlockMap& p3, hipStream_t s, bool adjoint) {
  if (adjoint) {
    // the reverse passes exist for order 2 only (the plan refuses the others)
    if (a.ng != 1) return hipErrorInvalidValue;
    return launch_poisson_R<T, R, true, 1>(a, p1, p2, p3, s);
  }
  switch (a.ng) {
    case 1: return launch_poisson_R<T, R, false, 1>(a, p1, p2, p3, s);
    case 2: return launch_poisson_R<T, R, false, 2>(a, p1, p2, p3, s);
    case 3: return launch_poisson_R<T, R, false, 3>(a, p1, p2, p3, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename T>
hipError_t launch_poisson(const MeshArgs<T>& a, int M, const BlockMap& p1, const BlockMap& p2,
                          const BlockMap& p3, hipStream_t s, bool adjoint) {
  switch (M) {
    case 16: return launch_poisson_RA<T, 1>(a, p1, p2, p3, s, adjoint);
    case 32: return launch_poisson_RA<T, 2>(a, p1, p2, p3, s, adjoint);
    case 48: return launch_poisson_RA<T, 3>(a, p1, p2, p3, s, adjoint);
    case 64: return launch_poisson_RA<T, 4>(a, p1, p2, p3, s, adjoint);
    case 80: return launch_poisson_RA<T, 5>(a, p1, p2, p3, s, adjoint);
    case 96: return launch_poisson_RA<T, 6>(a, p1, p2, p3, s, adjoint);
    case 112: return launch_poisson_RA<T, 7>(a, p1, p2, p3, s, adjoint);
    case 128: return launch_poisson_RA<T, 8>(a, p1, p2, p3, s, adjoint);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_poisson<float>(const MeshArgs<float>&, int, const BlockMap&,
                                          const BlockMap&, const BlockMap&, hipStream_t, bool);
template hipError_t launch_poisson<double>(const MeshArgs<double>&, int, const BlockMap&,
                                           const BlockMap&, const BlockMap&, hipStream_t, bool);
template size_t poisson_lds_bytes<float>(int, int, int);
template size_t poisson_lds_bytes<double>(int, int, int);

}  // namespace scola
