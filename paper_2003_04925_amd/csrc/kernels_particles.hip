// Particle kernels of the sCOLA step: CiC deposit (B^sCOLA, Sec. 3.4.1), the fused
// gradient + CiC interpolation + COLA kick + drift + deposit (App. A eq. kick-scola,
// App. B eqs. K_COLA and D_COLA), and the untiling of the core particles with the output
// CiC density (Sec. 3.2 B.2, Sec. 4.1).
//
// Layout: structure of arrays [3][P] over all boxes, box after box, particles of a box in
// lattice order (z fastest), so a 256-thread block reads 256 consecutive elements of each
// of the 12 particle streams.  Psi1 and Psi2 are held in the plan precision (differenced in
// FP64 at set-up) and every particle position is formed in FP64 (u = q - D1 Psi1 + D2 Psi2 +
// x_res) before its cell index is taken.
//
// The deposit accumulates rounded fixed-point weights in integers (2^40 units per
// particle in 64 bits for FP64 plans, 2^21 in 32 bits for FP32 plans): sums are exact and
// independent of the order of the atomics, which makes every run bitwise reproducible and
// a box computed alone bitwise equal to the same box in a batch.  The weights come from
// exact integer splits of the unit, so every particle carries exactly one unit of mass,
// split between deposited and dropped (outside the interior nodes), and no weight is
// negative.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"
#include "particle_step.h"

namespace scola {

namespace {

// OCC: waves per SIMD the register allocation is held to (6 or 8); a schedule choice.
template <typename T, int MODE, int OCC>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(OCC)))
k_particles(ParticleArgs<T> a, BlockMap m) {
  const int L = logical_block(m);
  if (L < m.count) particles_block<T, MODE>(a, m, L);
}

// The force-evaluating modes at gradient order 2 NG, NG = 2 or 3 (Sec. 3).
template <typename T, int MODE, int NG>
__global__ void __launch_bounds__(kBlock) k_particles_wide(ParticleArgs<T> a, BlockMap m) {
  const int L = logical_block(m);
  if (L < m.count) particles_block<T, MODE, NG>(a, m, L);
}

__global__ void k_zero_u32(unsigned* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__device__ inline int wrapi(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// B.2: core particles -> global lattice order; optional periodic CiC of the core
// particles on the N_out^3 output grid (nodes at integer multiples of L / N_out).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_output(OutputArgs<T> a, BlockMap m, int density) {
  const int L = logical_block(m);
  if (L >= m.count) return;
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int M = t.M;
  const int64_t pl = (int64_t)m.local[b] * kBlock + threadIdx.x;
  int i, j, k;
  brick_site(pl, M, i, j, k);
  const int lo = t.core_lo[0], hi = t.core_lo[0] + t.core_n;
  if (i < lo || i >= hi || j < lo || j >= hi || k < lo || k >= hi) return;
  const int64_t p = t.p_off + pl;
  const int64_t P = a.P;
  const int Np = a.Np;
  const int64_t gidx = ((int64_t)wrapi(t.origin[0] + i, Np) * Np + wrapi(t.origin[1] + j, Np)) *
                           Np + wrapi(t.origin[2] + k, Np);
  const int64_t Np3 = (int64_t)Np * Np * Np;
  const int idx[3] = {i, j, k};
  double ug[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    // the tile's own final growth factors (tiles may end at different scale factors)
    const double u = lpt_base(idx[c] + 0.5, t.D1f, a.psi1[c * P + p], t.D2f, a.psi2[c * P + p]) +
                     (double)a.xres[c * P + p];
    ug[c] = t.origin[c] + u;
    if (a.pos) {
      double x = fmod(ug[c], (double)Np);
      if (x < 0) x += Np;
      T xl = (T)(x * a.cell);
      if (xl >= (T)a.L) xl = T(0);          // rounding up to L wraps to 0
      a.pos[c * Np3 + gidx] = xl;
    }
    if (a.mom) a.mom[c * Np3 + gidx] = (T)((double)a.pres[c * P + p] * a.cell);
  }
  if (density) {
    const double s = (double)a.N_out / (double)Np;
    const int No = a.N_out;
    double f[3];
    int j0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double uo = ug[c] * s;
      const double fl = floor(uo);
      f[c] = uo - fl;
      j0[c] = wrapi((int)fmod(fl, (double)No), No);
    }
    long long w[8];
    split_weights<long long, double>(f[0], f[1], f[2], 1ll << 40, w);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int nx = (j0[0] + ((c >> 2) & 1)) % No, ny = (j0[1] + ((c >> 1) & 1)) % No,
                nz = (j0[2] + (c & 1)) % No;
      if (w[c] != 0)
        atomicAdd(a.grid + ((int64_t)nx * No + ny) * No + nz, (unsigned long long)w[c]);
    }
  }
}

template <typename T>
__global__ void k_density_convert(const unsigned long long* __restrict__ grid, T* out,
                                  int64_t n, double scale) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (T)((double)(long long)grid[i] * kFixedInv * scale - 1.0);
}

// One block per tile: the dropped mass of the tile's bricks (word 3 of each brick's hint,
// left by an FP32 deposit) summed into the tile's counter, and the words cleared.
__global__ void k_fold_drops(const TileDesc* __restrict__ tiles, unsigned* hints,
                             unsigned long long* dropped) {
  const TileDesc t = tiles[blockIdx.x];
  const int64_t b0 = t.p_off / kBlock, nb = (int64_t)t.M * t.M * t.M / kBlock;
  unsigned long long d = 0;
  for (int64_t e = threadIdx.x; e < nb; e += blockDim.x) {
    unsigned* w = hints + 4 * (b0 + e) + 3;
    d += *w;
    *w = 0u;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o);
  if ((threadIdx.x & 63) == 0 && d != 0ull) atomicAdd(dropped + blockIdx.x, d);
}

}  // namespace

hipError_t launch_fold_drops(const TileDesc* tiles, int n_tiles, unsigned* hints,
                             unsigned long long* dropped, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_drops, dim3((unsigned)n_tiles), dim3(kBlock), 0, s, tiles, hints,
                     dropped);
  return hipGetLastError();
}

hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)(blocks < 65536 ? blocks : 65536)),
                     dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)(blocks < 65536 ? blocks : 65536)),
                     dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

template <typename T, int OCC>
hipError_t launch_particles_occ(const ParticleArgs<T>& a, int mode, const BlockMap& m,
                                hipStream_t s) {
  if (m.count <= 0) return hipSuccess;
  const dim3 grid(padded_grid(m)), block(kBlock);
  switch (mode) {
    case kDepositOnly:
      hipLaunchKernelGGL((k_particles<T, kDepositOnly, OCC>), grid, block, 0, s, a, m);
      break;
    case kStep:
      hipLaunchKernelGGL((k_particles<T, kStep, OCC>), grid, block, 0, s, a, m);
      break;
    case kStepNoDeposit:
      hipLaunchKernelGGL((k_particles<T, kStepNoDeposit, OCC>), grid, block, 0, s, a, m);
      break;
    case kFinalKick:
      hipLaunchKernelGGL((k_particles<T, kFinalKick, OCC>), grid, block, 0, s, a, m);
      break;
    case kInit:
      hipLaunchKernelGGL((k_particles<T, kInit, OCC>), grid, block, 0, s, a, m);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int NG>
hipError_t launch_particles_wide(const ParticleArgs<T>& a, int mode, const BlockMap& m,
                                 hipStream_t s) {
  const dim3 grid(padded_grid(m)), block(kBlock);
  switch (mode) {
    case kStep:
      hipLaunchKernelGGL((k_particles_wide<T, kStep, NG>), grid, block, 0, s, a, m);
      break;
    case kStepNoDeposit:
      hipLaunchKernelGGL((k_particles_wide<T, kStepNoDeposit, NG>), grid, block, 0, s, a, m);
      break;
    case kFinalKick:
      hipLaunchKernelGGL((k_particles_wide<T, kFinalKick, NG>), grid, block, 0, s, a, m);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_particles(const ParticleArgs<T>& a, int mode, const BlockMap& m, int occ,
                            hipStream_t s) {
  // the deposit-only modes do not evaluate the force: one kernel for every order
  if (a.ng != 1 && mode != kDepositOnly && mode != kInit) {
    if (m.count <= 0) return hipSuccess;
    switch (a.ng) {
      case 2: return launch_particles_wide<T, 2>(a, mode, m, s);
      case 3: return launch_particles_wide<T, 3>(a, mode, m, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (occ) {
    case 6: return launch_particles_occ<T, 6>(a, mode, m, s);
    case 8: return launch_particles_occ<T, 8>(a, mode, m, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_output(const OutputArgs<T>& a, const BlockMap& m, bool density,
                         T* density_out, hipStream_t s) {
  const int64_t n_out = (int64_t)a.N_out * a.N_out * a.N_out;
  if (density) {
    hipError_t e = launch_zero_u64(a.grid, n_out, s);
    if (e != hipSuccess) return e;
  }
  if (m.count > 0)
    hipLaunchKernelGGL(k_output<T>, dim3(padded_grid(m)), dim3(kBlock), 0, s, a, m,
                       density ? 1 : 0);
  if (density) {
    const double r = (double)a.N_out / (double)a.Np;
    const int64_t blocks = (n_out + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_density_convert<T>,
                       dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(kBlock), 0, s,
                       a.grid, density_out, n_out, r * r * r);
  }
  return hipGetLastError();
}

template hipError_t launch_particles<float>(const ParticleArgs<float>&, int, const BlockMap&, int,
                                            hipStream_t);
template hipError_t launch_particles<double>(const ParticleArgs<double>&, int,
                                             const BlockMap&, int, hipStream_t);
template hipError_t launch_output<float>(const OutputArgs<float>&, const BlockMap&, bool,
                                         float*, hipStream_t);
template hipError_t launch_output<double>(const OutputArgs<double>&, const BlockMap&, bool,
                                          double*, hipStream_t);

}  // namespace scola
