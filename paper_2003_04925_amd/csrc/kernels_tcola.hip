// Monolithic periodic tCOLA (Sec. 2.2, App. A eqs. drift-cola and kick-tcola, App. B): the
// whole box of N^3 particles evolved at once with a periodic PM grid of N^3 nodes, so no
// tiling approximation is made.  It is the reference the sCOLA boxes are compared with
// (Sec. 4.2) and the source of the true density and potential of the consistency tests
// (Sec. 4.3).
//
// The operators are those of the boxes without the box cut: CiC deposit onto the periodic
// node grid (nodes at integer positions, one per lattice cell, global mean density one
// particle per cell), the Poisson equation solved in Fourier space with the symbol of the
// finite-difference Laplacian of the plan's order (-4 sum sin^2(k/2) at order 2, zero mode
// removed), the central-difference gradient of the same order and CiC interpolation, then
// the same COLA kick and drift.  Particles are in lattice order; every
// position is formed in FP64 as in the box kernels; deposits are 64-bit fixed point (2^40
// units per particle), exact and order independent.  The Poisson solve reuses the FP64
// FFTs of the set-up (a reference path: its cost is not part of the sCOLA step).
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"

namespace scola {

namespace {

// Central first-difference weights of order 2 ng: (1/2), (2/3, -1/12), (3/4, -3/20, 1/60).
__device__ inline double tc_grad_weight(int ng, int k) {
  return ng == 1 ? 0.5
       : ng == 2 ? (k == 1 ? 2.0 / 3.0 : -1.0 / 12.0)
                 : (k == 1 ? 0.75 : k == 2 ? -0.15 : 1.0 / 60.0);
}


__device__ __forceinline__ int pwrap(int i, int N) { return i & (N - 1); }   // N: power of 2

// Psi1 = D phi1, Psi2 = D phi2 (order-2 central differences) at every lattice site, and
// the operator L- (x_res = p_res = 0).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tcola_setup(TcolaArgs<T> a, const double* phi1,
                                                        const double* phi2) {
  const int N = a.N;
  const int64_t n3 = (int64_t)N * N * N;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int x = (int)(p / ((int64_t)N * N)), y = (int)((p / N) % N), z = (int)(p % N);
  auto at = [&](const double* f, int i, int j, int k) {
    return f[((int64_t)pwrap(i, N) * N + pwrap(j, N)) * N + pwrap(k, N)];
  };
  T* s1 = const_cast<T*>(a.psi1);
  T* s2 = const_cast<T*>(a.psi2);
  double g1[3] = {0.0, 0.0, 0.0}, g2[3] = {0.0, 0.0, 0.0};
  for (int k = 1; k <= a.ng; ++k) {
    const double c = tc_grad_weight(a.ng, k);
    g1[0] += c * (at(phi1, x + k, y, z) - at(phi1, x - k, y, z));
    g1[1] += c * (at(phi1, x, y + k, z) - at(phi1, x, y - k, z));
    g1[2] += c * (at(phi1, x, y, z + k) - at(phi1, x, y, z - k));
    g2[0] += c * (at(phi2, x + k, y, z) - at(phi2, x - k, y, z));
    g2[1] += c * (at(phi2, x, y + k, z) - at(phi2, x, y - k, z));
    g2[2] += c * (at(phi2, x, y, z + k) - at(phi2, x, y, z - k));
  }
  for (int c = 0; c < 3; ++c) {
    s1[c * n3 + p] = (T)g1[c];
    s2[c * n3 + p] = (T)g2[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.xres[c * n3 + p] = T(0);
    a.pres[c * n3 + p] = T(0);
  }
}

// One particle pass: (MODE kInit) L- and the deposit of the LPT positions; (kStep,
// kStepNoDeposit) force at u = q - D1 Psi1 + D2 Psi2 + x_res, kick, drift and (kStep) the
// deposit of the new positions; (kFinalKick) the last half kick and L+.
template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_tcola_particles(TcolaArgs<T> a) {
  const int N = a.N;
  const int64_t n3 = (int64_t)N * N * N;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int idx[3] = {(int)(p / ((int64_t)N * N)), (int)((p / N) % N), (int)(p % N)};
  const StepScalars sc = a.sc;
  double s1[3], s2[3], u[3];
  T xr[3], pr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s1[c] = a.psi1[c * n3 + p];
    s2[c] = a.psi2[c * n3 + p];
    if (MODE == kInit) {
      xr[c] = T(0);
      a.xres[c * n3 + p] = T(0);
      a.pres[c * n3 + p] = T(0);
    } else {
      xr[c] = a.xres[c * n3 + p];
    }
    u[c] = lpt_base(idx[c] + 0.5, sc.D1, s1[c], sc.D2, s2[c]) + (double)xr[c];
  }
  if (MODE != kInit) {
    // central-difference gradient of the periodic potential at the 8 CiC corners,
    // interpolated with the CiC weights
    int j0[3];
    T f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double fl = floor(u[c]);
      j0[c] = (int)fl;
      f[c] = (T)(u[c] - fl);
    }
    auto ph = [&](int i, int j, int k) {
      return a.phi[((int64_t)pwrap(i, N) * N + pwrap(j, N)) * N + pwrap(k, N)];
    };
    T g[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int cx = 0; cx < 2; ++cx)
#pragma unroll
      for (int cy = 0; cy < 2; ++cy)
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
          const T w = (cx ? f[0] : T(1) - f[0]) * (cy ? f[1] : T(1) - f[1]) *
                      (cz ? f[2] : T(1) - f[2]);
          const int i = j0[0] + cx, j = j0[1] + cy, k = j0[2] + cz;
          if (a.ng == 1) {
            g[0] += w * (T(0.5) * (ph(i + 1, j, k) - ph(i - 1, j, k)));
            g[1] += w * (T(0.5) * (ph(i, j + 1, k) - ph(i, j - 1, k)));
            g[2] += w * (T(0.5) * (ph(i, j, k + 1) - ph(i, j, k - 1)));
          } else {
            // central difference of order 2 ng
            T sx = 0, sy = 0, sz = 0;
            for (int o = 1; o <= a.ng; ++o) {
              const T c = (T)tc_grad_weight(a.ng, o);
              sx += c * (ph(i + o, j, k) - ph(i - o, j, k));
              sy += c * (ph(i, j + o, k) - ph(i, j - o, k));
              sz += c * (ph(i, j, k + o) - ph(i, j, k - o));
            }
            g[0] += w * sx;
            g[1] += w * sy;
            g[2] += w * sz;
          }
        }
    const double d2 = sc.D2 - sc.D1 * sc.D1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pr[c] = a.pres[c * n3 + p];
      pr[c] += (T)sc.beta * (g[c] - (T)(sc.D1 * s1[c] - d2 * s2[c]));
    }
    if (MODE == kFinalKick) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.pres[c * n3 + p] = pr[c] + (T)(sc.c1 * s1[c] + sc.c2 * s2[c]);
      return;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xr[c] += (T)sc.alpha * pr[c];
      a.xres[c * n3 + p] = xr[c];
      a.pres[c * n3 + p] = pr[c];
    }
    if (MODE == kStepNoDeposit) return;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      u[c] = lpt_base(idx[c] + 0.5, sc.D1n, s1[c], sc.D2n, s2[c]) + (double)xr[c];
  }
  // periodic CiC deposit, 2^40 units per particle
  int j0[3];
  double f[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double fl = floor(u[c]);
    j0[c] = (int)fl;
    f[c] = u[c] - fl;
  }
  long long w[8];
  split_weights<long long, double>(f[0], f[1], f[2], 1ll << 40, w);
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (w[c] != 0)
      atomicAdd(a.rho + ((int64_t)pwrap(j0[0] + ((c >> 2) & 1), N) * N +
                         pwrap(j0[1] + ((c >> 1) & 1), N)) * N + pwrap(j0[2] + (c & 1), N),
                (unsigned long long)w[c]);
}

// delta = mass - 1 (one particle per cell) as complex FFT input; the mass mesh is cleared
// for the next deposit, and delta optionally recorded.
template <typename T>
__global__ void k_tcola_density(unsigned long long* __restrict__ rho, double2* __restrict__ c,
                                T* __restrict__ record, int64_t n3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const double d = (double)(long long)rho[i] * kFixedInv - 1.0;
  rho[i] = 0ull;
  c[i] = make_double2(d, 0.0);
  if (record) record[i] = (T)d;
}

template <typename T>
__global__ void k_tcola_potential(const double2* __restrict__ c, T* __restrict__ phi,
                                  T* __restrict__ record, int64_t n3) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  const T v = (T)(c[i].x / (double)n3);
  phi[i] = v;
  if (record) record[i] = v;
}

// Final positions (Mpc/h in [0, L)) and momenta at the lattice index, and the periodic CiC of
// all particles on the N_out^3 output grid (2^40 units per particle).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_tcola_output(TcolaArgs<T> a, T* pos, T* mom,
                                                         unsigned long long* grid, int N_out,
                                                         double cell, double L) {
  const int N = a.N;
  const int64_t n3 = (int64_t)N * N * N;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n3) return;
  const int idx[3] = {(int)(p / ((int64_t)N * N)), (int)((p / N) % N), (int)(p % N)};
  double ug[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ug[c] = lpt_base(idx[c] + 0.5, a.sc.D1, a.psi1[c * n3 + p], a.sc.D2, a.psi2[c * n3 + p]) +
            (double)a.xres[c * n3 + p];
    if (pos) {
      double x = fmod(ug[c], (double)N);
      if (x < 0) x += N;
      T xl = (T)(x * cell);
      if (xl >= (T)L) xl = T(0);
      pos[c * n3 + p] = xl;
    }
    if (mom) mom[c * n3 + p] = (T)((double)a.pres[c * n3 + p] * cell);
  }
  if (grid) {
    const double s = (double)N_out / (double)N;
    double f[3];
    int j0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double uo = ug[c] * s;
      const double fl = floor(uo);
      f[c] = uo - fl;
      int j = (int)fmod(fl, (double)N_out);
      j0[c] = j < 0 ? j + N_out : j;
    }
    long long w[8];
    split_weights<long long, double>(f[0], f[1], f[2], 1ll << 40, w);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int nx = (j0[0] + ((c >> 2) & 1)) % N_out, ny = (j0[1] + ((c >> 1) & 1)) % N_out,
                nz = (j0[2] + (c & 1)) % N_out;
      if (w[c] != 0)
        atomicAdd(grid + ((int64_t)nx * N_out + ny) * N_out + nz, (unsigned long long)w[c]);
    }
  }
}

template <typename T>
__global__ void k_tcola_density_out(const unsigned long long* __restrict__ grid, T* out,
                                    int64_t n, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (T)((double)(long long)grid[i] * kFixedInv * scale - 1.0);
}

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename T>
hipError_t launch_tcola_setup(const TcolaArgs<T>& a, const double* phi1, const double* phi2,
                              hipStream_t s) {
  const int64_t n3 = (int64_t)a.N * a.N * a.N;
  hipLaunchKernelGGL(k_tcola_setup<T>, dim3(blocks_of(n3)), dim3(kBlock), 0, s, a, phi1, phi2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tcola_particles(const TcolaArgs<T>& a, int mode, hipStream_t s) {
  const dim3 grid(blocks_of((int64_t)a.N * a.N * a.N)), block(kBlock);
  switch (mode) {
    case kInit: hipLaunchKernelGGL((k_tcola_particles<T, kInit>), grid, block, 0, s, a); break;
    case kStep: hipLaunchKernelGGL((k_tcola_particles<T, kStep>), grid, block, 0, s, a); break;
    case kStepNoDeposit:
      hipLaunchKernelGGL((k_tcola_particles<T, kStepNoDeposit>), grid, block, 0, s, a);
      break;
    case kFinalKick:
      hipLaunchKernelGGL((k_tcola_particles<T, kFinalKick>), grid, block, 0, s, a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The FDA Poisson solve of the periodic box: mass mesh -> delta -> potential (FP64 FFTs).
template <typename T>
hipError_t launch_tcola_poisson(const TcolaArgs<T>& a, double2* cbuf, T* phi, T* rec_delta,
                                T* rec_phi, hipStream_t s) {
  const int N = a.N;
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_tcola_density<T>, dim3(blocks_of(n3)), dim3(kBlock), 0, s, a.rho, cbuf,
                     rec_delta, n3);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = fft3d_forward(cbuf, N, s)) != hipSuccess) return e;
  if ((e = launch_inverse_laplacian(cbuf, N, a.ng, s)) != hipSuccess) return e;
  if ((e = fft3d_inverse(cbuf, N, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tcola_potential<T>, dim3(blocks_of(n3)), dim3(kBlock), 0, s, cbuf, phi,
                     rec_phi, n3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tcola_output(const TcolaArgs<T>& a, T* pos, T* mom, unsigned long long* grid,
                               T* density, int N_out, double cell, double L, hipStream_t s) {
  const int64_t n3 = (int64_t)a.N * a.N * a.N;
  const int64_t no3 = (int64_t)N_out * N_out * N_out;
  if (density) {
    hipError_t e = launch_zero_u64(grid, no3, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_tcola_output<T>, dim3(blocks_of(n3)), dim3(kBlock), 0, s, a, pos, mom,
                     density ? grid : nullptr, N_out, cell, L);
  if (density) {
    const double r = (double)N_out / (double)a.N;
    hipLaunchKernelGGL(k_tcola_density_out<T>, dim3(blocks_of(no3)), dim3(kBlock), 0, s, grid,
                       density, no3, r * r * r);
  }
  return hipGetLastError();
}

#define SCOLA_TCOLA_INSTANTIATE(T)                                                         \
  template hipError_t launch_tcola_setup<T>(const TcolaArgs<T>&, const double*,             \
                                            const double*, hipStream_t);                    \
  template hipError_t launch_tcola_particles<T>(const TcolaArgs<T>&, int, hipStream_t);     \
  template hipError_t launch_tcola_poisson<T>(const TcolaArgs<T>&, double2*, T*, T*, T*,    \
                                              hipStream_t);                                 \
  template hipError_t launch_tcola_output<T>(const TcolaArgs<T>&, T*, T*, unsigned long long*, \
                                             T*, int, double, double, hipStream_t);
SCOLA_TCOLA_INSTANTIATE(float)
SCOLA_TCOLA_INSTANTIATE(double)
#undef SCOLA_TCOLA_INSTANTIATE

}  // namespace scola
