// Shared declarations of the tiled-sCOLA HIP library (device tables, launch helpers).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

namespace scola {

constexpr int kFixedBits = 40;                       // output-grid CiC weights, 2^40
constexpr double kFixedOne = 1099511627776.0;        // 2^40
constexpr double kFixedInv = 1.0 / 1099511627776.0;

// Fixed-point unit of one particle's mass in the box meshes.  FP64 plans: 2^40 (weights
// formed in FP64), block windows and the mesh in 64-bit integers.  FP32 plans: 2^21 (weights
// formed in FP32; the quantum 2^-21 is close to FP32 weight rounding), block windows and the
// mesh in 32-bit unsigned integers: a node can hold 2^32 / 2^21 = 2048 particles (density
// contrast below 2047; the workloads here peak far lower, and the Poisson pass flags any
// node above 1023), and a 256-particle block window at most 2^29 units.
template <typename T>
struct MeshFixed;
template <>
struct MeshFixed<double> {
  static constexpr int bits = 40;
  using window_t = unsigned long long;
  using rho_t = unsigned long long;
};
template <>
struct MeshFixed<float> {
  static constexpr int bits = 21;
  using window_t = unsigned int;
  using rho_t = unsigned int;
};
constexpr int kMaxM = 128;                            // boxes of 16..128 particles per side
constexpr int kBlock = 256;                           // threads of every mesh/particle block

// One sCOLA box (Sec. 3.2): M particles per side starting at lattice index origin.
struct TileDesc {
  int32_t M;
  int32_t origin[3];       // first box particle (lattice index, may be negative; wraps)
  int32_t core_lo[3];      // first core particle, relative to the box (= buffer)
  int32_t core_n;
  int64_t p_off;           // first particle in the [3][P] particle arrays
  int64_t g_off;           // first interior node in rho/work ((M-1)^3 per box)
  int64_t h_off;           // first padded node in phi/bc0 ((M+3)^3 per box)
  int32_t tw_off;          // first entry of this M's twiddle table (2M complex values)
  int32_t ev_off;          // first entry of this M's eigenvalue table (M-1 values)
  int32_t tclass;          // time class: index of the tile's final scale factor in the plan
  int32_t dm_off;          // FP32 plans: first half of this M's split sine matrix
  double D1f, D2f;         // growth factors at the tile's final scale factor
};

// Scalars of one fused particle step (App. B): kick factor, drift factor and the growth
// factors at the kick time t_k (D1, D2) and at the end of the drift (D1n, D2n).
struct StepScalars {
  double beta, alpha, D1, D2, D1n, D2n;
  double c1, c2;            // L+ coefficients (final kick only)
  // an evolution's start without stored zeros: L- (kInit) does not write x_res = p_res = 0,
  // and the first step takes them as zero instead of reading them
  int fresh;
};

// Cross-lane exchange v[lane ^ S] within 32-lane groups without LDS traffic: xor 1 and 2
// are DPP quad permutations; xor 4 = (xor 3 quad reverse) then (xor 7 half-row mirror);
// xor 8 = (xor 7 half-row mirror) then (xor 15 row mirror); xor 16 crosses 16-lane rows and
// uses ds_swizzle in bit-mask mode (and 0x1f, or 0, xor 0x10).
template <int S>
__device__ __forceinline__ int lane_xor(int v) {
  static_assert(S == 1 || S == 2 || S == 4 || S == 8 || S == 16, "xor distance");
  if constexpr (S == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);
  if constexpr (S == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);
  if constexpr (S == 4) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, true);
    return __builtin_amdgcn_mov_dpp(t, 0x141, 0xF, 0xF, true);
  }
  if constexpr (S == 8) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);
    return __builtin_amdgcn_mov_dpp(t, 0x140, 0xF, 0xF, true);
  }
  if constexpr (S == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
  return v;
}

template <int S>
__device__ __forceinline__ float lane_xor(float v) {
  return __int_as_float(lane_xor<S>(__float_as_int(v)));
}

template <int S>
__device__ __forceinline__ double lane_xor(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = lane_xor<S>((int)(b & 0xffffffffll));
  const int hi = lane_xor<S>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Particles of a box are stored brick by brick: bricks of 4 x 8 x 8 lattice sites (256
// particles, one thread block), bricks in lattice order, sites inside a brick in lattice
// order.  A block's particles therefore form a compact Lagrangian cube (small Eulerian
// footprint for the LDS-privatised deposit) while its loads stay fully contiguous.
// Requires M % 8 == 0.
__host__ __device__ inline void brick_site(int64_t pl, int M, int& i, int& j, int& k) {
  const int nb = M >> 3;
  const int brick = (int)(pl >> 8), w = (int)(pl & 255);
  const int bk = brick % nb, bj = (brick / nb) % nb, bi = brick / (nb * nb);
  i = bi * 4 + (w >> 6);
  j = bj * 8 + ((w >> 3) & 7);
  k = bk * 8 + (w & 7);
}

// Eisenstein & Hu (1998) no-wiggle transfer function, k in h/Mpc (Sec. 4: the initial
// power spectrum uses the Eisenstein-Hu fitting function).
__host__ __device__ inline double eh_nowiggle_transfer(double k, double Om, double Ob,
                                                       double h, double Tcmb) {
  const double theta = Tcmb / 2.7;
  const double om_m = Om * h * h;
  const double om_b = Ob * h * h;
  const double fb = Ob / Om;
  const double s = 44.5 * log(9.83 / om_m) / sqrt(1.0 + 10.0 * pow(om_b, 0.75));
  const double ag = 1.0 - 0.328 * log(431.0 * om_m) * fb + 0.38 * log(22.3 * om_m) * fb * fb;
  const double ks = 0.43 * k * h * s;
  const double geff = Om * h * (ag + (1.0 - ag) / (1.0 + ks * ks * ks * ks));
  const double q = k * theta * theta / geff;
  const double L0 = log(2.0 * 2.718281828459045 + 1.8 * q);
  const double C0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return L0 / (L0 + C0 * q * q);
}

}  // namespace scola
