// Reverse mode of the tiled-sCOLA forward pass: d loss / d white noise for a loss on the
// output density.  The paper has no adjoint; every kernel here is the transpose of one
// forward operation (Sec. 3.1-3.4, App. A-C) and is derived from it:
//   output CiC              -> W'-gather of the density adjoint at the final positions
//   drift / kick (App. B)   -> linear updates of the particle adjoints (lam_x, lam_p) and
//                              FP64 accumulation of lam_Psi1, lam_Psi2
//   CiC interpolation and   -> one scalar scatter of beta lam_p through the transposed
//   central gradient           gradient stencil onto the padded nodes (shell part ->
//                              lam Phi_BC), and a W'-gather of lam_g . grad Phi
//   Dirichlet DST solve     -> the same solve (the FDA-2 Dirichlet Laplacian is symmetric)
//   CiC deposit B^sCOLA     -> W'-gather of lam_rho at the particle
//   Psi = D phi, Phi_BC^0, second-order source, IC filter -> their transposes (FP64)
// Positions are again formed in FP64 and take the same cells as in the forward pass; the
// piecewise-linear CiC weights are differentiated with the cell held fixed.
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"

namespace scola {

namespace {

__device__ inline int wrapn(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Position (FP64) of particle p with lattice site idx at a time with growth factors D1, D2
// and residual displacement x.
__device__ inline void lpt_position(const double (&s1)[3], const double (&s2)[3], const int (&idx)[3],
                                    double D1, double D2, const double (&x)[3], double (&u)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = lpt_base(idx[c] + 0.5, D1, s1[c], D2, s2[c]) + x[c];
}

// Cell and CiC weights of the interpolation at u (corners outside [0, M]^3 weigh nothing);
// returns false for a particle outside [-1, M+1)^3, which touches no node.
template <typename T>
__device__ inline bool interp_cell(int M, const double (&u)[3], int (&j0)[3], T (&f)[3]) {
  const double hiu = (double)M + 1.0;
  const bool in = u[0] >= -1.0 && u[0] < hiu && u[1] >= -1.0 && u[1] < hiu && u[2] >= -1.0 &&
                  u[2] < hiu;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    j0[c] = 0;
    f[c] = T(0);
    if (in) {
      const double fl = floor(u[c]);
      j0[c] = (int)fl;
      f[c] = (T)(u[c] - fl);
    }
  }
  return in;
}

// Gather half of a reverse step (transpose of deposit and interpolation at the force
// positions u of step g):
//   lam_u = sum_c grad W(u - n_c) [lam_g . grad Phi(n_c) + lam_rho(n_c)],
// the first term over the interpolation corners in [0, M]^3, the second over the interior
// deposit corners [1, M-1]^3.  The potential and lam_rho on the nodes of the block's
// stencils are staged in LDS: in the fixed kFw^3 windows when the block's extent fits
// (lam_rho zero off the interior, potential zero off the padded grid, where only
// zero-weight terms read it), else in a window sized to the extent (potential only), else
// read from global memory.  Every form sums the same terms in the same order.  Must be
// called by all threads of the block.
template <typename T>
__device__ __forceinline__ void block_adjoint_gather(const T* __restrict__ phi,
                                                     const T* __restrict__ lr, int M,
                                                     const double (&u)[3], const T (&lg)[3],
                                                     T* win, T* win2, int* bounds, T (&lu)[3]) {
  const int Mp = M + 3, n = M - 1;
  int j0[3];
  T f[3];
  const bool in = interp_cell<T>(M, u, j0, f);
  lu[0] = lu[1] = lu[2] = T(0);
  // the corner term with node values at(kx, ky, kz) = potential at j0 - 1 + k and
  // rho(dx, dy, dz) = lam_rho at corner j0 + d (zero off the interior)
  auto corners = [&](auto at, auto rho) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int d[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
      const int nx = j0[0] + d[0], ny = j0[1] + d[1], nz = j0[2] + d[2];
      const bool inr = nx >= 0 && nx <= M && ny >= 0 && ny <= M && nz >= 0 && nz <= M;
      T wa[3], dw[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) wa[q] = d[q] ? f[q] : T(1) - f[q];
      dw[0] = (d[0] ? T(1) : T(-1)) * wa[1] * wa[2];
      dw[1] = (d[1] ? T(1) : T(-1)) * wa[0] * wa[2];
      dw[2] = (d[2] ? T(1) : T(-1)) * wa[0] * wa[1];
      const T gx = T(0.5) * (at(2 + d[0], 1 + d[1], 1 + d[2]) - at(d[0], 1 + d[1], 1 + d[2]));
      const T gy = T(0.5) * (at(1 + d[0], 2 + d[1], 1 + d[2]) - at(1 + d[0], d[1], 1 + d[2]));
      const T gz = T(0.5) * (at(1 + d[0], 1 + d[1], 2 + d[2]) - at(1 + d[0], 1 + d[1], d[2]));
      T s = inr ? lg[0] * gx + lg[1] * gy + lg[2] * gz : T(0);
      s += rho(d[0], d[1], d[2]);
#pragma unroll
      for (int q = 0; q < 3; ++q) lu[q] += dw[q] * s;
    }
  };
  const CellRange cr = block_cells(in, j0, bounds);
  if (cr.any) {
    // the stencils of the block's particles span [min j0 - 1, max j0 + 2] per axis
    const int ox = cr.lo[0] - 1, oy = cr.lo[1] - 1, oz = cr.lo[2] - 1;
    const int ex = cr.hi[0] - ox + 3, ey = cr.hi[1] - oy + 3, ez = cr.hi[2] - oz + 3;
    if (ex <= kFw && ey <= kFw && ez <= kFw) {
      const int t = threadIdx.x, ty = t / kFw, tz = t % kFw;
      const int ny = oy + ty, nz = oz + tz;
      const bool cin = ty < ey && tz < ez;
      const bool colp = cin && ny >= -1 && ny <= M + 1 && nz >= -1 && nz <= M + 1;
      const bool colr = cin && ny >= 1 && ny <= n && nz >= 1 && nz <= n;
      const int xa = max(-1 - ox, 0), xb = min(M + 2 - ox, ex);     // padded-grid planes
      const int ra = max(1 - ox, 0), rb = min(n + 1 - ox, ex);      // interior planes
      const unsigned gp = colp ? (unsigned)(((ny + 1) * Mp + (nz + 1)) * (int)sizeof(T)) : 0u;
      const unsigned gr = colr ? (unsigned)(((ny - 1) * n + (nz - 1)) * (int)sizeof(T)) : 0u;
      T v[kFw], r[kFw];
#pragma unroll
      for (int xi = 0; xi < kFw; ++xi) v[xi] = r[xi] = T(0);
      if (colp) {
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi)
          if (xi >= xa && xi < xb) v[xi] = *byte_offset(phi + (int64_t)(ox + 1 + xi) * (Mp * Mp), gp);
      }
      if (colr) {
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi)
          if (xi >= ra && xi < rb) r[xi] = *byte_offset(lr + (int64_t)(ox - 1 + xi) * (n * n), gr);
      }
#pragma unroll
      for (int xi = 0; xi < kFw; ++xi)
        if (xi < ex) {
          win[t + kFwX * xi] = v[xi];
          win2[t + kFwX * xi] = r[xi];
        }
      __syncthreads();
      if (in) {
        const int base = (j0[0] - 1 - ox) * kFwX + (j0[1] - 1 - oy) * kFwY + (j0[2] - 1 - oz);
        const T* wp = win + base;
        const T* rp = win2 + base + kFwX + kFwY + 1;   // node j0
        corners([&](int kx, int ky, int kz) { return wp[kx * kFwX + ky * kFwY + kz]; },
                [&](int dx, int dy, int dz) { return rp[dx * kFwX + dy * kFwY + dz]; });
      }
    } else {
      // sized window over the padded grid, potential only
      const int lx = max(ox, -1), ly = max(oy, -1), lz = max(oz, -1);
      const int wx = min(cr.hi[0] + 2, M + 1) - lx + 1, wy = min(cr.hi[1] + 2, M + 1) - ly + 1,
                wz = min(cr.hi[2] + 2, M + 1) - lz + 1;
      const int wyz = wy * wz;
      const bool use_lds = wx * wyz <= kWindow;
      if (use_lds) {
        const float inv_wz = 1.0f / (float)wz;
        const unsigned gstep = (unsigned)(Mp * Mp);
        for (int pos = threadIdx.x; pos < wyz; pos += blockDim.x) {
          const int ey2 = (int)(((float)pos + 0.5f) * inv_wz), ez2 = pos - ey2 * wz;
          unsigned widx = (unsigned)pos;
          unsigned gidx = idx3(lx + 1, ly + ey2 + 1, lz + ez2 + 1, Mp, Mp);
#pragma unroll 4
          for (int x = 0; x < wx; ++x, widx += (unsigned)wyz, gidx += gstep) win[widx] = phi[gidx];
        }
      }
      __syncthreads();
      if (in) {
        auto cl = [&](int v) { return min(max(v, -1), M + 1); };
        auto rho = [&](int dx, int dy, int dz) -> T {
          const int x = j0[0] + dx, y = j0[1] + dy, z = j0[2] + dz;
          if (x >= 1 && x <= n && y >= 1 && y <= n && z >= 1 && z <= n)
            return lr[idx3(x - 1, y - 1, z - 1, n, n)];
          return T(0);
        };
        if (use_lds)
          corners([&](int kx, int ky, int kz) {
            return win[idx3(cl(j0[0] - 1 + kx) - lx, cl(j0[1] - 1 + ky) - ly,
                            cl(j0[2] - 1 + kz) - lz, wy, wz)];
          }, rho);
        else
          corners([&](int kx, int ky, int kz) {
            return phi[idx3(cl(j0[0] - 1 + kx) + 1, cl(j0[1] - 1 + ky) + 1,
                            cl(j0[2] - 1 + kz) + 1, Mp, Mp)];
          }, rho);
      }
    }
  }
  __syncthreads();   // the windows and `bounds` are free again
}

// Scatter half of a reverse step: the transpose of "central gradient, then CiC
// interpolation at u" applied to the particle's lam_g, i.e.
//   lam_Phi(n) += sum_a lam_g_a sum_c W(u - n_c) (delta(n, n_c + e_a) - delta(n, n_c - e_a)) / 2
// over the interpolation corners n_c in [0, M]^3.  Along axis a this is a 4-point stencil
// {-w0, -w1, w0, w1} / 2 on nodes j0 - 1 .. j0 + 2, times the CiC weights across; the union
// is the 2x2x2 corner block plus six 2x2 arms, 32 nodes in all.  Every node with a non-zero
// coefficient lies in [-1, M+1]^3.  Interior nodes [1, M-1]^3 feed the adjoint Poisson
// solve (`work`, zeroed beforehand); shell nodes hold D1 Phi_BC^0, so D1 lam_Phi goes to
// lam_bc0.
//
// The block privatises its nodes in an LDS window of integers: LDS atomics on integers
// run at full rate while floating-point LDS atomics serialise.  Each contribution is
// rounded to a fixed-point grid of step 2^(e + 9 - Q) with 2^e above the block's largest
// |lam_g| and Q = 30 (FP32 plans, int32) or 62 (FP64 plans, int64): a node receives at
// most 256 particles x 1.5 |lam_g| < 2^(e + 9), so sums cannot overflow, and the rounding
// error per contribution is below 2^(-Q + 8) of the block's largest |lam_g| (2^-22 for
// FP32, 2^-54 for FP64).  The window (fixed kFw^3 geometry when the block's extent fits,
// else sized to it) is flushed with floating-point atomics to global memory; blocks whose
// footprint exceeds both add straight into global memory.  Must be called by all threads.
template <typename T>
__device__ __forceinline__ void block_adjoint_scatter(T* __restrict__ work,
                                                      double* __restrict__ lam_bc0, double D1,
                                                      int M, const double (&u)[3],
                                                      const T (&lg)[3], T* win_raw,
                                                      int* bounds) {
  using Q = typename std::conditional<std::is_same<T, float>::value, int, long long>::type;
  using UQ = typename std::make_unsigned<Q>::type;
  constexpr int kQ = std::is_same<T, float>::value ? 30 : 62;
  static_assert(sizeof(Q) == sizeof(T), "the integer window reuses the potential window");
  Q* win = reinterpret_cast<Q*>(win_raw);
  const int Mp = M + 3, n = M - 1;
  int j0[3];
  T f[3];
  const bool in = interp_cell<T>(M, u, j0, f);
  T w[3][2], h[3][4];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a][0] = (j0[a] < 0 || j0[a] > M) ? T(0) : T(1) - f[a];
    w[a][1] = (j0[a] + 1 < 0 || j0[a] + 1 > M) ? T(0) : f[a];
    h[a][0] = T(-0.5) * w[a][0];    // node j0 - 1
    h[a][1] = T(-0.5) * w[a][1];    // node j0
    h[a][2] = T(0.5) * w[a][0];     // node j0 + 1
    h[a][3] = T(0.5) * w[a][1];     // node j0 + 2
  }
  constexpr int kNoExp = -900;
  int ex_l = kNoExp;
  if (in) {
    const double mx = (double)fmax(fmax(fabs(lg[0]), fabs(lg[1])), fabs(lg[2]));
    if (mx > 0.0) frexp(mx, &ex_l);
  }
  int emax_b;
  const CellRange cr = block_cells_max(in, j0, ex_l, bounds, emax_b);
  if (!cr.any) return;
  const int emax = max(emax_b, kNoExp);
  const double qscale = ldexp(1.0, kQ - 9 - emax), qstep = ldexp(1.0, emax + 9 - kQ);
  auto to_global = [&](int x, int y, int z, T v) {
    if (x >= 1 && x <= n && y >= 1 && y <= n && z >= 1 && z <= n)
      unsafeAtomicAdd(work + idx3(x - 1, y - 1, z - 1, n, n), v);
    else
      unsafeAtomicAdd(lam_bc0 + idx3(x + 1, y + 1, z + 1, Mp, Mp), D1 * (double)v);
  };
  // the 32 contributions: node offset k = 0..3 from j0 - 1 per axis and value
  auto contributions = [&](auto add) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
      const T kx = h[0][dx + 1] * w[1][dy] * w[2][dz];
      const T ky = w[0][dx] * h[1][dy + 1] * w[2][dz];
      const T kz = w[0][dx] * w[1][dy] * h[2][dz + 1];
      add(1 + dx, 1 + dy, 1 + dz, (kx != T(0) || ky != T(0) || kz != T(0)),
          lg[0] * kx + lg[1] * ky + lg[2] * kz);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int o = e ? 3 : 0, hk = e ? 3 : 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = (q >> 1) & 1, s = q & 1;
        const T kx = h[0][hk] * w[1][r] * w[2][s];
        add(o, 1 + r, 1 + s, kx != T(0), lg[0] * kx);
        const T ky = w[0][r] * h[1][hk] * w[2][s];
        add(1 + r, o, 1 + s, ky != T(0), lg[1] * ky);
        const T kz = w[0][r] * w[1][s] * h[2][hk];
        add(1 + r, 1 + s, o, kz != T(0), lg[2] * kz);
      }
    }
  };
  // stencil nodes of the block span [min j0 - 1, max j0 + 2] per axis
  const int ox = cr.lo[0] - 1, oy = cr.lo[1] - 1, oz = cr.lo[2] - 1;
  const int ex = cr.hi[0] - ox + 3, ey = cr.hi[1] - oy + 3, ez = cr.hi[2] - oz + 3;
  if (ex <= kFw && ey <= kFw && ez <= kFw) {
    const int t = threadIdx.x, ty = t / kFw, tz = t % kFw;
#pragma unroll
    for (int xi = 0; xi < kFw; ++xi)
      if (xi < ex) win[t + kFwX * xi] = Q(0);
    __syncthreads();
    if (in) {
      // zero contributions add nothing, so every node is added unconditionally
      UQ* qp = reinterpret_cast<UQ*>(win) + (j0[0] - 1 - ox) * kFwX + (j0[1] - 1 - oy) * kFwY +
               (j0[2] - 1 - oz);
      contributions([&](int kx, int ky, int kz, bool, T v) {
        atomicAdd(qp + kx * kFwX + ky * kFwY + kz, (UQ)(Q)__double2ll_rn((double)v * qscale));
      });
    }
    __syncthreads();
    const int ny = oy + ty, nz = oz + tz;
    if (ty < ey && tz < ez && ny >= -1 && ny <= M + 1 && nz >= -1 && nz <= M + 1) {
      const int xa = max(-1 - ox, 0), xb = min(M + 2 - ox, ex);
      Q qv[kFw];
#pragma unroll
      for (int xi = 0; xi < kFw; ++xi) qv[xi] = (xi >= xa && xi < xb) ? win[t + kFwX * xi] : Q(0);
#pragma unroll
      for (int xi = 0; xi < kFw; ++xi)
        if (qv[xi] != Q(0)) to_global(ox + xi, ny, nz, (T)((double)qv[xi] * qstep));
    }
    return;
  }
  // sized window over the padded grid
  const int lx = max(ox, -1), ly = max(oy, -1), lz = max(oz, -1);
  const int wx = min(cr.hi[0] + 2, M + 1) - lx + 1, wy = min(cr.hi[1] + 2, M + 1) - ly + 1,
            wz = min(cr.hi[2] + 2, M + 1) - lz + 1;
  const int wyz = wy * wz;
  const bool use_lds = wx * wyz <= kWindow;
  if (use_lds) {
    for (int e = threadIdx.x; e < wx * wyz; e += blockDim.x) win[e] = Q(0);
    __syncthreads();
  }
  if (in) {
    // a node is touched only through a non-zero coefficient, which keeps it in [-1, M+1]^3
    contributions([&](int kx, int ky, int kz, bool nonzero, T v) {
      if (!nonzero) return;
      const int x = j0[0] - 1 + kx, y = j0[1] - 1 + ky, z = j0[2] - 1 + kz;
      if (use_lds)
        atomicAdd(reinterpret_cast<UQ*>(win) + idx3(x - lx, y - ly, z - lz, wy, wz),
                  (UQ)(Q)__double2ll_rn((double)v * qscale));
      else
        to_global(x, y, z, v);
    });
  }
  if (use_lds) {
    __syncthreads();
    // flush: each thread takes a (y, z) column of the window and walks it along x
    const float inv_wz = 1.0f / (float)wz;
    for (int pos = threadIdx.x; pos < wyz; pos += blockDim.x) {
      const int ey2 = (int)(((float)pos + 0.5f) * inv_wz), ez2 = pos - ey2 * wz;
      unsigned widx = (unsigned)pos;
      for (int x = 0; x < wx; ++x, widx += (unsigned)wyz) {
        const Q q = win[widx];
        if (q != Q(0)) to_global(lx + x, ly + ey2, lz + ez2, (T)((double)q * qstep));
      }
    }
  }
}

// One reverse step on the particles, two halves fused so each particle's adjoint state and
// Psi are streamed once:
//   GATHER  (force of step g = k+1): lam_x += lam_u(u_g) with lam_g = beta_g lam_p;
//   SCATTER (kick and drift of step k, App. B): lam_p += alpha lam_x (drift transpose),
//           lam_g = beta lam_p (kick transpose), then the interpolation/gradient transpose of
//           lam_g at u_k into the nodes;
// and the Psi terms: u = q - D1 Psi1 + D2 Psi2 + x_res gives lam_Psi1 -= D1 lam_u,
// lam_Psi2 += D2 lam_u; the kick's -D1 Psi1 + (D2 - D1^2) Psi2 gives lam_Psi1 -= beta D1
// lam_p, lam_Psi2 += beta (D2 - D1^2) lam_p.  Positions are formed in FP64 exactly as in the
// forward pass, so every particle takes the cell it took there.
template <typename T, bool GATHER, bool SCATTER>
__global__ void __launch_bounds__(kBlock) k_adj_particles(AdjointArgs<T> a, BlockMap m) {
  const int L = logical_block(m);
  if (L >= m.count) return;
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int M = t.M;
  const int64_t pl = (int64_t)m.local[b] * kBlock + threadIdx.x;
  const int64_t p = t.p_off + pl;
  const int64_t P = a.P;
  int idx[3];
  brick_site(pl, M, idx[0], idx[1], idx[2]);
  double s1[3], s2[3], acc1[3], acc2[3];
  T lx[3], lp[3], xsc[3], lq1[3], lq2[3];
  // every particle stream of the pass is loaded up front, so the block waits on global
  // memory once before its windows are staged; the streams are touched once per step, so
  // they are read and written non-temporally (they do not compete for cache lines with the
  // meshes that neighbouring blocks reuse)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s1[c] = (double)__builtin_nontemporal_load(a.psi1 + c * P + p);
    s2[c] = (double)__builtin_nontemporal_load(a.psi2 + c * P + p);
    lx[c] = __builtin_nontemporal_load(a.lam_x + c * P + p);
    lp[c] = __builtin_nontemporal_load(a.lam_p + c * P + p);
    if (SCATTER) xsc[c] = __builtin_nontemporal_load(a.xs + c * P + p);
    lq1[c] = __builtin_nontemporal_load(a.lam_psi1 + c * P + p);
    lq2[c] = __builtin_nontemporal_load(a.lam_psi2 + c * P + p);
    acc1[c] = acc2[c] = 0.0;
  }
  __shared__ T win[kWindow];
  __shared__ T win2[GATHER ? kWindow : 1];   // lam_rho window of the gather half
  __shared__ int bounds[kCellScratch];
  if constexpr (GATHER) {
    double x[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = (double)__builtin_nontemporal_load(a.xg + c * P + p);
    lpt_position(s1, s2, idx, a.D1g, a.D2g, x, u);
    T lg[3], lu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) lg[c] = (T)a.beta_g * lp[c];
    block_adjoint_gather<T>(a.phi + t.h_off, a.lam_rho + t.g_off, M, u, lg, win, win2, bounds,
                            lu);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lx[c] += lu[c];
      acc1[c] -= a.D1g * (double)lu[c];
      acc2[c] += a.D2g * (double)lu[c];
    }
  }
  if constexpr (SCATTER) {
    const double d2 = a.D2 - a.D1 * a.D1;
    T lg[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lp[c] += (T)a.alpha * lx[c];
      lg[c] = (T)a.beta * lp[c];
      acc1[c] -= a.beta * a.D1 * (double)lp[c];
      acc2[c] += a.beta * d2 * (double)lp[c];
    }
    double x[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = (double)xsc[c];
    lpt_position(s1, s2, idx, a.D1, a.D2, x, u);
    block_adjoint_scatter<T>(a.work + t.g_off, a.lam_bc0 + t.h_off, a.D1, M, u, lg, win, bounds);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (GATHER) __builtin_nontemporal_store(lx[c], a.lam_x + c * P + p);
    if (SCATTER) __builtin_nontemporal_store(lp[c], a.lam_p + c * P + p);
    __builtin_nontemporal_store(lq1[c] + (T)acc1[c], a.lam_psi1 + c * P + p);
    __builtin_nontemporal_store(lq2[c] + (T)acc2[c], a.lam_psi2 + c * P + p);
  }
}

// Transpose of the output density (Sec. 4.1 CiC of the core particles on N_out^3 nodes):
// lam_u = s^4 sum_c W'(s u_g - n_c) lam_delta(n_c) with s = N_out / N_p; this seeds the
// particle adjoints at the final time: lam_x = lam_u, lam_p = 0, lam_Psi1 = -D1 lam_u,
// lam_Psi2 = D2 lam_u (buffer particles: zero).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_output(AdjointArgs<T> a, BlockMap m,
                                                       const T* __restrict__ lam_dens, int Np,
                                                       int N_out) {
  const int L = logical_block(m);
  if (L >= m.count) return;
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int M = t.M;
  const int64_t pl = (int64_t)m.local[b] * kBlock + threadIdx.x;
  const int64_t p = t.p_off + pl;
  const int64_t P = a.P;
  int i, j, k;
  brick_site(pl, M, i, j, k);
  const int lo = t.core_lo[0], hi = t.core_lo[0] + t.core_n;
  const bool core = i >= lo && i < hi && j >= lo && j < hi && k >= lo && k < hi;
  T lu[3] = {T(0), T(0), T(0)};
  if (core) {
    double s1[3], s2[3], x[3], u[3];
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s1[c] = a.psi1[c * P + p];
      s2[c] = a.psi2[c * P + p];
      x[c] = (double)a.xg[c * P + p];
    }
    lpt_position(s1, s2, idx, a.D1g, a.D2g, x, u);
    const double s = (double)N_out / (double)Np;
    int j0[3];
    T f[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double uo = (t.origin[c] + u[c]) * s;
      const double fl = floor(uo);
      f[c] = (T)(uo - fl);
      j0[c] = wrapn((int)fmod(fl, (double)N_out), N_out);
    }
    const T scale = (T)(s * s * s * s);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int d[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
      T wa[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) wa[q] = d[q] ? f[q] : T(1) - f[q];
      const int nx = (j0[0] + d[0]) % N_out, ny = (j0[1] + d[1]) % N_out,
                nz = (j0[2] + d[2]) % N_out;
      const T v = scale * lam_dens[((int64_t)nx * N_out + ny) * N_out + nz];
      lu[0] += (d[0] ? T(1) : T(-1)) * wa[1] * wa[2] * v;
      lu[1] += (d[1] ? T(1) : T(-1)) * wa[0] * wa[2] * v;
      lu[2] += (d[2] ? T(1) : T(-1)) * wa[0] * wa[1] * v;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.lam_x[c * P + p] = lu[c];
    a.lam_p[c * P + p] = T(0);
    a.lam_psi1[c * P + p] = (T)(-a.D1g * (double)lu[c]);
    a.lam_psi2[c * P + p] = (T)(a.D2g * (double)lu[c]);
  }
}

// ---- set-up adjoint (FP64) -----------------------------------------------------------------

// Box particles -> global lattice sites: lam_Psi_global += lam_Psi (boxes overlap in their
// buffers, hence the atomics).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_psi_scatter(const TileDesc* __restrict__ tiles,
                                                            const int* __restrict__ blk_tile,
                                                            const int* __restrict__ blk_first,
                                                            const T* __restrict__ lp1,
                                                            const T* __restrict__ lp2,
                                                            double* __restrict__ g, int N,
                                                            int64_t P) {
  const TileDesc t = tiles[blk_tile[blockIdx.x]];
  const int M = t.M;
  const int64_t pl = (int64_t)blk_first[blockIdx.x] * kBlock + threadIdx.x;
  int i, j, k;
  brick_site(pl, M, i, j, k);
  const int64_t p = t.p_off + pl;
  const int64_t N3 = (int64_t)N * N * N;
  const int64_t gs = ((int64_t)wrapn(t.origin[0] + i, N) * N + wrapn(t.origin[1] + j, N)) * N +
                     wrapn(t.origin[2] + k, N);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v1 = (double)lp1[c * P + p], v2 = (double)lp2[c * P + p];
    if (v1 != 0.0) unsafeAtomicAdd(g + c * N3 + gs, v1);
    if (v2 != 0.0) unsafeAtomicAdd(g + (3 + c) * N3 + gs, v2);
  }
}

// Transpose of Phi_BC^0 = mean of the 8 LPT nodes around each shell node.
__global__ void k_adj_boundary(const TileDesc* __restrict__ tiles, int n_tiles,
                               const double* __restrict__ lam_bc0, double* __restrict__ lam_phi1,
                               int N) {
  const int ti = blockIdx.y;
  if (ti >= n_tiles) return;
  const TileDesc t = tiles[ti];
  const int Mp = t.M + 3;
  const int64_t n3 = (int64_t)Mp * Mp * Mp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n3;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double v = lam_bc0[t.h_off + e];
    if (v == 0.0) continue;
    const int a = (int)(e / ((int64_t)Mp * Mp)) - 1, b = (int)((e / Mp) % Mp) - 1,
              c = (int)(e % Mp) - 1;
    const int gx = t.origin[0] + a, gy = t.origin[1] + b, gz = t.origin[2] + c;
    for (int dx = -1; dx <= 0; ++dx)
      for (int dy = -1; dy <= 0; ++dy)
        for (int dz = -1; dz <= 0; ++dz)
          unsafeAtomicAdd(lam_phi1 + ((int64_t)wrapn(gx + dx, N) * N + wrapn(gy + dy, N)) * N +
                              wrapn(gz + dz, N), 0.125 * v);
  }
}

// Transpose of Psi = D phi (central difference, periodic): D^T f (q) = (f(q-e) - f(q+e)) / 2.
// lam_phi1 += D^T lam_Psi1_global; the second-order part D^T lam_Psi2_global goes to the
// complex FFT buffer.
__global__ void k_adj_phi_from_psi(const double* __restrict__ g, double* __restrict__ lam_phi1,
                                   double2* __restrict__ cbuf, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N3 = (int64_t)N * N * N;
  if (i >= N3) return;
  const int x = (int)(i / ((int64_t)N * N)), y = (int)((i / N) % N), z = (int)(i % N);
  auto at = [&](int c, int dx, int dy, int dz) {
    return g[c * N3 + ((int64_t)wrapn(x + dx, N) * N + wrapn(y + dy, N)) * N + wrapn(z + dz, N)];
  };
  double a1 = 0.5 * (at(0, -1, 0, 0) - at(0, 1, 0, 0) + at(1, 0, -1, 0) - at(1, 0, 1, 0) +
                     at(2, 0, 0, -1) - at(2, 0, 0, 1));
  double a2 = 0.5 * (at(3, -1, 0, 0) - at(3, 1, 0, 0) + at(4, 0, -1, 0) - at(4, 0, 1, 0) +
                     at(5, 0, 0, -1) - at(5, 0, 0, 1));
  lam_phi1[i] += a1;
  cbuf[i] = make_double2(a2, 0.0);
}

// Fields of the second-order source transpose: with S = sum_{i>j} [phi_,ii phi_,jj -
// phi_,ij^2], dS/dphi^T lam_S = sum_i D_iD_i (lam_S sum_{j != i} phi_,jj)
//                             - 2 sum_{i>j} D_iD_j (lam_S phi_,ij).
// Writes B_i = lam_S sum_{j != i} phi_,jj (3 fields) and C_ij = lam_S phi_,ij (3 fields).
__global__ void k_adj_source_fields(const double* __restrict__ phi, const double* __restrict__ lam_s,
                                    double* __restrict__ f6, int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N3 = (int64_t)N * N * N;
  if (i >= N3) return;
  const int x = (int)(i / ((int64_t)N * N)), y = (int)((i / N) % N), z = (int)(i % N);
  auto P = [&](int dx, int dy, int dz) {
    return phi[((int64_t)wrapn(x + dx, N) * N + wrapn(y + dy, N)) * N + wrapn(z + dz, N)];
  };
  const double c0 = P(0, 0, 0);
  const double xx = 0.25 * (P(2, 0, 0) - 2.0 * c0 + P(-2, 0, 0));
  const double yy = 0.25 * (P(0, 2, 0) - 2.0 * c0 + P(0, -2, 0));
  const double zz = 0.25 * (P(0, 0, 2) - 2.0 * c0 + P(0, 0, -2));
  const double xy = 0.25 * (P(1, 1, 0) - P(1, -1, 0) - P(-1, 1, 0) + P(-1, -1, 0));
  const double xz = 0.25 * (P(1, 0, 1) - P(1, 0, -1) - P(-1, 0, 1) + P(-1, 0, -1));
  const double yz = 0.25 * (P(0, 1, 1) - P(0, 1, -1) - P(0, -1, 1) + P(0, -1, -1));
  const double l = lam_s[i];
  f6[0 * N3 + i] = l * (yy + zz);
  f6[1 * N3 + i] = l * (xx + zz);
  f6[2 * N3 + i] = l * (xx + yy);
  f6[3 * N3 + i] = l * xy;
  f6[4 * N3 + i] = l * xz;
  f6[5 * N3 + i] = l * yz;
}

__global__ void k_adj_source_apply(const double* __restrict__ f6, double* __restrict__ lam_phi1,
                                   int N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N3 = (int64_t)N * N * N;
  if (i >= N3) return;
  const int x = (int)(i / ((int64_t)N * N)), y = (int)((i / N) % N), z = (int)(i % N);
  auto F = [&](int c, int dx, int dy, int dz) {
    return f6[c * N3 + ((int64_t)wrapn(x + dx, N) * N + wrapn(y + dy, N)) * N + wrapn(z + dz, N)];
  };
  auto dd = [&](int c, int a) {   // D_a D_a applied to field c (wide second difference)
    const int e[3] = {a == 0, a == 1, a == 2};
    return 0.25 * (F(c, 2 * e[0], 2 * e[1], 2 * e[2]) - 2.0 * F(c, 0, 0, 0) +
                   F(c, -2 * e[0], -2 * e[1], -2 * e[2]));
  };
  auto dm = [&](int c, int a, int b) {   // D_a D_b applied to field c
    int ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
    ea[a] = 1;
    eb[b] = 1;
    return 0.25 * (F(c, ea[0] + eb[0], ea[1] + eb[1], ea[2] + eb[2]) -
                   F(c, ea[0] - eb[0], ea[1] - eb[1], ea[2] - eb[2]) -
                   F(c, -ea[0] + eb[0], -ea[1] + eb[1], -ea[2] + eb[2]) +
                   F(c, -ea[0] - eb[0], -ea[1] - eb[1], -ea[2] - eb[2]));
  };
  lam_phi1[i] += dd(0, 0) + dd(1, 1) + dd(2, 2) -
                 2.0 * (dm(3, 0, 1) + dm(4, 0, 2) + dm(5, 1, 2));
}

__global__ void k_real_to_complex_adj(const double* __restrict__ in, double2* __restrict__ out,
                                      int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2(in[i], 0.0);
}

}  // namespace

template <typename T>
hipError_t launch_adj_output(const AdjointArgs<T>& a, const BlockMap& m, const T* lam_dens,
                             int Np, int N_out, hipStream_t s) {
  if (m.count > 0)
    hipLaunchKernelGGL(k_adj_output<T>, dim3(padded_grid(m)), dim3(kBlock), 0, s, a, m, lam_dens,
                       Np, N_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_step(const AdjointArgs<T>& a, const BlockMap& part, bool gather,
                           bool scatter, hipStream_t s) {
  if (part.count == 0) return hipSuccess;
  const dim3 grid(padded_grid(part)), block(kBlock);
  if (gather && scatter)
    hipLaunchKernelGGL((k_adj_particles<T, true, true>), grid, block, 0, s, a, part);
  else if (gather)
    hipLaunchKernelGGL((k_adj_particles<T, true, false>), grid, block, 0, s, a, part);
  else if (scatter)
    hipLaunchKernelGGL((k_adj_particles<T, false, true>), grid, block, 0, s, a, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_adj_setup_scatter(const BoxSetupArgs& b, const T* lam_psi1,
                                    const T* lam_psi2, double* lam_psig,
                                    const double* lam_bc0, double* lam_phi1, hipStream_t s) {
  if (b.n_blocks > 0)
    hipLaunchKernelGGL(k_adj_psi_scatter<T>, dim3(b.n_blocks), dim3(kBlock), 0, s, b.tiles,
                       b.blk_tile, b.blk_first, lam_psi1, lam_psi2, lam_psig, b.N, b.P);
  hipLaunchKernelGGL(k_adj_boundary, dim3(64, b.n_tiles), dim3(kBlock), 0, s, b.tiles, b.n_tiles,
                     lam_bc0, lam_phi1, b.N);
  return hipGetLastError();
}

hipError_t launch_adj_phi_from_psi(const double* lam_psig, double* lam_phi1, double2* cbuf,
                                   int N, hipStream_t s) {
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_adj_phi_from_psi, dim3((unsigned)((n3 + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, lam_psig, lam_phi1, cbuf, N);
  return hipGetLastError();
}

hipError_t launch_adj_source(const double* phi1, const double* lam_s, double* f6,
                             double* lam_phi1, int N, hipStream_t s) {
  const int64_t n3 = (int64_t)N * N * N;
  const unsigned g = (unsigned)((n3 + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adj_source_fields, dim3(g), dim3(kBlock), 0, s, phi1, lam_s, f6, N);
  hipLaunchKernelGGL(k_adj_source_apply, dim3(g), dim3(kBlock), 0, s, f6, lam_phi1, N);
  return hipGetLastError();
}

hipError_t launch_real_to_complex(const double* in, double2* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_real_to_complex_adj, dim3((unsigned)((n + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}

template hipError_t launch_adj_output<float>(const AdjointArgs<float>&, const BlockMap&,
                                             const float*, int, int, hipStream_t);
template hipError_t launch_adj_output<double>(const AdjointArgs<double>&, const BlockMap&,
                                              const double*, int, int, hipStream_t);
template hipError_t launch_adj_setup_scatter<float>(const BoxSetupArgs&, const float*,
                                                    const float*, double*, const double*, double*,
                                                    hipStream_t);
template hipError_t launch_adj_setup_scatter<double>(const BoxSetupArgs&, const double*,
                                                     const double*, double*, const double*,
                                                     double*, hipStream_t);
template hipError_t launch_adj_step<float>(const AdjointArgs<float>&, const BlockMap&, bool, bool,
                                           hipStream_t);
template hipError_t launch_adj_step<double>(const AdjointArgs<double>&, const BlockMap&, bool,
                                            bool, hipStream_t);

}  // namespace scola
