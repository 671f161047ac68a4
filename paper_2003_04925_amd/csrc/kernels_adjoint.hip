// Reverse mode of the tiled-sCOLA forward pass: d loss / d white noise for a loss on the
// output density.  The paper has no adjoint; every kernel here is the transpose of one
// forward operation (Sec. 3.1-3.4, App. A-C) and is derived from it:
//   output CiC              -> W'-gather of the density adjoint at the final positions
//   drift / kick (App. B)   -> linear updates of the particle adjoints (lam_x, lam_p) and
//                              FP64 accumulation of lam_Psi1, lam_Psi2
//   CiC interpolation       -> 3-component CiC scatter of beta lam_p onto the nodes, and a
//                              W'-gather of lam_g . grad Phi at the particle
//   central gradient        -> minus the central divergence; shell part -> lam Phi_BC
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

__device__ inline void atomic_add_real(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add_real(double* p, double v) { unsafeAtomicAdd(p, v); }

// Position at the step's time (FP64) of particle p with lattice site (i, j, k).
template <typename T>
__device__ inline void particle_position(const AdjointArgs<T>& a, int64_t p, int i, int j,
                                         int k, double (&s1)[3], double (&s2)[3], double (&u)[3]) {
  const int idx[3] = {i, j, k};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s1[c] = a.psi1[c * a.P + p];
    s2[c] = a.psi2[c * a.P + p];
    u[c] = idx[c] + 0.5 - a.D1 * s1[c] + a.D2 * s2[c] + (double)a.xk[c * a.P + p];
  }
}

// Pass A of one reverse step: through the drift (lam_p += alpha lam_x) and the kick (lam_g
// = beta lam_p, Psi terms of K~), then the interpolation transpose: lam_G(n) += W(u - n)
// lam_g for the corners n in [0, M]^3, privatised per block in an LDS window (one
// component at a time), floating-point atomics to global memory.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_scatter(AdjointArgs<T> a, BlockMap m) {
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
  double s1[3], s2[3], u[3];
  particle_position(a, p, i, j, k, s1, s2, u);
  T lg[3];
  const double d2 = a.D2 - a.D1 * a.D1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T lt = a.lam_p[c * P + p] + (T)a.alpha * a.lam_x[c * P + p];
    a.lam_p[c * P + p] = lt;
    lg[c] = (T)a.beta * lt;
    a.lam_psi1[c * P + p] += -a.beta * a.D1 * (double)lt;
    a.lam_psi2[c * P + p] += a.beta * d2 * (double)lt;
  }
  // interpolation corners and weights (corners outside [0, M]^3 carry no weight)
  const double hiu = (double)M + 1.0;
  const bool in = u[0] >= -1.0 && u[0] < hiu && u[1] >= -1.0 && u[1] < hiu && u[2] >= -1.0 &&
                  u[2] < hiu;
  int j0[3] = {0, 0, 0};
  T w[3][2];
  int lo[3], hi[3];
  bool any = in;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T f = T(0);
    if (in) {
      const double fl = floor(u[c]);
      j0[c] = (int)fl;
      f = (T)(u[c] - fl);
    }
    w[c][0] = (j0[c] < 0 || j0[c] > M) ? T(0) : T(1) - f;
    w[c][1] = (j0[c] + 1 < 0 || j0[c] + 1 > M) ? T(0) : f;
    lo[c] = max(j0[c], 0);
    hi[c] = min(j0[c] + 1, M);
    any = any && lo[c] <= hi[c];
  }
  __shared__ T win[kWindow];
  __shared__ int bounds[6];
  block_bounds(any, lo, hi, bounds);
  const int lx = bounds[0], ly = bounds[1], lz = bounds[2];
  const int wx = bounds[3] - lx + 1, wy = bounds[4] - ly + 1, wz = bounds[5] - lz + 1;
  const bool empty = wx <= 0 || wy <= 0 || wz <= 0;
  const int vol = empty ? 0 : wx * wy * wz;
  const bool use_lds = !empty && vol <= kWindow;
  const int Mp = M + 3;
  const int64_t Hs = a.H;
  for (int comp = 0; comp < 3; ++comp) {
    T* dst = a.lam_G + comp * Hs + t.h_off;
    if (use_lds) {
      for (int e = threadIdx.x; e < vol; e += blockDim.x) win[e] = T(0);
      __syncthreads();
    }
    if (any) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
        const T wc = w[0][dx] * w[1][dy] * w[2][dz];
        if (wc == T(0)) continue;
        const int nx = j0[0] + dx, ny = j0[1] + dy, nz = j0[2] + dz;
        if (use_lds)
          atomicAdd(win + ((nx - lx) * wy + (ny - ly)) * wz + (nz - lz), wc * lg[comp]);
        else
          atomic_add_real(dst + ((int64_t)(nx + 1) * Mp + (ny + 1)) * Mp + (nz + 1),
                          wc * lg[comp]);
      }
    }
    if (use_lds) {
      __syncthreads();
      const int wyz = wy * wz;
      const float inv_wz = 1.0f / (float)wz, inv_wyz = 1.0f / (float)wyz;
      for (int e = threadIdx.x; e < vol; e += blockDim.x) {
        const T v = win[e];
        if (v != T(0)) {
          int ex, ey, ez;
          window_coords(e, wz, wyz, inv_wz, inv_wyz, ex, ey, ez);
          atomic_add_real(dst + ((int64_t)(lx + ex + 1) * Mp + (ly + ey + 1)) * Mp +
                              (lz + ez + 1), v);
        }
      }
      __syncthreads();
    }
  }
}

// Transpose of the central gradient: lam_Phi(i) = 1/2 sum_a (lam_G_a(i - e_a) -
// lam_G_a(i + e_a)) on [-1, M+1]^3 (lam_G vanishes outside [0, M]^3).  Interior nodes feed
// the adjoint Poisson solve (written to `work`); shell nodes are the LEP boundary values
// D1 Phi_BC^0, so lam_bc0 += D1 lam_Phi there.
template <typename T>
__global__ void k_adj_divergence(AdjointArgs<T> a, T* __restrict__ work, double* __restrict__ lam_bc0,
                                 int n_tiles) {
  const int ti = blockIdx.y;
  if (ti >= n_tiles) return;
  const TileDesc t = a.tiles[ti];
  const int M = t.M, Mp = M + 3, n = M - 1;
  const int64_t n3 = (int64_t)Mp * Mp * Mp;
  const T* G0 = a.lam_G + t.h_off;
  const T* G1 = G0 + a.H;
  const T* G2 = G1 + a.H;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n3;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int A = (int)(e / ((int64_t)Mp * Mp)), B = (int)((e / Mp) % Mp), C = (int)(e % Mp);
    T v = T(0);
    const int64_t sx = (int64_t)Mp * Mp, sy = Mp;
    if (A >= 1) v += G0[e - sx];
    if (A + 1 < Mp) v -= G0[e + sx];
    if (B >= 1) v += G1[e - sy];
    if (B + 1 < Mp) v -= G1[e + sy];
    if (C >= 1) v += G2[e - 1];
    if (C + 1 < Mp) v -= G2[e + 1];
    v *= T(0.5);
    const int ix = A - 1, iy = B - 1, iz = C - 1;      // node coordinates
    if (ix >= 1 && ix <= n && iy >= 1 && iy <= n && iz >= 1 && iz <= n)
      work[t.g_off + ((int64_t)(ix - 1) * n + (iy - 1)) * n + (iz - 1)] = v;
    else
      lam_bc0[t.h_off + e] += a.D1 * (double)v;
  }
}

// Pass B of one reverse step: lam_u = sum_c W'(u - n_c) [lam_g . grad Phi(n_c)] over the
// interpolation corners plus sum_c W'(u - n_c) lam_rho(n_c) over the interior deposit
// corners; then lam_x += lam_u and the Psi terms of u = q - D1 Psi1 + D2 Psi2 + x_res.
// Also clears this block's slice of lam_G for the next reverse step.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_gather(AdjointArgs<T> a, BlockMap m) {
  const int L = logical_block(m);
  if (L >= m.count) return;
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int M = t.M, Mp = M + 3, n = M - 1;
  const int64_t pl = (int64_t)m.local[b] * kBlock + threadIdx.x;
  const int64_t p = t.p_off + pl;
  const int64_t P = a.P;
  int i, j, k;
  brick_site(pl, M, i, j, k);
  double s1[3], s2[3], u[3];
  particle_position(a, p, i, j, k, s1, s2, u);
  T lg[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) lg[c] = (T)a.beta * a.lam_p[c * P + p];
  const double hiu = (double)M + 1.0;
  const bool in = u[0] >= -1.0 && u[0] < hiu && u[1] >= -1.0 && u[1] < hiu && u[2] >= -1.0 &&
                  u[2] < hiu;
  int j0[3] = {0, 0, 0};
  T f[3] = {T(0), T(0), T(0)};
  int lo[3], hi[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (in) {
      const double fl = floor(u[c]);
      j0[c] = (int)fl;
      f[c] = (T)(u[c] - fl);
    }
    lo[c] = max(j0[c] - 1, -1);
    hi[c] = min(j0[c] + 2, M + 1);
  }
  // stage the potential of the block's stencils in LDS (global fallback)
  __shared__ T win[kWindow];
  __shared__ int bounds[6];
  block_bounds(in, lo, hi, bounds);
  const int lx = bounds[0], ly = bounds[1], lz = bounds[2];
  const int wx = bounds[3] - lx + 1, wy = bounds[4] - ly + 1, wz = bounds[5] - lz + 1;
  const bool empty = wx <= 0 || wy <= 0 || wz <= 0;
  const int vol = empty ? 0 : wx * wy * wz;
  const bool use_lds = !empty && vol <= kWindow;
  const T* phi = a.phi + t.h_off;
  if (use_lds) {
    const int wyz = wy * wz;
    const float inv_wz = 1.0f / (float)wz, inv_wyz = 1.0f / (float)wyz;
#pragma unroll 4
    for (int e = threadIdx.x; e < vol; e += blockDim.x) {
      int ex, ey, ez;
      window_coords(e, wz, wyz, inv_wz, inv_wyz, ex, ey, ez);
      win[e] = phi[((int64_t)(lx + ex + 1) * Mp + (ly + ey + 1)) * Mp + (lz + ez + 1)];
    }
  }
  __syncthreads();
  T lu[3] = {T(0), T(0), T(0)};
  if (in) {
    auto at = [&](int x, int y, int z) -> T {
      if (use_lds) return win[((x - lx) * wy + (y - ly)) * wz + (z - lz)];
      return phi[((int64_t)(x + 1) * Mp + (y + 1)) * Mp + (z + 1)];
    };
    const T* lr = a.lam_rho + t.g_off;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int d[3] = {(c >> 2) & 1, (c >> 1) & 1, c & 1};
      const int nx = j0[0] + d[0], ny = j0[1] + d[1], nz = j0[2] + d[2];
      if (nx < 0 || nx > M || ny < 0 || ny > M || nz < 0 || nz > M) continue;
      T wa[3], dw[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) wa[q] = d[q] ? f[q] : T(1) - f[q];
      dw[0] = (d[0] ? T(1) : T(-1)) * wa[1] * wa[2];
      dw[1] = (d[1] ? T(1) : T(-1)) * wa[0] * wa[2];
      dw[2] = (d[2] ? T(1) : T(-1)) * wa[0] * wa[1];
      const T gx = T(0.5) * (at(nx + 1, ny, nz) - at(nx - 1, ny, nz));
      const T gy = T(0.5) * (at(nx, ny + 1, nz) - at(nx, ny - 1, nz));
      const T gz = T(0.5) * (at(nx, ny, nz + 1) - at(nx, ny, nz - 1));
      T s = lg[0] * gx + lg[1] * gy + lg[2] * gz;
      if (nx >= 1 && nx <= n && ny >= 1 && ny <= n && nz >= 1 && nz <= n)
        s += lr[((int64_t)(nx - 1) * n + (ny - 1)) * n + (nz - 1)];
#pragma unroll
      for (int q = 0; q < 3; ++q) lu[q] += dw[q] * s;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    a.lam_x[c * P + p] += lu[c];
    a.lam_psi1[c * P + p] += -a.D1 * (double)lu[c];
    a.lam_psi2[c * P + p] += a.D2 * (double)lu[c];
  }
  // clear this block's share of the box's lam_G (read by no kernel after pass A)
  const int nblk = (M * M * M) / kBlock;
  const int64_t len = (int64_t)Mp * Mp * Mp;
  const int64_t chunk = (len + nblk - 1) / nblk;
  const int64_t e0 = (int64_t)m.local[b] * chunk;
  for (int comp = 0; comp < 3; ++comp) {
    T* g = a.lam_G + comp * a.H + t.h_off;
    for (int64_t e = e0 + threadIdx.x; e < e0 + chunk && e < len; e += blockDim.x) g[e] = T(0);
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
    double s1[3], s2[3], u[3];
    particle_position(a, p, i, j, k, s1, s2, u);
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
    a.lam_psi1[c * P + p] = -a.D1 * (double)lu[c];
    a.lam_psi2[c * P + p] = a.D2 * (double)lu[c];
  }
}

// ---- set-up adjoint (FP64) -----------------------------------------------------------------

// Box particles -> global lattice sites: lam_Psi_global += lam_Psi (boxes overlap in their
// buffers, hence the atomics).
__global__ void __launch_bounds__(kBlock) k_adj_psi_scatter(const TileDesc* __restrict__ tiles,
                                                            const int* __restrict__ blk_tile,
                                                            const int* __restrict__ blk_first,
                                                            const double* __restrict__ lp1,
                                                            const double* __restrict__ lp2,
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
    const double v1 = lp1[c * P + p], v2 = lp2[c * P + p];
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
hipError_t launch_adj_step(const AdjointArgs<T>& a, const BlockMap& part, int stage, T* work,
                           double* lam_bc0, int n_tiles, hipStream_t s) {
  switch (stage) {
    case 0:
      if (part.count > 0)
        hipLaunchKernelGGL(k_adj_scatter<T>, dim3(padded_grid(part)), dim3(kBlock), 0, s, a, part);
      break;
    case 1:
      hipLaunchKernelGGL(k_adj_divergence<T>, dim3(64, n_tiles), dim3(kBlock), 0, s, a, work,
                         lam_bc0, n_tiles);
      break;
    case 2:
      if (part.count > 0)
        hipLaunchKernelGGL(k_adj_gather<T>, dim3(padded_grid(part)), dim3(kBlock), 0, s, a, part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_adj_setup_scatter(const BoxSetupArgs& b, const double* lam_psi1,
                                    const double* lam_psi2, double* lam_psig,
                                    const double* lam_bc0, double* lam_phi1, hipStream_t s) {
  if (b.n_blocks > 0)
    hipLaunchKernelGGL(k_adj_psi_scatter, dim3(b.n_blocks), dim3(kBlock), 0, s, b.tiles,
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
template hipError_t launch_adj_step<float>(const AdjointArgs<float>&, const BlockMap&, int,
                                           float*, double*, int, hipStream_t);
template hipError_t launch_adj_step<double>(const AdjointArgs<double>&, const BlockMap&, int,
                                            double*, double*, int, hipStream_t);

}  // namespace scola
