// FP64 set-up kernels: Gaussian initial conditions, Lagrangian potentials phi1 / phi2 on
// the periodic LPT grid, per-box Psi1 / Psi2 and the LEP boundary potential Phi_BC^0.
//
// Paper: Sec. 3.1 (A.1 convolution approach; A.2 Poisson-like equations LPTpotential1/2,
// second-order source by nine 1-D gradient operations), Sec. 3.3 (C.1-C.3: exact Psi in
// the box, Phi_BCs interpolated from the LPT grid to the PM grid), Sec. 3 (finite
// differences of order 2, 4 or 6: ng = 1, 2, 3 neighbours per side; Sec. 4 runs order 2).
#include "common.h"
#include "kernels.h"

namespace scola {

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int wrap(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Batched complex FFT (FP64, power-of-two length n) along one axis of an n^3 array held as
// [outer][n][inner].  Each block transforms `lines` lines staged in LDS with a radix-2
// Stockham pass per stage.  sign = -1 forward, +1 inverse (unnormalised).
__global__ void __launch_bounds__(kBlock) k_fft_axis(double2* __restrict__ data, int n,
                                                      int log2n, int64_t inner, int lines,
                                                      double sign) {
  extern __shared__ double2 lds[];
  double2* buf0 = lds;
  double2* buf1 = lds + (size_t)lines * n;
  const int64_t total_lines = (int64_t)n * n;       // n^3 / n
  const int64_t first = (int64_t)blockIdx.x * lines;
  const int tid = threadIdx.x;
  const int count = lines * n;
  // element e of the block -> (line b, position i) with coalesced global addresses
  auto address = [&](int e, int& b, int& i) -> int64_t {
    if (inner == 1) {
      b = e / n;
      i = e % n;
      return (first + b) * n + i;
    }
    b = e % lines;
    i = e / lines;
    const int64_t line = first + b;
    const int64_t o = line / inner, c = line % inner;
    return o * n * inner + (int64_t)i * inner + c;
  };
  for (int e = tid; e < count; e += blockDim.x) {
    int b, i;
    const int64_t a = address(e, b, i);
    if (first + b < total_lines) buf0[b * n + i] = data[a];
  }
  __syncthreads();
  double2* src = buf0;
  double2* dst = buf1;
  const int half = n / 2;
  for (int ns = 1; ns < n; ns <<= 1) {
    for (int e = tid; e < lines * half; e += blockDim.x) {
      const int b = e / half, j = e % half;
      const int k = j & (ns - 1);
      double s, c;
      sincospi(sign * (double)k / (double)ns, &s, &c);
      const double2 x0 = src[b * n + j];
      const double2 x1 = cmul(src[b * n + j + half], make_double2(c, s));
      const int o = b * n + ((j - k) << 1) + k;
      dst[o] = make_double2(x0.x + x1.x, x0.y + x1.y);
      dst[o + ns] = make_double2(x0.x - x1.x, x0.y - x1.y);
    }
    __syncthreads();
    double2* t = src;
    src = dst;
    dst = t;
  }
  for (int e = tid; e < count; e += blockDim.x) {
    int b, i;
    const int64_t a = address(e, b, i);
    if (first + b < total_lines) data[a] = src[b * n + i];
  }
}

__global__ void k_real_to_complex(const double* __restrict__ in, double2* __restrict__ out,
                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_double2(in[i], 0.0);
}

__global__ void k_take_real(const double2* __restrict__ in, double* __restrict__ out,
                            double scale, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i].x * scale;
}

// Central-difference weights of order 2 ng: first derivative sum_k c_k (f(i+k) - f(i-k)),
// c = (1/2), (2/3, -1/12), (3/4, -3/20, 1/60); second derivative
// sum_k a_k (f(i+k) + f(i-k) - 2 f(i)), a = (1), (4/3, -1/12), (3/2, -3/20, 1/90).
__device__ inline double d1_weight(int ng, int k) {
  return ng == 1 ? 0.5
       : ng == 2 ? (k == 1 ? 2.0 / 3.0 : -1.0 / 12.0)
                 : (k == 1 ? 0.75 : k == 2 ? -0.15 : 1.0 / 60.0);
}
__device__ inline double d2_weight(int ng, int k) {
  return ng == 1 ? 1.0
       : ng == 2 ? (k == 1 ? 4.0 / 3.0 : -1.0 / 12.0)
                 : (k == 1 ? 1.5 : k == 2 ? -0.15 : 1.0 / 90.0);
}

// Fourier symbol of the FDA Laplacian of order 2 ng, one-cell spacing: per axis
// sum_k a_k (2 cos(2 pi k m / N) - 2), i.e. -4 sin^2(pi m / N) at order 2.
__device__ inline double fda_symbol(int mx, int my, int mz, int N, int ng) {
  if (ng == 1) {
    double sx = sinpi((double)mx / N), sy = sinpi((double)my / N), sz = sinpi((double)mz / N);
    return -4.0 * (sx * sx + sy * sy + sz * sz);
  }
  double s = 0.0;
  for (int k = 1; k <= ng; ++k)
    s += d2_weight(ng, k) * (2.0 * (cospi(2.0 * k * mx / N) + cospi(2.0 * k * my / N) +
                                    cospi(2.0 * k * mz / N)) - 6.0);
  return s;
}

__device__ inline int signed_mode(int i, int N) { return i < N / 2 ? i : i - N; }

// A.1 + A.2 (first order): multiply FFT(w) by sqrt(P(k, a_i) N^3 / L^3) and divide by the
// FDA Laplacian symbol; the zero mode is set to zero.
__global__ void k_ic_filter(double2* __restrict__ c, int N, double L, double amplitude,
                            double ns, double Om, double Ob, double h, double Tcmb,
                            double growth2, int ng) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n3 = (int64_t)N * N * N;
  if (i >= n3) return;
  const int ix = (int)(i / ((int64_t)N * N)), iy = (int)((i / N) % N), iz = (int)(i % N);
  const int mx = signed_mode(ix, N), my = signed_mode(iy, N), mz = signed_mode(iz, N);
  if (mx == 0 && my == 0 && mz == 0) {
    c[i] = make_double2(0.0, 0.0);
    return;
  }
  const double kf = 2.0 * M_PI / L;
  const double k = kf * sqrt((double)mx * mx + (double)my * my + (double)mz * mz);
  const double T = eh_nowiggle_transfer(k, Om, Ob, h, Tcmb);
  const double P = amplitude * pow(k, ns) * T * T * growth2;
  const double f = sqrt(P * (double)N * N * N / (L * L * L)) / fda_symbol(mx, my, mz, N, ng);
  c[i] = make_double2(c[i].x * f, c[i].y * f);
}

// Division by the FDA Laplacian symbol (A.2, second order), zero mode to zero.
__global__ void k_inverse_laplacian(double2* __restrict__ c, int N, int ng) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n3 = (int64_t)N * N * N;
  if (i >= n3) return;
  const int ix = (int)(i / ((int64_t)N * N)), iy = (int)((i / N) % N), iz = (int)(i % N);
  const int mx = signed_mode(ix, N), my = signed_mode(iy, N), mz = signed_mode(iz, N);
  if (mx == 0 && my == 0 && mz == 0) {
    c[i] = make_double2(0.0, 0.0);
    return;
  }
  const double inv = 1.0 / fda_symbol(mx, my, mz, N, ng);
  c[i] = make_double2(c[i].x * inv, c[i].y * inv);
}

// Second-order source sum_{i>j} [phi_,ii phi_,jj - phi_,ij^2] with phi_,ij = D_i D_j phi,
// D the central difference of order 2 ng (wide stencils), periodic; written as complex
// input of the next FFT.
__global__ void k_second_order_source(const double* __restrict__ phi, double2* __restrict__ out,
                                      int N, int ng) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n3 = (int64_t)N * N * N;
  if (i >= n3) return;
  const int x = (int)(i / ((int64_t)N * N)), y = (int)((i / N) % N), z = (int)(i % N);
  auto P = [&](int dx, int dy, int dz) {
    return phi[((int64_t)wrap(x + dx, N) * N + wrap(y + dy, N)) * N + wrap(z + dz, N)];
  };
  if (ng > 1) {
    // D_i (D_j phi) = sum_k c_k sum_l c_l [phi(+k e_i + l e_j) - phi(+k e_i - l e_j)
    //                                      - phi(-k e_i + l e_j) + phi(-k e_i - l e_j)]
    double d[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = a; b < 3; ++b) {
        double acc = 0.0;
        for (int k = 1; k <= ng; ++k)
          for (int l = 1; l <= ng; ++l) {
            double t = 0.0;
            for (int sk = -1; sk <= 1; sk += 2)
              for (int sl = -1; sl <= 1; sl += 2) {
                int o[3] = {0, 0, 0};
                o[a] += sk * k;
                o[b] += sl * l;
                t += sk * sl * P(o[0], o[1], o[2]);
              }
            acc += d1_weight(ng, k) * d1_weight(ng, l) * t;
          }
        d[a][b] = d[b][a] = acc;
      }
    const double s = d[1][1] * d[0][0] - d[0][1] * d[0][1] + d[2][2] * d[0][0] -
                     d[0][2] * d[0][2] + d[2][2] * d[1][1] - d[1][2] * d[1][2];
    out[i] = make_double2(s, 0.0);
    return;
  }
  const double c0 = P(0, 0, 0);
  const double xx = 0.25 * (P(2, 0, 0) - 2.0 * c0 + P(-2, 0, 0));
  const double yy = 0.25 * (P(0, 2, 0) - 2.0 * c0 + P(0, -2, 0));
  const double zz = 0.25 * (P(0, 0, 2) - 2.0 * c0 + P(0, 0, -2));
  const double xy = 0.25 * (P(1, 1, 0) - P(1, -1, 0) - P(-1, 1, 0) + P(-1, -1, 0));
  const double xz = 0.25 * (P(1, 0, 1) - P(1, 0, -1) - P(-1, 0, 1) + P(-1, 0, -1));
  const double yz = 0.25 * (P(0, 1, 1) - P(0, 1, -1) - P(0, -1, 1) + P(0, -1, -1));
  const double s = yy * xx - xy * xy + zz * xx - xz * xz + zz * yy - yz * yz;
  out[i] = make_double2(s, 0.0);
}

// C.1-C.2: Psi1 = D phi1 and Psi2 = D phi2 at every box particle; also the operator L-
// (x_res = p_res = 0).  With an LPT grid of N = Np nodes per side the nodes coincide with
// the particles (no interpolation); with N < Np (Np / N an integer) the node m sits at the
// centre (m + 1/2) Np / N of its cell, the gradient is taken at the 8 nodes around the
// particle's LPT coordinate u = (g + 1/2) N / Np - 1/2 and interpolated by CiC, then
// converted from LPT-grid cells to lattice cells (x Np / N).
template <typename T>
__global__ void k_extract_psi(const TileDesc* __restrict__ tiles,
                              const int* __restrict__ blk_tile, const int* __restrict__ blk_first,
                              const double* __restrict__ phi1, const double* __restrict__ phi2,
                              T* __restrict__ psi1, T* __restrict__ psi2,
                              T* __restrict__ xres, T* __restrict__ pres, int N, int64_t P,
                              int ng, int Np) {
  const TileDesc t = tiles[blk_tile[blockIdx.x]];
  const int64_t pl = (int64_t)blk_first[blockIdx.x] * kBlock + threadIdx.x;
  const int M = t.M;
  const int64_t M3 = (int64_t)M * M * M;
  if (pl >= M3) return;
  int i, j, k;
  brick_site(pl, M, i, j, k);
  auto at = [&](const double* f, int x, int y, int z) {
    return f[((int64_t)wrap(x, N) * N + wrap(y, N)) * N + wrap(z, N)];
  };
  const int64_t p = t.p_off + pl;
  if (N != Np) {
    const int g[3] = {wrap(t.origin[0] + i, Np), wrap(t.origin[1] + j, Np),
                      wrap(t.origin[2] + k, Np)};
    const double r = (double)N / (double)Np;
    int m0[3];
    double w[3][2];
    for (int c = 0; c < 3; ++c) {
      const double u = ((double)g[c] + 0.5) * r - 0.5;
      const double fl = floor(u);
      m0[c] = (int)fl;
      w[c][1] = u - fl;
      w[c][0] = 1.0 - w[c][1];
    }
    double s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
    for (int cn = 0; cn < 8; ++cn) {
      const int dx = (cn >> 2) & 1, dy = (cn >> 1) & 1, dz = cn & 1;
      const double wc = w[0][dx] * w[1][dy] * w[2][dz];
      const int x = m0[0] + dx, y = m0[1] + dy, z = m0[2] + dz;
      for (int kk = 1; kk <= ng; ++kk) {
        const double c = wc * d1_weight(ng, kk);
        s1[0] += c * (at(phi1, x + kk, y, z) - at(phi1, x - kk, y, z));
        s1[1] += c * (at(phi1, x, y + kk, z) - at(phi1, x, y - kk, z));
        s1[2] += c * (at(phi1, x, y, z + kk) - at(phi1, x, y, z - kk));
        s2[0] += c * (at(phi2, x + kk, y, z) - at(phi2, x - kk, y, z));
        s2[1] += c * (at(phi2, x, y + kk, z) - at(phi2, x, y - kk, z));
        s2[2] += c * (at(phi2, x, y, z + kk) - at(phi2, x, y, z - kk));
      }
    }
    const double scale = (double)Np / (double)N;
    for (int c = 0; c < 3; ++c) {
      psi1[c * P + p] = (T)(scale * s1[c]);
      psi2[c * P + p] = (T)(scale * s2[c]);
      xres[c * P + p] = T(0);
      pres[c * P + p] = T(0);
    }
    return;
  }
  const int gx = wrap(t.origin[0] + i, N), gy = wrap(t.origin[1] + j, N),
            gz = wrap(t.origin[2] + k, N);
  // differenced in FP64, stored in the plan precision (FP32 plans keep the paper's
  // single-precision particle record)
  if (ng == 1) {
    psi1[p] = (T)(0.5 * (at(phi1, gx + 1, gy, gz) - at(phi1, gx - 1, gy, gz)));
    psi1[P + p] = (T)(0.5 * (at(phi1, gx, gy + 1, gz) - at(phi1, gx, gy - 1, gz)));
    psi1[2 * P + p] = (T)(0.5 * (at(phi1, gx, gy, gz + 1) - at(phi1, gx, gy, gz - 1)));
    psi2[p] = (T)(0.5 * (at(phi2, gx + 1, gy, gz) - at(phi2, gx - 1, gy, gz)));
    psi2[P + p] = (T)(0.5 * (at(phi2, gx, gy + 1, gz) - at(phi2, gx, gy - 1, gz)));
    psi2[2 * P + p] = (T)(0.5 * (at(phi2, gx, gy, gz + 1) - at(phi2, gx, gy, gz - 1)));
  } else {
    double s1[3] = {0.0, 0.0, 0.0}, s2[3] = {0.0, 0.0, 0.0};
    for (int k = 1; k <= ng; ++k) {
      const double c = d1_weight(ng, k);
      s1[0] += c * (at(phi1, gx + k, gy, gz) - at(phi1, gx - k, gy, gz));
      s1[1] += c * (at(phi1, gx, gy + k, gz) - at(phi1, gx, gy - k, gz));
      s1[2] += c * (at(phi1, gx, gy, gz + k) - at(phi1, gx, gy, gz - k));
      s2[0] += c * (at(phi2, gx + k, gy, gz) - at(phi2, gx - k, gy, gz));
      s2[1] += c * (at(phi2, gx, gy + k, gz) - at(phi2, gx, gy - k, gz));
      s2[2] += c * (at(phi2, gx, gy, gz + k) - at(phi2, gx, gy, gz - k));
    }
    for (int c = 0; c < 3; ++c) {
      psi1[c * P + p] = (T)s1[c];
      psi2[c * P + p] = (T)s2[c];
    }
  }
  for (int c = 0; c < 3; ++c) {
    xres[c * P + p] = T(0);
    pres[c * P + p] = T(0);
  }
}

// C.3: Phi_BC^0 at the padded PM nodes j in [-ng, M+ng]^3 outside [1, M-1]^3: trilinear
// interpolation of phi1 at the PM node, i.e. with N = Np the mean of the 8 LPT nodes around
// it (PM nodes sit half a cell from the LPT nodes).  Interior entries are set to zero.
__global__ void k_boundary_potential(const TileDesc* __restrict__ tiles, int n_tiles,
                                     const double* __restrict__ phi1, double* __restrict__ bc0,
                                     int N, int ng, int Np) {
  const int ti = blockIdx.y;
  if (ti >= n_tiles) return;
  const TileDesc t = tiles[ti];
  const int Mp = t.M + 1 + 2 * ng;
  const int64_t n = (int64_t)Mp * Mp * Mp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e / ((int64_t)Mp * Mp)) - ng, b = (int)((e / Mp) % Mp) - ng,
              c = (int)(e % Mp) - ng;
    double v = 0.0;
    const bool inside = a >= 1 && a <= t.M - 1 && b >= 1 && b <= t.M - 1 && c >= 1 &&
                        c <= t.M - 1;
    if (!inside && N != Np) {
      // LPT grid coarser than the lattice: CiC at the node's LPT coordinate X N / Np - 1/2,
      // converted from LPT-grid cells^2 to lattice cells^2
      const double r = (double)N / (double)Np;
      const int X[3] = {t.origin[0] + a, t.origin[1] + b, t.origin[2] + c};
      int m0[3];
      double w[3][2];
      for (int d = 0; d < 3; ++d) {
        const double u = (double)X[d] * r - 0.5;
        const double fl = floor(u);
        m0[d] = (int)fl;
        w[d][1] = u - fl;
        w[d][0] = 1.0 - w[d][1];
      }
      for (int cn = 0; cn < 8; ++cn) {
        const int dx = (cn >> 2) & 1, dy = (cn >> 1) & 1, dz = cn & 1;
        v += w[0][dx] * w[1][dy] * w[2][dz] *
             phi1[((int64_t)wrap(m0[0] + dx, N) * N + wrap(m0[1] + dy, N)) * N +
                  wrap(m0[2] + dz, N)];
      }
      v *= ((double)Np / (double)N) * ((double)Np / (double)N);
    } else if (!inside) {
      const int gx = t.origin[0] + a, gy = t.origin[1] + b, gz = t.origin[2] + c;
      for (int dx = -1; dx <= 0; ++dx)
        for (int dy = -1; dy <= 0; ++dy)
          for (int dz = -1; dz <= 0; ++dz)
            v += phi1[((int64_t)wrap(gx + dx, N) * N + wrap(gy + dy, N)) * N +
                      wrap(gz + dz, N)];
      v *= 0.125;
    }
    bc0[t.h_off + e] = v;
  }
}

inline unsigned grid1(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

hipError_t fft3d(double2* c, int N, double sign, hipStream_t s) {
  int log2n = 0;
  while ((1 << log2n) < N) ++log2n;
  const int lines = N >= 1024 ? 1 : 1024 / N;     // 32 KiB of LDS per block
  const size_t lds = (size_t)2 * lines * N * sizeof(double2);
  const int64_t total_lines = (int64_t)N * N;
  const unsigned blocks = (unsigned)((total_lines + lines - 1) / lines);
  const int64_t inners[3] = {(int64_t)N * N, N, 1};   // axes x, y, z
  for (int ax = 0; ax < 3; ++ax) {
    hipLaunchKernelGGL(k_fft_axis, dim3(blocks), dim3(kBlock), lds, s, c, N, log2n,
                       inners[ax], lines, sign);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t fft3d_forward(double2* c, int N, hipStream_t s) { return fft3d(c, N, -1.0, s); }
hipError_t fft3d_inverse(double2* c, int N, hipStream_t s) { return fft3d(c, N, +1.0, s); }

hipError_t launch_ic_filter(const SetupArgs& a, hipStream_t s) {
  const int64_t n3 = (int64_t)a.N * a.N * a.N;
  hipLaunchKernelGGL(k_ic_filter, dim3(grid1(n3)), dim3(kBlock), 0, s, a.cbuf, a.N, a.L,
                     a.amplitude, a.ns, a.Om, a.Ob, a.h, a.Tcmb, a.growth2, a.ng);
  return hipGetLastError();
}

hipError_t launch_inverse_laplacian(double2* c, int N, int ng, hipStream_t s) {
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_inverse_laplacian, dim3(grid1(n3)), dim3(kBlock), 0, s, c, N, ng);
  return hipGetLastError();
}

hipError_t launch_take_real(const double2* c, double* out, double scale, int64_t n,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_take_real, dim3(grid1(n)), dim3(kBlock), 0, s, c, out, scale, n);
  return hipGetLastError();
}

hipError_t launch_setup_potentials(const SetupArgs& a, hipStream_t s) {
  const int N = a.N;
  const int64_t n3 = (int64_t)N * N * N;
  hipLaunchKernelGGL(k_real_to_complex, dim3(grid1(n3)), dim3(kBlock), 0, s, a.white_noise,
                     a.cbuf, n3);
  hipError_t e = fft3d(a.cbuf, N, -1.0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ic_filter, dim3(grid1(n3)), dim3(kBlock), 0, s, a.cbuf, N, a.L,
                     a.amplitude, a.ns, a.Om, a.Ob, a.h, a.Tcmb, a.growth2, a.ng);
  if ((e = fft3d(a.cbuf, N, +1.0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_take_real, dim3(grid1(n3)), dim3(kBlock), 0, s, a.cbuf, a.phi1,
                     1.0 / (double)n3, n3);
  hipLaunchKernelGGL(k_second_order_source, dim3(grid1(n3)), dim3(kBlock), 0, s, a.phi1,
                     a.cbuf, N, a.ng);
  if ((e = fft3d(a.cbuf, N, -1.0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_inverse_laplacian, dim3(grid1(n3)), dim3(kBlock), 0, s, a.cbuf, N, a.ng);
  if ((e = fft3d(a.cbuf, N, +1.0, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_take_real, dim3(grid1(n3)), dim3(kBlock), 0, s, a.cbuf, a.phi2,
                     1.0 / (double)n3, n3);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_setup_boxes(const BoxSetupArgs& a, T* xres, T* pres, hipStream_t s) {
  if (a.n_blocks > 0)
    hipLaunchKernelGGL(k_extract_psi<T>, dim3(a.n_blocks), dim3(kBlock), 0, s, a.tiles,
                       a.blk_tile, a.blk_first, a.phi1, a.phi2, static_cast<T*>(a.psi1),
                       static_cast<T*>(a.psi2), xres, pres,
                       a.N, a.P, a.ng, a.Np);
  hipLaunchKernelGGL(k_boundary_potential, dim3(64, a.n_tiles), dim3(kBlock), 0, s, a.tiles,
                     a.n_tiles, a.phi1, a.bc0, a.N, a.ng, a.Np);
  return hipGetLastError();
}

template hipError_t launch_setup_boxes<float>(const BoxSetupArgs&, float*, float*, hipStream_t);
template hipError_t launch_setup_boxes<double>(const BoxSetupArgs&, double*, double*,
                                               hipStream_t);

}  // namespace scola
