// Device code of the Dirichlet Poisson solve by DST-I (App. C): for FP64 plans the
// in-register and cross-lane FFTs and the half-length sine transform of two lines; for FP32
// plans the matrix-core products of dst_mfma.h; and the three passes as device functions of
// one logical block (see kernels_poisson.hip for the pass structure).
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"
#include "dst_mfma.h"

namespace scola {

namespace {


template <typename T>
using cx = typename std::conditional<std::is_same<T, float>::value, float2, double2>::type;

template <typename C>
__device__ inline C c_add(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ inline C c_sub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename C>
__device__ inline C c_mul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}

// 1 / d: the hardware reciprocal (1 ulp) in FP32 plans, a correctly rounded division in FP64
__device__ __forceinline__ float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double recip(double d) { return 1.0 / d; }

__device__ inline int bitrev5(int l) { return (int)(__brev((unsigned)l) >> 27); }

// exp(-2 pi i m / R) for R = 1..8 (row R - 1), m < R: the in-register DFT multiplies by
// these compile-time constants, so the trivial ones (1, -1, +-i) cost no arithmetic.
constexpr double kDftW[8][8][2] = {
    {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {-1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {-0.5, -0.8660254037844386}, {-0.5, 0.8660254037844386}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {0.0, -1.0}, {-1.0, 0.0}, {0.0, 1.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {0.30901699437494745, -0.9510565162951535}, {-0.8090169943749473, -0.5877852522924732}, {-0.8090169943749473, 0.5877852522924732}, {0.30901699437494745, 0.9510565162951535}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {0.5, -0.8660254037844386}, {-0.5, -0.8660254037844386}, {-1.0, 0.0}, {-0.5, 0.8660254037844386}, {0.5, 0.8660254037844386}, {0.0, 0.0}, {0.0, 0.0}},
    {{1.0, 0.0}, {0.6234898018587336, -0.7818314824680298}, {-0.22252093395631434, -0.9749279121818236}, {-0.900968867902419, -0.43388373911755823}, {-0.900968867902419, 0.43388373911755823}, {-0.22252093395631434, 0.9749279121818236}, {0.6234898018587336, 0.7818314824680298}, {0.0, 0.0}},
    {{1.0, 0.0}, {0.7071067811865476, -0.7071067811865476}, {0.0, -1.0}, {-0.7071067811865476, -0.7071067811865476}, {-1.0, 0.0}, {-0.7071067811865476, 0.7071067811865476}, {0.0, 1.0}, {0.7071067811865476, 0.7071067811865476}},
};

// a * W_R^m with W_R^m = exp(-2 pi i m / R); R and m are compile-time constants after
// unrolling, and the branches on the table entries fold away.
template <typename T>
__device__ __forceinline__ cx<T> mul_wr(cx<T> a, int R, int m) {
  const double c = kDftW[R - 1][m][0], s = kDftW[R - 1][m][1];
  cx<T> r;
  if (c == 1.0 && s == 0.0) return a;
  if (c == -1.0 && s == 0.0) {
    r.x = -a.x;
    r.y = -a.y;
  } else if (c == 0.0 && s == -1.0) {
    r.x = a.y;
    r.y = -a.x;
  } else if (c == 0.0 && s == 1.0) {
    r.x = -a.y;
    r.y = a.x;
  } else {
    r.x = a.x * (T)c - a.y * (T)s;
    r.y = a.x * (T)s + a.y * (T)c;
  }
  return r;
}

// Lane l of a quarter wavefront holds data index n(l) of the 16-point transforms across
// lanes.  The lane bits are a GF(2)-linear relabelling of the data bits chosen so that the
// partner of every radix-2 stage is a single DPP move away: data bit 0 -> lane xor 1, bit 1
// -> xor 2 (quad permutations), bit 2 -> xor 7 (half-row mirror), bit 3 -> xor 15 (row
// mirror).  n(0) = 0.  stage_partner also offers bit 4 -> xor 16 (ds_swizzle across two
// 16-lane rows) for transforms over 32 lanes, which the solver does not use.
__device__ __forceinline__ int fft_index(int l) {
  const int l0 = l & 1, l1 = (l >> 1) & 1, l2 = (l >> 2) & 1, l3 = (l >> 3) & 1;
  return (l0 ^ l2) | ((l1 ^ l2) << 1) | ((l2 ^ l3) << 2) | (l & 0x18);
}

template <int B>
__device__ __forceinline__ int stage_partner(int v) {
  static_assert(B >= 0 && B <= 4, "data bit");
  if constexpr (B == 0) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // xor 1
  if constexpr (B == 1) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // xor 2
  if constexpr (B == 2) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // xor 7
  if constexpr (B == 3) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true);  // xor 15
  if constexpr (B == 4) return __builtin_amdgcn_ds_swizzle(v, 0x401F);              // xor 16
  return v;
}
template <int B>
__device__ __forceinline__ float stage_partner(float v) {
  return __int_as_float(stage_partner<B>(__float_as_int(v)));
}
template <int B>
__device__ __forceinline__ double stage_partner(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = stage_partner<B>((int)(b & 0xffffffffll));
  const int hi = stage_partner<B>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One radix-2 decimation-in-frequency stage on data bit B (distance S = 2^B) of K x R
// independent 16-point transforms across lanes, without divergent branches: every lane
// forms v = own + s * partner with s = +1 where its data bit B is clear and -1 where it is
// set, i.e. a + b on the lower and -(a - b) on the upper element of each pair; the upper
// element's twiddle is taken negated, -W_{2S}^(n mod S) = W_{32R}^(((n mod S) 16/S + 16) R),
// which restores (a - b) W_{2S}^(n mod S).  The last stage (S = 1) has no twiddle and leaves
// the upper elements (odd n) negated; the caller undoes that sign where it reads them.
template <int B, int R, int K, typename T>
__device__ __forceinline__ void dif_stage(cx<T> (&x)[K][R], const cx<T>* __restrict__ tw,
                                          int n) {
  constexpr int S = 1 << B;
  const bool upper = ((n >> B) & 1) != 0;
  const T s = upper ? T(-1) : T(1);
  cx<T> w;
  if constexpr (S > 1) w = tw[upper ? ((n & (S - 1)) * (16 / S) + 16) * R : 0];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      cx<T> v;
      v.x = fma(stage_partner<B>(x[k][k1].x), s, x[k][k1].x);
      v.y = fma(stage_partner<B>(x[k][k1].y), s, x[k][k1].y);
      if constexpr (S > 1) {
        x[k][k1].x = v.x * w.x - v.y * w.y;
        x[k][k1].y = v.x * w.y + v.y * w.x;
      } else {
        x[k][k1] = v;
      }
    }
}

// In-register DFT of odd length R (forward): inputs n and R - n enter through their sum a_n
// and difference b_n, because W^(n k) and W^((R - n) k) are complex conjugates; with
// W^(n k) = c + i s, y_k = p_k + i q_k and y_(R-k) = p_k - i q_k for
// p_k = x_0 + sum_n c a_n, q_k = sum_n s b_n (n, k = 1 .. (R - 1) / 2).  About 4 H^2
// multiply-adds for H = (R - 1) / 2 instead of the direct sum's (R - 1)^2 complex products.
template <int R, typename T>
__device__ __forceinline__ void dft_odd(cx<T> (&x)[R]) {
  constexpr int H = (R - 1) / 2;
  cx<T> a[H + 1], b[H + 1];
  cx<T> y0 = x[0];
#pragma unroll
  for (int n = 1; n <= H; ++n) {
    a[n] = c_add(x[n], x[R - n]);
    b[n] = c_sub(x[n], x[R - n]);
    y0 = c_add(y0, a[n]);
  }
  cx<T> y[R];
  y[0] = y0;
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    cx<T> pk = x[0], qk;
    qk.x = T(0);
    qk.y = T(0);
#pragma unroll
    for (int n = 1; n <= H; ++n) {
      const int m = (n * k) % R;
      const T c = (T)kDftW[R - 1][m][0], sn = (T)kDftW[R - 1][m][1];
      pk.x = fma(c, a[n].x, pk.x);
      pk.y = fma(c, a[n].y, pk.y);
      qk.x = fma(sn, b[n].x, qk.x);
      qk.y = fma(sn, b[n].y, qk.y);
    }
    y[k].x = pk.x - qk.y;        // p + i q
    y[k].y = pk.y + qk.x;
    y[R - k].x = pk.x + qk.y;    // p - i q
    y[R - k].y = pk.y - qk.x;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) x[k] = y[k];
}

// In-register DFT of R points (forward, W_R = exp(-2 pi i / R)): radix-2 and radix-4
// butterflies for R = 2, 4, 8, the paired form for odd R, and R = 6 as two 3-point DFTs
// (even and odd inputs) joined by one twiddled radix-2 step.
template <int R, typename T>
__device__ __forceinline__ void small_dft(cx<T> (&x)[R]) {
  if constexpr (R == 2) {
    const cx<T> a = x[0], b = x[1];
    x[0] = c_add(a, b);
    x[1] = c_sub(a, b);
  } else if constexpr (R == 4) {
    const cx<T> t0 = c_add(x[0], x[2]), t1 = c_sub(x[0], x[2]);
    const cx<T> t2 = c_add(x[1], x[3]), t3 = c_sub(x[1], x[3]);
    x[0] = c_add(t0, t2);
    x[2] = c_sub(t0, t2);
    x[1].x = t1.x + t3.y;   // t1 - i t3
    x[1].y = t1.y - t3.x;
    x[3].x = t1.x - t3.y;   // t1 + i t3
    x[3].y = t1.y + t3.x;
  } else if constexpr (R == 8) {
    cx<T> e[4] = {x[0], x[2], x[4], x[6]}, o[4] = {x[1], x[3], x[5], x[7]};
    small_dft<4, T>(e);
    small_dft<4, T>(o);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const cx<T> t = mul_wr<T>(o[k], 8, k);
      x[k] = c_add(e[k], t);
      x[k + 4] = c_sub(e[k], t);
    }
  } else if constexpr (R == 6) {
    cx<T> e[3] = {x[0], x[2], x[4]}, o[3] = {x[1], x[3], x[5]};
    dft_odd<3, T>(e);
    dft_odd<3, T>(o);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const cx<T> t = mul_wr<T>(o[k], 6, k);
      x[k] = c_add(e[k], t);
      x[k + 3] = c_sub(e[k], t);
    }
  } else if constexpr (R % 2 == 1 && R > 1) {
    dft_odd<R, T>(x);
  } else {
    static_assert(R == 1, "in-register DFT lengths: 1 to 8");
  }
}

// K independent complex FFTs of length N = 16R on one quarter wavefront (16 lanes),
// interleaved for instruction-level parallelism.  Lane l holds x[k][n2] = input k at position
// 16 n2 + n with n = fft_index(l) (4 bits); on return it holds Z_k at position
// k1 + R bitrev4(n) in x[k][k1] (negated where n is odd).  The transform factors as an
// R-point DFT across registers, the twiddle W_N^(n k1), and a 16-point radix-2
// decimation-in-frequency FFT across lanes (every partner one DPP move away).
// tw = W_2N^m, m < 2N (in LDS): W_N^i = tw[2 i], and the stage twiddles W_2S^m are the
// same entries as for any N.
template <int R, int K, typename T>
__device__ __forceinline__ void quarter_fft(cx<T> (&x)[K][R], const cx<T>* __restrict__ tw,
                                            int n) {
  if constexpr (R > 1) {
    cx<T> tl[R];
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) tl[k1] = tw[2 * n * k1];    // W_N^(n k1)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      small_dft<R, T>(x[k]);
#pragma unroll
      for (int k1 = 1; k1 < R; ++k1) x[k][k1] = c_mul(x[k][k1], tl[k1]);
    }
  }
  dif_stage<3, R, K, T>(x, tw, n);
  dif_stage<2, R, K, T>(x, tw, n);
  dif_stage<1, R, K, T>(x, tw, n);
  dif_stage<0, R, K, T>(x, tw, n);
}

__device__ inline int bitrev4(int l) { return (int)(__brev((unsigned)l) >> 28); }

// v from the lane D places lower in the same 16-lane row (0 below the row's first lane).
template <int D>
__device__ __forceinline__ float row_shr(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + D, 0xF, 0xF,
                                                    true));
}
template <int D>
__device__ __forceinline__ double row_shr(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x110 + D, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x110 + D, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Inclusive prefix sum over the eight lanes t & 7 = 0..7 of each half of a 16-lane row.
template <typename T>
__device__ __forceinline__ T scan8(T v, int t) {
  const int g = t & 7;
  T s = row_shr<1>(v);
  v += g >= 1 ? s : T(0);
  s = row_shr<2>(v);
  v += g >= 2 ? s : T(0);
  s = row_shr<4>(v);
  v += g >= 4 ? s : T(0);
  return v;
}

// In-place DST-I (unnormalised, eq. DST_delta) of K pairs of lines (a_k, b_k), each
// n = N - 1 = 16R - 1 values y_1..y_n at the compile-time stride S in LDS, one pair per
// quarter wavefront; output j (1..n) of pair k is multiplied by sa(k, j) / sb(k, j).  Pairs
// with valid[k] false are not written and has_b[k] false means line b is absent; the
// pointers of absent lines must still point at readable LDS (their values are discarded).
//
// Method (the real-data sine transform through a half-length FFT of Cooley, Lewis and
// Welch, as used in FFTPACK's sint): with y_0 = y_N = 0 and s_j = sin(pi j / N), the
// sequence x_j = (s_j + 1/2) y_j + (s_j - 1/2) y_(N-j), j = 0..N-1, has the N-point DFT X
// with S_2k = -Im X_k and S_(2k+1) - S_(2k-1) = Re X_k (S_-1 = -S_1): x_j splits into a part
// symmetric under j -> N - j, which carries the odd sine sums, and an antisymmetric part,
// which carries the even ones.  Two lines share one complex FFT, z = x^a + i x^b, separated
// through X^a_k = (Z_k + conj Z_(N-k)) / 2 and X^b_k = (Z_k - conj Z_(N-k)) / 2i.  The
// odd outputs are a prefix sum of Re X_k over k = 0..N/2-1, taken as a running sum inside
// each lane followed by a scan over eight lanes.
//
// Steps: load and combine (lane base plus compile-time offsets), FFT, Z_k (k != N/2) written
// over the pair's own lines (real parts to line a, imaginary parts to line b, slot k for
// k < N/2 and k - 1 above; without line b the slots above N/2 take Im Z_(N-k), as Z is then
// Hermitian), read back in pairs (Z_k, Z_(N-k)) by lane t & 7 for k in [R (t & 7),
// R (t & 7) + R) of line a (t < 8) or line b (t >= 8), scan, outputs written.  A quarter
// wavefront reads only the lines it wrote, in program order, so no barrier is needed.
template <int R, int K, int S, typename T, typename SA, typename SB>
__device__ __forceinline__ void dst_quarter(T* const (&la)[K], T* const (&lb)[K],
                                            const bool (&valid)[K], const bool (&has_b)[K],
                                            const cx<T>* tw, int l, SA sa, SB sb) {
  constexpr int N = 16 * R, H = N / 2;
  const int n = fft_index(l);    // data index of this lane (l < 16)
  cx<T> x[K][R];
#pragma unroll
  for (int n2 = 0; n2 < R; ++n2) {
    const int j = 16 * n2 + n;
    const T sj = -tw[j].y;                                   // sin(pi j / N)
    const T cp = j > 0 ? sj + T(0.5) : T(0), cm = j > 0 ? sj - T(0.5) : T(0);
    // y_j at index j - 1 and y_(N-j) at N - j - 1 = 16 (R - 1 - n2) + 15 - n: one lane base
    // each plus compile-time offsets; j = 0 reads an in-line entry with zero weight
    const int lo = n2 == 0 ? max(n - 1, 0) : 16 * n2 + n - 1;
    const int hi = 16 * (R - 1 - n2) + 15 - n - (n2 == 0 && n == 0 ? 1 : 0);
    // the loads are unconditional (absent lines point at readable LDS) and their values
    // selected afterwards, so no branch precedes the FFT's hand-placed DPP blocks
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const T ya = la[k][lo * S], yna = la[k][hi * S];
      const T yb = lb[k][lo * S], ynb = lb[k][hi * S];
      cx<T> v;
      v.x = valid[k] ? cp * ya + cm * yna : T(0);
      v.y = valid[k] && has_b[k] ? cp * yb + cm * ynb : T(0);
      x[k][n2] = v;
    }
  }
  quarter_fft<R, K, T>(x, tw, n);
  // lane n holds Z at k1 + R bitrev4(n), negated where n is odd
  const int br = bitrev4(n);
  const T sgn = (n & 1) ? T(-1) : T(1);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!valid[k]) continue;
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const int kk = k1 + R * br;
      if (kk == H) continue;
      const int slot = kk < H ? kk : kk - 1;
      const T re = sgn * x[k][k1].x, im = sgn * x[k][k1].y;
      if (has_b[k]) {
        la[k][slot * S] = re;
        lb[k][slot * S] = im;
      } else {
        la[k][slot * S] = kk < H ? re : -im;
      }
    }
  }
  // read back (Z_k, Z_(N-k)) for this lane's k and form Re X_k and the even outputs; Re X_0
  // (Re Z_0 for line a, Im Z_0 for line b: Z_0 is its own partner) is read by every lane
  const int g = l & 7;
  const bool line_b = l >= 8;
  T rx[K][R], ev[K][R], half0[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    half0[k] = T(0);
    if (valid[k]) half0[k] = T(0.5) * ((line_b && has_b[k]) ? lb[k][0] : la[k][0]);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int kk = R * g + m;                          // 0 .. N/2 - 1
      const int sk = kk, sn = kk == 0 ? 0 : N - kk - 1;  // slots of Z_k and Z_(N-k)
      T rz = T(0), rzn = T(0), iz = T(0), izn = T(0);
      if (valid[k]) {
        rz = la[k][sk * S];
        if (has_b[k]) {
          rzn = la[k][sn * S];
          iz = lb[k][sk * S];
          izn = lb[k][sn * S];
        } else {
          rzn = rz;
          iz = kk == 0 ? T(0) : la[k][sn * S];
          izn = -iz;
        }
      }
      if (!line_b) {
        rx[k][m] = T(0.5) * (rz + rzn);
        ev[k][m] = T(0.5) * (izn - iz);
      } else {
        rx[k][m] = T(0.5) * (iz + izn);
        ev[k][m] = T(0.5) * (rz - rzn);
      }
    }
  }
  // S_(2k+1) = sum_(m <= k) Re X_m - Re X_0 / 2: running sums in the lane, then the scan over
  // the eight lanes of the line
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int m = 1; m < R; ++m) rx[k][m] += rx[k][m - 1];
    const T incl = scan8(rx[k][R - 1], l);
    const T offset = incl - rx[k][R - 1] - half0[k];
#pragma unroll
    for (int m = 0; m < R; ++m) rx[k][m] += offset;
  }
  // outputs: even j = 2k (k >= 1) at index 2k - 1, odd j = 2k + 1 at index 2k
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (!valid[k] || (line_b && !has_b[k])) continue;
    T* const out = line_b ? lb[k] : la[k];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int kk = R * g + m;
      if (kk >= 1)
        out[(2 * kk - 1) * S] = ev[k][m] * (line_b ? sb(k, 2 * kk) : sa(k, 2 * kk));
      out[2 * kk * S] = rx[k][m] * (line_b ? sb(k, 2 * kk + 1) : sa(k, 2 * kk + 1));
    }
  }
}

// Line pairs of a plane handled at once by one quarter wavefront (interleaved in registers):
// a plane direction has 8R pairs for 16 quarter wavefronts, R / 2 each; the count is chosen so
// that few register slots hold absent pairs while the registers stay below spilling.
template <int R>
struct PairBatch {
  static constexpr int K = R == 3 ? 2 : 1;
  static constexpr int rounds = (8 * R + 16 * K - 1) / (16 * K);
};

// DST-I of all lines of an n x n plane in LDS along one direction: lines at distance STEP,
// entries at stride S.  Pair p = (lines 2p, 2p + 1) goes to quarter wavefront p mod 16.
template <int R, int S, int STEP, typename T>
__device__ __forceinline__ void plane_lines(T* plane, const cx<T>* tw, int qw, int l) {
  constexpr int n = 16 * R - 1, pairs = 8 * R, K = PairBatch<R>::K;
  auto one = [](int, int) { return T(1); };
#pragma unroll
  for (int r = 0; r < PairBatch<R>::rounds; ++r) {
    T* la[K];
    T* lb[K];
    bool valid[K], hb[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int pr = qw + 16 * (r * K + k);
      valid[k] = pr < pairs;
      hb[k] = 2 * pr + 1 < n;
      la[k] = plane + (valid[k] ? 2 * pr : 0) * STEP;
      lb[k] = plane + (valid[k] && hb[k] ? 2 * pr + 1 : 0) * STEP;
    }
    T* const (&cla)[K] = la;
    T* const (&clb)[K] = lb;
    dst_quarter<R, K, S, T>(cla, clb, valid, hb, tw, l, one, one);
  }
}

// DST-I along z (rows, stride 1) then y (columns, stride n) of an n x n plane in LDS.
template <int R, typename T>
__device__ __forceinline__ void plane_dst(T* plane, const cx<T>* tw) {
  constexpr int n = 16 * R - 1;
  const int qw = threadIdx.x >> 4, l = threadIdx.x & 15;
  plane_lines<R, 1, n, T>(plane, tw, qw, l);
  __syncthreads();
  plane_lines<R, n, 1, T>(plane, tw, qw, l);
  __syncthreads();
}

// Fixed-point mass of a node in units: 64-bit words are read as signed (a total can only be
// non-negative, and the signed reading keeps a rounding below zero harmless), 32-bit words
// as unsigned (2^21 units per particle: up to 2048 particles per node).
__device__ __forceinline__ double mass_units(unsigned long long r) { return (double)(long long)r; }
__device__ __forceinline__ double mass_units(unsigned int r) { return (double)r; }

// Value of a full-box periodic field [N^3] at the box's local node (jx, jy, jz).
template <typename T>
__device__ __forceinline__ T full_at(const T* f, int N, const TileDesc& t, int jx, int jy,
                                     int jz) {
  const int m = N - 1;   // N is a power of two
  return f[((int64_t)((t.origin[0] + jx) & m) * N + ((t.origin[1] + jy) & m)) * N +
           ((t.origin[2] + jz) & m)];
}

template <typename T>
__device__ inline void load_twiddles(cx<T>* tw, const MeshArgs<T>& a, const TileDesc& t) {
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.twiddles) + t.tw_off;
  for (int i = threadIdx.x; i < 2 * t.M; i += blockDim.x) tw[i] = src[i];
}

// The three passes as device functions of one logical block L (< m.count) with the dynamic
// LDS `smem`: called by their own kernels below and by the persistent step kernel.
// Weights a_k (k = 1..NG) of the central second difference of order 2 NG, sum_k a_k (f(i+k)
// + f(i-k) - 2 f(i)): (1), (4/3, -1/12), (3/2, -3/20, 1/90).
template <int NG>
__device__ __forceinline__ constexpr double lap_weight(int k) {
  return NG == 1 ? 1.0
       : NG == 2 ? (k == 1 ? 4.0 / 3.0 : -1.0 / 12.0)
                 : (k == 1 ? 1.5 : k == 2 ? -0.15 : 1.0 / 90.0);
}

// What a pass's plane transform needs in registers: the wave's sine fragments for FP32
// plans (requested at the start of the pass), nothing for the FFT.
template <typename T, int R>
struct PlaneOperands {
  __device__ void load(const MeshArgs<T>&, const TileDesc&) {}
};
template <int R>
struct PlaneOperands<float, R> {
  SineFrag<R> s;
  __device__ void load(const MeshArgs<float>& a, const TileDesc& t) {
    s = load_sine<R>(reinterpret_cast<const _Float16*>(a.sine) + t.dm_off);
  }
};

// Element i < 4 (n - 1) of the perimeter of an n x n plane: the first row (y = 0), then the
// last column, the last row backwards and the first column backwards.
__device__ __forceinline__ void perimeter_yz(int i, int n, int& y, int& z) {
  const int side = i / (n - 1), o = i - side * (n - 1);
  y = side == 0 ? 0 : side == 1 ? o : side == 2 ? n - 1 : n - 1 - o;
  z = side == 0 ? o : side == 1 ? n - 1 : side == 2 ? n - 1 - o : 0;
}

// Inverse of perimeter_yz: the perimeter index of node (y, z) on the perimeter.
__device__ __forceinline__ int perimeter_index(int y, int z, int n) {
  if (y == 0) return z;
  if (z == n - 1) return (n - 1) + y;
  if (y == n - 1) return 2 * (n - 1) + (n - 1 - z);
  return 3 * (n - 1) + (n - 1 - y);
}

// Where a plane's perimeter terms wait in its consumed `work` plane (MeshArgs::bc_handoff):
// the plane's first 8-byte aligned address; 4 (n - 1) doubles fit in its n^2 values.
template <typename T>
__device__ __forceinline__ double* handoff_terms(T* plane) {
  return reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(plane) + 7) & ~uintptr_t(7));
}

// FP32 plans, first pass: the waves' sums of the plane's mass, in the LDS head behind the
// block-maximum slots of the transform (which use its first 2 kBlock / 64 floats).
__device__ __forceinline__ unsigned long long* found_slots(unsigned char* smem) {
  static_assert(kMfmaHead >= 32 + 8 * (kBlock / 64), "LDS head holds both slot sets");
  return reinterpret_cast<unsigned long long*>(smem + 32);
}

// The unnormalised 2-D DST-I of a pass's n x n plane in LDS: on the matrix cores for FP32
// plans (split lines aliasing the plane, slots at the start of smem), else by the FFT with
// the twiddles at the start of smem.
template <typename T, int R>
__device__ __forceinline__ void plane_transform(T* plane, unsigned char* smem,
                                                const PlaneOperands<T, R>& op) {
  if constexpr (std::is_same<T, float>::value)
    plane_dst_mfma<R>(plane, reinterpret_cast<_Float16*>(plane), reinterpret_cast<float*>(smem),
                      op.s);
  else
    plane_dst<R, T>(plane, reinterpret_cast<const cx<T>*>(smem));
}

// Floats of a pass's plane region: the n x n plane, or for FP32 plans the larger of it and
// the split lines that alias it.
template <typename T, int R>
__host__ __device__ constexpr size_t plane_region_elems() {
  return std::is_same<T, float>::value
             ? ((size_t)(16 * R - 1) * (16 * R - 1) * sizeof(float) > mfma_split_bytes(R)
                    ? (size_t)(16 * R - 1) * (16 * R - 1)
                    : mfma_split_bytes(R) / sizeof(float))
             : (size_t)(16 * R - 1) * (16 * R - 1);
}

// NG: ghost layers of the finite-difference order 2 NG (Sec. 3): the box's Phi_BC^0 and
// potential live on the padded nodes [-NG, M + NG]^3 (padded index = node + NG), and
// Phi_BCs occupies the NG layers outside the interior on each side.
template <typename T, int R, bool ADJ, int NG = 1>
__device__ __forceinline__ void poisson_p1_block(const MeshArgs<T>& a, const BlockMap& m, int L,
                                                 unsigned char* smem) {
  static_assert(!ADJ || NG == 1, "the reverse passes exist for order 2 only");
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int x = m.local[b];
  constexpr int M = 16 * R, n = M - 1, Mp = M + 1 + 2 * NG;
  // FP32 plans transform on the matrix cores (no twiddles: the block-maximum slots lead)
  constexpr bool kMfma = std::is_same<T, float>::value;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem);
  T* plane = reinterpret_cast<T*>(smem + (kMfma ? kMfmaHead : 2 * M * sizeof(cx<T>)));
  if constexpr (!kMfma) load_twiddles(tw, a, t);
  PlaneOperands<T, R> op;
  const int64_t base = t.g_off + (int64_t)x * n * n;
  const double* bc = a.bc0 + t.h_off;
  const double D1 = a.D1_bc;
  if constexpr (ADJ) {
    op.load(a, t);
    const T* const wk = a.work + base;
#pragma unroll 8
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) plane[e] = wk[e];
  } else {
    using Rho = typename MeshFixed<T>::rho_t;
    Rho* const rp = a.rho + base;   // the plane's first node (block-uniform)
    constexpr int kBatch = 16;   // independent loads in flight per thread
    constexpr double kUnit = 1.0 / (double)(1ll << MeshFixed<T>::bits);
    // delta' = delta - Delta Phi_BCs (App. C.1): an interior node next to a face takes
    // D1 Phi_BC^0 of its face-layer neighbour (padded index = node index + 1; interior node
    // index = array index + 1).  Interior x planes need it on their perimeter only (one
    // element per thread, its face values fetched before the mass so that the latencies
    // overlap); the two x-face planes need it everywhere.
    const bool xface = x == 0 || x == n - 1;
    // Phi_BC at the padded node (A, B, C) (node = padded index - 1) over D1: Phi_BC^0, or the
    // full-box potential over D1 in the consistency tests (D1 multiplies it back)
    auto bcv = [&](int A, int B, int C) {
      if (a.ov_phi) return (double)full_at(a.ov_phi, a.ov_N, t, A - NG, B - NG, C - NG) / D1;
      return bc[((int64_t)A * Mp + B) * Mp + C];
    };
    auto yz_term = [&](int y, int z) {
      double s = 0.0;
      if (y == 0) s += bcv(x + 2, 1, z + 2);
      if (y == n - 1) s += bcv(x + 2, M + 1, z + 2);
      if (z == 0) s += bcv(x + 2, y + 2, 1);
      if (z == n - 1) s += bcv(x + 2, y + 2, M + 1);
      return s;
    };
    int pe = -1;
    double pterm = 0.0;
    // the previous solve's third pass left the perimeter terms in this plane of `work`
    const double* const pin =
        NG == 1 && (a.bc_handoff & 1) && !a.ov_phi ? handoff_terms(a.work + base) : nullptr;
    if (NG == 1 && !xface && (int)threadIdx.x < 4 * (n - 1)) {
      int y, z;
      perimeter_yz(threadIdx.x, n, y, z);
      pe = y * n + z;
      pterm = pin ? pin[threadIdx.x] : yz_term(y, z);
    }
    // FP32 plans: the mass the deposit dropped, left per brick of kBlock particles in word 3
    // of the brick's hint; block x = 1 of the box (an interior plane, lighter than the x
    // faces) folds all nb of them into the box's counter and clears them, so the counter
    // takes a few atomics per solve rather than one per block
    constexpr int nb = M * M * M / kBlock;
    const int f0 = 0, f1 = x == 1 ? nb : 0;
    unsigned long long drop = 0;
    if constexpr (std::is_same<T, float>::value) {
      unsigned* const hw = a.hints + (t.p_off / kBlock) * 4 + 3;
      for (int e = f0 + (int)threadIdx.x; e < f1; e += kBlock) {
        drop += hw[4 * e];
        hw[4 * e] = 0u;
      }
    }
    unsigned long long found = 0;   // FP32 plans: the plane's total mass in units
    unsigned near = 0;              // FP32 plans: node masses within a factor 2 of wrapping
    for (int e0 = 0; e0 < n * n; e0 += kBatch * kBlock) {
      Rho r[kBatch];
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int e = e0 + q * kBlock + threadIdx.x;
        r[q] = e < n * n ? rp[e] : Rho(0);
      }
#pragma unroll
      for (int q = 0; q < kBatch; ++q) {
        const int e = e0 + q * kBlock + threadIdx.x;
        if (e >= n * n) continue;
        rp[e] = Rho(0);
        if constexpr (std::is_same<T, float>::value) {
          near += r[q] >> 31;
          found += r[q];
          // FP32: the unit count converted in single precision (exact below 2^24 units,
          // i.e. 8 particles; beyond, one rounding of relative size 2^-24, as the FP32
          // result itself has), times 2^-21 exactly, minus one
          plane[e] = fmaf((float)r[q], (float)kUnit, -1.0f);
        } else {
          plane[e] = (T)(mass_units(r[q]) * kUnit - 1.0);
        }
      }
    }
    // the transform's operands, requested once the mass batch has left the registers
    op.load(a, t);
    if constexpr (std::is_same<T, float>::value) {
      if (near) atomicAdd(a.alarm, (unsigned long long)near);
      // mass identity of FP32 plans: summed over a box's planes, the mass found plus the
      // mass dropped equals one unit per particle and deposit unless a 32-bit node wrapped
      // (each wrap loses exactly 2^32 units).  One atomic per block: the n blocks of a box
      // add to one word and the counters of 16 boxes share a cache line, so the waves'
      // sums meet in LDS first (behind the block-maximum slots; added up after the barrier
      // before the transform)
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) found += __shfl_xor(found, d);
      if ((threadIdx.x & 63) == 0) found_slots(smem)[threadIdx.x >> 6] = found;
      if ((int)(threadIdx.x & ~63u) < f1 - f0) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) drop += __shfl_xor(drop, d);
        if ((threadIdx.x & 63) == 0 && drop != 0ull) atomicAdd(a.dropped + m.tile[b], drop);
      }
    }
    if (a.ov_delta) {
      // the deposit's mass was consumed above; the solve takes the full-box density
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int y = e / n, z = e - (e / n) * n;
        plane[e] = full_at(a.ov_delta, a.ov_N, t, x + 1, y + 1, z + 1);
      }
    }
    __syncthreads();
    if constexpr (NG > 1) {
      // wide stencils: an interior node within NG of a face picks up, along each axis,
      // a_k Phi_BCs at the nodes k = 1..NG away that lie outside [1, M-1]
      const int jx = x + 1;
      const bool xb = jx <= NG || jx >= M - NG;
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int jy = e / n + 1, jz = e - (e / n) * n + 1;
        if (!(xb || jy <= NG || jy >= M - NG || jz <= NG || jz >= M - NG)) continue;
        double s = 0.0;
#pragma unroll
        for (int k = 1; k <= NG; ++k) {
          double o = 0.0;
          if (jx - k <= 0) o += bcv(jx - k + NG, jy + NG, jz + NG);
          if (jx + k >= M) o += bcv(jx + k + NG, jy + NG, jz + NG);
          if (jy - k <= 0) o += bcv(jx + NG, jy - k + NG, jz + NG);
          if (jy + k >= M) o += bcv(jx + NG, jy + k + NG, jz + NG);
          if (jz - k <= 0) o += bcv(jx + NG, jy + NG, jz - k + NG);
          if (jz + k >= M) o += bcv(jx + NG, jy + NG, jz + k + NG);
          s += lap_weight<NG>(k) * o;
        }
        plane[e] = (T)((double)plane[e] - D1 * s);
      }
    } else if (xface) {
      const int A = x == 0 ? 1 : M + 1;   // padded x index of the face layer
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int y = e / n, z = e - (e / n) * n;
        const double s = bcv(A, y + 2, z + 2) + yz_term(y, z);
        plane[e] = (T)((double)plane[e] - D1 * s);
      }
    } else {
      // the remaining perimeter elements of planes wider than the block
      for (int i = threadIdx.x + blockDim.x; i < 4 * (n - 1); i += blockDim.x) {
        int y, z;
        perimeter_yz(i, n, y, z);
        plane[y * n + z] = (T)((double)plane[y * n + z] - D1 * (pin ? pin[i] : yz_term(y, z)));
      }
      if (pe >= 0) plane[pe] = (T)((double)plane[pe] - D1 * pterm);
    }
  }
  __syncthreads();
  if constexpr (!ADJ && std::is_same<T, float>::value) {
    if (threadIdx.x == 0) {
      unsigned long long f = 0;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) f += found_slots(smem)[w];
      if (f != 0ull) atomicAdd(a.kept + m.tile[b], f);
    }
  }
  plane_transform<T, R>(plane, smem, op);
  T* const wk = a.work + base;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) wk[e] = plane[e];
}

// The cw <= kPencilChunk x pencils p0 .. p0 + cw - 1 (pencil p = n y + z) staged in `tile`
// (x rows of kPencilChunk + 1): forward DST-I, the sine-space solve, inverse DST-I.
template <int R, typename T>
__device__ __forceinline__ void pencil_solve(T* tile, int cw, int p0, const T* ev,
                                             const cx<T>* tw) {
  constexpr int M = 16 * R, n = M - 1, pitch = kPencilChunk + 1;
  const int qw = threadIdx.x >> 4, l = threadIdx.x & 15;
  const T norm = T(8.0 / ((double)M * M * M));
  // column pair (2 qw, 2 qw + 1) of the chunk, and lambda_m, lambda_n of each
  T* const la[1] = {tile + 2 * qw};
  T* const lb[1] = {tile + 2 * qw + 1};
  const bool valid[1] = {2 * qw < cw};
  const bool hb[1] = {2 * qw + 1 < cw};
  const int pa = p0 + 2 * qw, pb = pa + 1, ya = pa / n, yb = pb / n;
  const T lya = valid[0] ? ev[ya] : T(-1), lza = valid[0] ? ev[pa - ya * n] : T(-1);
  const T lyb = hb[0] ? ev[yb] : T(-1), lzb = hb[0] ? ev[pb - yb * n] : T(-1);
  // forward DST along x, then Phi^{lmn} = delta^{lmn} 8/M^3 / (lambda_l + lambda_m + lambda_n)
  auto sa = [&](int, int j) { return norm * recip(ev[j - 1] + lya + lza); };
  auto sb = [&](int, int j) { return norm * recip(ev[j - 1] + lyb + lzb); };
  dst_quarter<R, 1, pitch, T>(la, lb, valid, hb, tw, l, sa, sb);
  // the same quarter wavefront reads back only the lines it wrote
  auto one = [](int, int) { return T(1); };
  dst_quarter<R, 1, pitch, T>(la, lb, valid, hb, tw, l, one, one);
  __syncthreads();
}

template <typename T, int R>
__device__ __forceinline__ void poisson_p2_block(const MeshArgs<T>& a, const BlockMap& m, int L,
                                                 unsigned char* smem) {
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  constexpr int M = 16 * R, n = M - 1;
  constexpr int C = pencil_chunk<T>();
  // chunks of C consecutive pencils of the box's n^2 (only the box's last one partial); the
  // chunk's nodes of one x plane are C consecutive words
  const int p0 = m.local[b] * C, cw = min(C, n * n - p0);
  if constexpr (std::is_same<T, float>::value) {
    pencils_mfma<R>(a.work + t.g_off + p0, p0, cw, a.eigen + t.ev_off,
                    reinterpret_cast<const _Float16*>(a.sine) + t.dm_off, smem);
    return;
  }
  constexpr int pitch = kPencilChunk + 1;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem);
  T* ev = reinterpret_cast<T*>(smem + 2 * M * sizeof(cx<T>));
  T* tile = ev + M;
  load_twiddles(tw, a, t);
  for (int i = threadIdx.x; i < n; i += blockDim.x) ev[i] = a.eigen[t.ev_off + i];
  // thread -> (x row x0 + 8 i, chunk column zc): rows of 32 consecutive pencils, coalesced
  static_assert(kPencilChunk == 32 && kBlock == 256, "eight rows of 32 columns per sweep");
  const int zc = threadIdx.x & 31, x0 = threadIdx.x >> 5;
  const bool zin = zc < cw;
  // the chunk's first pencil (block-uniform) plus the thread's 32-bit offset; each sweep of
  // eight rows adds a uniform 8 n^2
  T* const col = a.work + t.g_off + p0;
  const int lo = x0 * n * n + zc;
#pragma unroll
  for (int i = 0; i < (n + 7) / 8; ++i) {
    const int x = x0 + 8 * i;
    if (zin && x < n) tile[x * pitch + zc] = (col + (int64_t)8 * i * n * n)[lo];
  }
  __syncthreads();
  pencil_solve<R, T>(tile, cw, p0, ev, tw);
#pragma unroll
  for (int i = 0; i < (n + 7) / 8; ++i) {
    const int x = x0 + 8 * i;
    if (zin && x < n) (col + (int64_t)8 * i * n * n)[lo] = tile[x * pitch + zc];
  }
}

template <typename T, int R, bool ADJ, int NG = 1>
__device__ __forceinline__ void poisson_p3_block(const MeshArgs<T>& a, const BlockMap& m, int L,
                                                 unsigned char* smem) {
  static_assert(!ADJ || NG == 1, "the reverse passes exist for order 2 only");
  const int b = m.base + L;
  const TileDesc t = a.tiles[m.tile[b]];
  const int local = m.local[b];
  constexpr int M = 16 * R, n = M - 1, Mp = M + 1 + 2 * NG;
  const double* bc = a.bc0 + t.h_off;
  T* phi = a.phi + t.h_off;
  const double D1 = a.D1_bc;
  if (local >= n) {
    if (ADJ) return;
    // one of the 2 (NG + 1) shell planes: padded x index 0..NG (nodes -NG..0) and
    // M + NG..M + 2 NG (nodes M..M + NG)
    const int s = local - n;
    const int A = s <= NG ? s : M + s - 1;
    if (a.ov_phi) {
      for (int e = threadIdx.x; e < Mp * Mp; e += blockDim.x)
        phi[(int64_t)A * Mp * Mp + e] = full_at(a.ov_phi, a.ov_N, t, A - NG, e / Mp - NG,
                                                e - (e / Mp) * Mp - NG);
      return;
    }
    for (int e = threadIdx.x; e < Mp * Mp; e += blockDim.x)
      phi[(int64_t)A * Mp * Mp + e] = (T)(D1 * bc[(int64_t)A * Mp * Mp + e]);
    return;
  }
  constexpr bool kMfma = std::is_same<T, float>::value;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem);
  T* plane = reinterpret_cast<T*>(smem + (kMfma ? kMfmaHead : 2 * M * sizeof(cx<T>)));
  if constexpr (!kMfma) load_twiddles(tw, a, t);
  PlaneOperands<T, R> op;
  op.load(a, t);
  const int x = local;
  const int64_t base = t.g_off + (int64_t)x * n * n;
  const int A = x + 1 + NG;
  // the padded plane's border (NG + 1 layers on each side) takes D1 Phi_BC^0: those values
  // are fetched first so that their latency overlaps the load of the plane, and held in
  // registers until the plane is written.  Border element i: rows 0..NG and M+NG..M+2NG
  // whole, then columns 0..NG and M+NG..M+2NG of the rows in between.
  constexpr int kBorder = Mp * Mp - n * n;
  constexpr int kPerThread = (kBorder + kBlock - 1) / kBlock;
  constexpr int kW = 2 * (NG + 1);   // border rows, and border columns per inner row
  auto border_offset = [](int i) {
    int B, C;
    if (i < kW * Mp) {
      const int r = i / Mp;
      B = r <= NG ? r : M - 1 + r;
      C = i - r * Mp;
    } else {
      const int j = i - kW * Mp, r = j / kW, c = j - r * kW;
      B = NG + 1 + r;
      C = c <= NG ? c : M - 1 + c;
    }
    return B * Mp + C;
  };
  double bval[kPerThread];
  if constexpr (!ADJ) {
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int i = q * kBlock + threadIdx.x;
      bval[q] = i < kBorder ? bc[(int64_t)A * Mp * Mp + border_offset(i)] : 0.0;
    }
  }
  // adjoint: lam_bc0 -= D1 C^T lam_delta' on the face layer.  Each face node has exactly
  // one interior neighbour, so plain updates do not collide.  On an interior x plane only
  // the perimeter touches a face (one element per thread): the old values of its face nodes
  // are fetched here, so that their latency overlaps the load of the plane.
  double* lb = a.lam_bc0 + t.h_off;
  const bool xface = x == 0 || x == n - 1;
  int pe = -1, iy = -1, iz = -1;   // indices into the box's padded grid (< 2^31)
  double oy = 0.0, oz = 0.0;
  if constexpr (ADJ) {
    if (!xface && (int)threadIdx.x < 4 * (n - 1)) {
      const int i = threadIdx.x, side = i / (n - 1), o = i - side * (n - 1);
      const int y = side == 0 ? 0 : side == 1 ? o : side == 2 ? n - 1 : n - 1 - o;
      const int z = side == 0 ? o : side == 1 ? n - 1 : side == 2 ? n - 1 - o : 0;
      pe = y * n + z;
      if (y == 0) iy = ((x + 2) * Mp + 1) * Mp + z + 2;
      if (y == n - 1) iy = ((x + 2) * Mp + M + 1) * Mp + z + 2;
      if (z == 0) iz = ((x + 2) * Mp + y + 2) * Mp + 1;
      if (z == n - 1) iz = ((x + 2) * Mp + y + 2) * Mp + M + 1;
      if (iy >= 0) oy = lb[iy];
      if (iz >= 0) oz = lb[iz];
    }
  }
  const T* const wk = a.work + base;
#pragma unroll 8
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) plane[e] = wk[e];
  // order 2, evolution: the first pass of the next solve takes this plane's perimeter terms
  // (the same padded plane A's face-layer values, which bval holds) from its `work` plane;
  // they are summed in LDS right behind the n x n plane (for FP32 plans inside the region
  // that the transform's split lines take later) in the first pass's order (the y face,
  // then the z face), one writer per term in each of two phases around the barrier below,
  // and stored before the transform
  const bool hand_out = NG == 1 && !ADJ && (a.bc_handoff & 2) != 0;
  double* const pacc = handoff_terms(plane + n * n);
  static_assert(!std::is_same<T, float>::value ||
                    (plane_region_elems<T, R>() - (size_t)n * n) * sizeof(float) >=
                        8 + 4 * (size_t)(n - 1) * sizeof(double),
                "the perimeter terms fit behind the plane in the FP32 region");
  T bv[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) bv[q] = T(0);
  if constexpr (!ADJ) {
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int i = q * kBlock + threadIdx.x;
      if (i < kBorder) bv[q] = (T)(D1 * bval[q]);
      // rows B = 1 and B = M + 1: the y faces of interior rows y = 0 and y = n - 1
      if (hand_out && i >= Mp && i < 3 * Mp) {
        const int C = i - (i >= 2 * Mp ? 2 * Mp : Mp);
        if (C >= 2 && C <= M) pacc[perimeter_index(i < 2 * Mp ? 0 : n - 1, C - 2, n)] = bval[q];
      }
    }
    if (a.ov_phi) {
#pragma unroll
      for (int q = 0; q < kPerThread; ++q) {
        const int i = q * kBlock + threadIdx.x;
        if (i < kBorder) {
          const int o = border_offset(i);
          bv[q] = full_at(a.ov_phi, a.ov_N, t, A - NG, o / Mp - NG, o - (o / Mp) * Mp - NG);
        }
      }
    }
  }
  __syncthreads();
  if (hand_out) {
    // columns C = 1 and C = M + 1 of the inner rows: the z faces of z = 0 and z = n - 1,
    // added to the y face's value at the four corners
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int i = q * kBlock + threadIdx.x;
      if (i >= 4 * Mp && i < kBorder) {
        const int j = i - 4 * Mp, y = j >> 2, c = j & 3;
        if (c == 1 || c == 2) {
          const int pi = perimeter_index(y, c == 1 ? 0 : n - 1, n);
          pacc[pi] = (y == 0 || y == n - 1) ? pacc[pi] + bval[q] : bval[q];
        }
      }
    }
    __syncthreads();
    // every thread's loads of the work plane ended before the barrier above; the
    // transform's first barrier orders these reads of pacc before its split lines
    double* const out = handoff_terms(a.work + base);
    for (int i = threadIdx.x; i < 4 * (n - 1); i += blockDim.x) out[i] = pacc[i];
  }
  plane_transform<T, R>(plane, smem, op);
  if constexpr (ADJ) {
    // lam_rho = lam_delta', and the plane of `work` is cleared (the next reverse step
    // accumulates into a zeroed source)
    T* const lr = a.lam_rho + base;
    T* const wz = a.work + base;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      lr[e] = plane[e];
      wz[e] = T(0);
    }
    if (xface) {
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int y = e / n, z = e - (e / n) * n;
        const double d = -D1 * (double)plane[e];
        if (x == 0) lb[((int64_t)1 * Mp + y + 2) * Mp + z + 2] += d;
        if (x == n - 1) lb[((int64_t)(M + 1) * Mp + y + 2) * Mp + z + 2] += d;
        if (y == 0) lb[((int64_t)(x + 2) * Mp + 1) * Mp + z + 2] += d;
        if (y == n - 1) lb[((int64_t)(x + 2) * Mp + M + 1) * Mp + z + 2] += d;
        if (z == 0) lb[((int64_t)(x + 2) * Mp + y + 2) * Mp + 1] += d;
        if (z == n - 1) lb[((int64_t)(x + 2) * Mp + y + 2) * Mp + M + 1] += d;
      }
    } else {
      // perimeter elements beyond the first blockDim.x (planes wider than the block)
      for (int i = threadIdx.x + blockDim.x; i < 4 * (n - 1); i += blockDim.x) {
        const int side = i / (n - 1), o = i - side * (n - 1);
        const int y = side == 0 ? 0 : side == 1 ? o : side == 2 ? n - 1 : n - 1 - o;
        const int z = side == 0 ? o : side == 1 ? n - 1 : side == 2 ? n - 1 - o : 0;
        const double d = -D1 * (double)plane[y * n + z];
        if (y == 0) lb[((int64_t)(x + 2) * Mp + 1) * Mp + z + 2] += d;
        if (y == n - 1) lb[((int64_t)(x + 2) * Mp + M + 1) * Mp + z + 2] += d;
        if (z == 0) lb[((int64_t)(x + 2) * Mp + y + 2) * Mp + 1] += d;
        if (z == n - 1) lb[((int64_t)(x + 2) * Mp + y + 2) * Mp + M + 1] += d;
      }
      if (pe >= 0) {
        const double d = -D1 * (double)plane[pe];
        if (iy >= 0) lb[iy] = oy + d;
        if (iz >= 0) lb[iz] = oz + d;
      }
    }
    return;
  }
  T* out = phi + (int64_t)A * Mp * Mp;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int y = e / n, z = e - (e / n) * n;
    out[(y + 1 + NG) * Mp + z + 1 + NG] = plane[e];
  }
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int i = q * kBlock + threadIdx.x;
    if (i < kBorder) out[border_offset(i)] = bv[q];
  }
}

}  // namespace
}  // namespace scola
