// DST-I of FP32 plans (App. C.2, eq. DST_delta) as products with the sine matrix on the
// matrix cores.  A line has n = 16R - 1 points, short enough that the dense product (n^2
// multiply-adds per line) costs less on the matrix cores than an FFT on the vector units,
// where the three Poisson passes are issue-bound.
//
// Precision: the products run in FP16 with FP32 accumulation.  Every FP32 operand v enters
// split in two halves, v = hi + lo with hi = fp16(v) and lo = fp16(v - hi) (v - hi is exact
// in FP32; together 22 significant bits, representation error below 2^-23 |v|), after a
// power-of-two scaling per block that keeps |v| at most 2^13 (no FP16 overflow; values far
// below the block maximum keep an absolute error below 2^-38 of it).  The sine matrix is
// split the same way on the host, and hi*hi + hi*lo + lo*hi are accumulated; the dropped
// lo*lo term is below 2^-22 of each product.  The result is within a small multiple of FP32
// rounding of the exact transform.
//
// Operand layout of v_mfma_f32_16x16x32_f16 as used here: lane l supplies row (A) or column
// (B) l mod 16 and eight K values of slot group l / 16; the result holds rows 4 (l / 16) + r,
// r = 0..3, of column l mod 16.  A and B take their K values through the same slot mapping,
// k = 32 kc + 8 (l / 16) + s, so the contraction does not depend on how the hardware orders
// K inside an instruction.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace scola {
namespace {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Shapes of the transform of lines of M = 16R nodes (n = M - 1 values, index j <-> node
// j + 1): rows and lines padded to M, the contraction padded to K = 32 KC, split lines in LDS
// at a pitch of KP halves (K + 8: rows 16 bytes apart in bank phase, conflict-free 16-byte
// reads).  Each wave owns the 16-row tiles w, w + 4 (TW of them) of the sine matrix.
template <int R>
struct MfmaDst {
  static constexpr int M = 16 * R, n = M - 1;
  static constexpr int KC = (R + 1) / 2, K = 32 * KC, KP = K + 8;
  static constexpr int kWavesPerBlock = kBlock / 64;
  static constexpr int TW = (R + kWavesPerBlock - 1) / kWavesPerBlock;
};

// Bytes of one split buffer: M lines of KP halves, hi then lo.
__host__ __device__ constexpr size_t mfma_split_bytes(int R) {
  return (size_t)16 * R * (32 * ((R + 1) / 2) + 8) * 2 * sizeof(_Float16);
}
// Bytes in front of the passes' LDS data (the block-maximum slots), keeping it 16-byte aligned.
constexpr size_t kMfmaHead = 64;

// The wave's sine fragments: rows 16 (w + 4 tw) + l mod 16 of S (hi and lo) for every K
// chunk, zero for rows beyond the padded length.  S points at this M's table: M rows of K
// halves, hi, then the same for lo (rows and columns >= n are zero).
template <int R>
struct SineFrag {
  h8 hi[MfmaDst<R>::TW][MfmaDst<R>::KC];
  h8 lo[MfmaDst<R>::TW][MfmaDst<R>::KC];
};

template <int R>
__device__ __forceinline__ SineFrag<R> load_sine(const _Float16* __restrict__ S) {
  using D = MfmaDst<R>;
  SineFrag<R> f;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int tw = 0; tw < D::TW; ++tw) {
    const int rt = w + D::kWavesPerBlock * tw;
#pragma unroll
    for (int kc = 0; kc < D::KC; ++kc) {
      if (rt < R) {
        const int o = (16 * rt + (l & 15)) * D::K + 32 * kc + 8 * (l >> 4);
        f.hi[tw][kc] = *reinterpret_cast<const h8*>(S + o);
        f.lo[tw][kc] = *reinterpret_cast<const h8*>(S + D::M * D::K + o);
      } else {
        f.hi[tw][kc] = h8{};
        f.lo[tw][kc] = h8{};
      }
    }
  }
  return f;
}

__device__ __forceinline__ f4 mfma3(h8 ah, h8 al, h8 bh, h8 bl, f4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh, c, 0, 0, 0);
  return c;
}

// Block-wide maximum of a non-negative value per thread (NaN-free inputs), uniform; `slots`
// holds kWavesPerBlock floats that no other thread reads until a later barrier.  Contains
// one barrier.
__device__ __forceinline__ float block_max_abs(float m, float* slots) {
  m = fmaxf(m, lane_xor<1>(m));
  m = fmaxf(m, lane_xor<2>(m));
  m = fmaxf(m, lane_xor<4>(m));
  m = fmaxf(m, lane_xor<8>(m));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 16));
  const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 32));
  const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(m), 48));
  if ((threadIdx.x & 63) == 0) slots[threadIdx.x >> 6] = fmaxf(fmaxf(a, b), fmaxf(c, d));
  __syncthreads();
  float r = slots[0];
#pragma unroll
  for (int w = 1; w < kBlock / 64; ++w) r = fmaxf(r, slots[w]);
  return r;
}

// 2^(13 - e) for a block maximum m = f 2^e (f in [0.5, 1)): m times it lies in [2^12, 2^13];
// 1 for m = 0.  The exponent is clamped so that the scale stays a finite normal number.
__device__ __forceinline__ float pow2_scale(float m) {
  if (!(m > 0.0f)) return 1.0f;
  const int e = min(max(__builtin_amdgcn_frexp_expf(m), -100), 100);
  return __builtin_amdgcn_ldexpf(1.0f, 13 - e);
}

__device__ __forceinline__ void split_half(float v, _Float16& h, _Float16& l) {
  h = (_Float16)v;
  l = (_Float16)(v - (float)h);
}

// Out[line][j] = sum_k In[line][k] S[j][k] for every line tile (16 lines each, LT of them)
// and the wave's sine rows j: the data lines are the A operand (row = line), the sine rows
// the B operand.  Element r of d[lt][tw] is line 16 lt + 4 (l / 16) + r, sine row
// 16 (w + 4 tw) + l mod 16.
template <int R, int LT>
__device__ __forceinline__ void lines_times_sine(const _Float16* bh, const _Float16* bl,
                                                 const SineFrag<R>& s, f4 (&d)[LT][MfmaDst<R>::TW]) {
  using D = MfmaDst<R>;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int lt = 0; lt < LT; ++lt)
#pragma unroll
    for (int tw = 0; tw < D::TW; ++tw) d[lt][tw] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int lt = 0; lt < LT; ++lt)
#pragma unroll
    for (int kc = 0; kc < D::KC; ++kc) {
      const int o = (16 * lt + (l & 15)) * D::KP + 32 * kc + 8 * (l >> 4);
      const h8 xh = *reinterpret_cast<const h8*>(bh + o);
      const h8 xl = *reinterpret_cast<const h8*>(bl + o);
#pragma unroll
      for (int tw = 0; tw < D::TW; ++tw)
        if (w + D::kWavesPerBlock * tw < R)
          d[lt][tw] = mfma3(xh, xl, s.hi[tw][kc], s.lo[tw][kc], d[lt][tw]);
    }
}

// Out[j][line] = sum_k S[j][k] In[line][k] for the wave's sine rows j and every line tile:
// the sine rows are the A operand.  Element r of d[tw][lt] is sine row 16 (w + 4 tw) +
// 4 (l / 16) + r, line 16 lt + l mod 16.
template <int R, int LT>
__device__ __forceinline__ void sine_times_lines(const SineFrag<R>& s, const _Float16* bh,
                                                 const _Float16* bl, f4 (&d)[MfmaDst<R>::TW][LT]) {
  using D = MfmaDst<R>;
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int tw = 0; tw < D::TW; ++tw)
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) d[tw][lt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int lt = 0; lt < LT; ++lt)
#pragma unroll
    for (int kc = 0; kc < D::KC; ++kc) {
      const int o = (16 * lt + (l & 15)) * D::KP + 32 * kc + 8 * (l >> 4);
      const h8 xh = *reinterpret_cast<const h8*>(bh + o);
      const h8 xl = *reinterpret_cast<const h8*>(bl + o);
#pragma unroll
      for (int tw = 0; tw < D::TW; ++tw)
        if (w + D::kWavesPerBlock * tw < R)
          d[tw][lt] = mfma3(s.hi[tw][kc], s.lo[tw][kc], xh, xl, d[tw][lt]);
    }
}

// Four consecutive K positions of one line, scaled and split, as two 8-byte LDS stores.
__device__ __forceinline__ void store_split4(_Float16* bh, _Float16* bl, int o, f4 v, float sc) {
  h4 hv, lv;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    _Float16 h, lo;
    split_half(v[r] * sc, h, lo);
    hv[r] = h;
    lv[r] = lo;
  }
  *reinterpret_cast<h4*>(bh + o) = hv;
  *reinterpret_cast<h4*>(bl + o) = lv;
}

// In-place unnormalised DST-I along z (rows, stride 1) and y (stride n) of the n x n plane
// at `plane`.  `buf` (mfma_split_bytes(R), 16-byte aligned) may alias the plane: the plane
// is read into registers before it is written.  `slots` holds 2 kWavesPerBlock floats; `s`
// are the wave's sine fragments (load_sine, issued early by the caller so that their
// latency overlaps its own loads).  Must be called by all threads of the block; ends with
// a barrier.
template <int R>
__device__ __forceinline__ void plane_dst_mfma(float* plane, _Float16* buf, float* slots,
                                               const SineFrag<R>& s) {
  using D = MfmaDst<R>;
  constexpr int n = D::n, M = D::M, K = D::K, KP = D::KP;
  _Float16* const bh = buf;
  _Float16* const bl = buf + M * KP;
  // the plane (zero beyond n x n, up to M lines of K values) in registers, and its maximum
  constexpr int kElems = M * K, kPer = (kElems + kBlock - 1) / kBlock;
  float v[kPer];
  float m = 0.0f;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = q * kBlock + (int)threadIdx.x, y = e / K, z = e - (e / K) * K;
    v[q] = (e < kElems && y < n && z < n) ? plane[y * n + z] : 0.0f;
    m = fmaxf(m, fabsf(v[q]));
  }
  const float s1 = pow2_scale(block_max_abs(m, slots));   // its barrier ends the plane reads
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int e = q * kBlock + (int)threadIdx.x, y = e / K, z = e - (e / K) * K;
    if (e < kElems) split_half(v[q] * s1, bh[y * KP + z], bl[y * KP + z]);
  }
  __syncthreads();
  // along z: A[y][kz] = sum_z Y[y][z] S[kz][z]
  f4 da[R][D::TW];
  lines_times_sine<R, R>(bh, bl, s, da);
  float m2 = 0.0f;
#pragma unroll
  for (int lt = 0; lt < R; ++lt)
#pragma unroll
    for (int tw = 0; tw < D::TW; ++tw)
#pragma unroll
      for (int r = 0; r < 4; ++r) m2 = fmaxf(m2, fabsf(da[lt][tw][r]));
  const float s2 = pow2_scale(block_max_abs(m2, slots + D::kWavesPerBlock));
  // A transposed into the lines of the y pass: line kz, positions y (four per lane); the
  // positions K > M of odd R keep the zeros written above
  {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int lt = 0; lt < R; ++lt)
#pragma unroll
      for (int tw = 0; tw < D::TW; ++tw)
        if (w + D::kWavesPerBlock * tw < R) {
          const int kz = 16 * (w + D::kWavesPerBlock * tw) + (l & 15);
          store_split4(bh, bl, kz * KP + 16 * lt + 4 * (l >> 4), da[lt][tw], s2);
        }
  }
  __syncthreads();
  // along y: Z[ky][kz] = sum_y S[ky][y] A[y][kz]
  f4 db[D::TW][R];
  sine_times_lines<R, R>(s, bh, bl, db);
  __syncthreads();   // every read of the split lines is done before the plane is written
  const float inv = 1.0f / (s1 * s2);   // a power of two: exact
  {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int tw = 0; tw < D::TW; ++tw)
#pragma unroll
      for (int lt = 0; lt < R; ++lt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ky = 16 * (w + D::kWavesPerBlock * tw) + 4 * (l >> 4) + r;
          const int kz = 16 * lt + (l & 15);
          if (w + D::kWavesPerBlock * tw < R && ky < n && kz < n)
            plane[ky * n + kz] = db[tw][lt][r] * inv;
        }
  }
  __syncthreads();
}

// The x pencils of one chunk of the pencil pass: the cw <= C (C = kPencilChunkMfma)
// consecutive pencils p0 .. p0 + cw - 1 of the box's n^2 pencils, pencil p = n y + z (the
// (y, z) column p / n, p mod n, so a chunk may span two rows): forward DST-I along x,
// Phi^{lmn} = delta^{lmn} 8 / M^3 / (lambda_l + lambda_m + lambda_n) (eq.
// Poisson_sine_space), inverse DST-I along x.  `col` is the chunk's first node (x = 0,
// pencil p0) of the box's work array, where the chunk's nodes of one x plane are C
// consecutive words; smem holds the block-maximum slots (kMfmaHead), the eigenvalues (M
// floats), then the split lines of the C columns, which the output tile (n rows of C + 1
// floats) later overwrites.
template <int R>
__device__ __forceinline__ void pencils_mfma(float* __restrict__ col, int p0, int cw,
                                             const float* __restrict__ eigen,
                                             const _Float16* __restrict__ S,
                                             unsigned char* smem) {
  using D = MfmaDst<R>;
  constexpr int M = D::M, n = D::n, K = D::K, KP = D::KP, C = kPencilChunkMfma, pitch = C + 1;
  constexpr int LT = C / 16, kSweep = kBlock / C;   // line tiles; x rows per sweep
  static_assert(C == 64 && kBlock % C == 0, "one wave per row of the chunk");
  float* const slots = reinterpret_cast<float*>(smem);
  float* const ev = reinterpret_cast<float*>(smem + kMfmaHead);
  _Float16* const bh = reinterpret_cast<_Float16*>(smem + kMfmaHead + M * sizeof(float));
  _Float16* const bl = bh + C * KP;
  float* const tile = reinterpret_cast<float*>(bh);
  const SineFrag<R> s = load_sine<R>(S);
  for (int i = threadIdx.x; i < n; i += blockDim.x) ev[i] = eigen[i];
  // thread -> (x rows x0 + kSweep i, z column zc): rows of C consecutive z, coalesced; the
  // rows run to K so that the padding of the split lines is written as zeros
  const int zc = threadIdx.x % C, x0 = threadIdx.x / C;
  const bool zin = zc < cw;
  const int lo = x0 * n * n + zc;
  constexpr int kRows = K / kSweep;
  float v[kRows];
  float m = 0.0f;
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int x = x0 + kSweep * i;
    v[i] = (zin && x < n) ? (col + (int64_t)kSweep * i * n * n)[lo] : 0.0f;
    m = fmaxf(m, fabsf(v[i]));
  }
  const float s1 = pow2_scale(block_max_abs(m, slots));   // its barrier also publishes ev
#pragma unroll
  for (int i = 0; i < kRows; ++i) {
    const int x = x0 + kSweep * i;
    split_half(v[i] * s1, bh[zc * KP + x], bl[zc * KP + x]);
  }
  __syncthreads();
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  // forward along x, then the sine-space solve
  f4 d[D::TW][LT];
  sine_times_lines<R, LT>(s, bh, bl, d);
  const float norm = (float)(8.0 / ((double)M * M * M));
  // lambda_m and lambda_n of the lane's column in each line tile (pencil p0 + 16 lt + l mod
  // 16; columns beyond the chunk take index 0 and a zero factor below)
  float ly[LT], lz[LT];
#pragma unroll
  for (int lt = 0; lt < LT; ++lt) {
    const int c = 16 * lt + (l & 15), p = c < cw ? p0 + c : 0, py = p / n;
    ly[lt] = ev[py];
    lz[lt] = ev[p - py * n];
  }
  float m2 = 0.0f;
#pragma unroll
  for (int tw = 0; tw < D::TW; ++tw)
#pragma unroll
    for (int lt = 0; lt < LT; ++lt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int kx = 16 * (w + D::kWavesPerBlock * tw) + 4 * (l >> 4) + r;
        const int z = 16 * lt + (l & 15);
        const float f =
            (kx < n && z < cw) ? norm * __builtin_amdgcn_rcpf(ev[kx] + ly[lt] + lz[lt]) : 0.0f;
        d[tw][lt][r] *= f;
        m2 = fmaxf(m2, fabsf(d[tw][lt][r]));
      }
  const float s2 = pow2_scale(block_max_abs(m2, slots + D::kWavesPerBlock));
#pragma unroll
  for (int tw = 0; tw < D::TW; ++tw)
    if (w + D::kWavesPerBlock * tw < R)
#pragma unroll
      for (int lt = 0; lt < LT; ++lt)
        store_split4(bh, bl,
                     (16 * lt + (l & 15)) * KP + 16 * (w + D::kWavesPerBlock * tw) + 4 * (l >> 4),
                     d[tw][lt], s2);
  __syncthreads();
  // inverse along x
  sine_times_lines<R, LT>(s, bh, bl, d);
  __syncthreads();   // the tile overwrites the split lines
  const float inv = 1.0f / (s1 * s2);
#pragma unroll
  for (int tw = 0; tw < D::TW; ++tw)
#pragma unroll
    for (int lt = 0; lt < LT; ++lt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int x = 16 * (w + D::kWavesPerBlock * tw) + 4 * (l >> 4) + r;
        const int z = 16 * lt + (l & 15);
        if (w + D::kWavesPerBlock * tw < R && x < n && z < cw)
          tile[x * pitch + z] = d[tw][lt][r] * inv;
      }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < (n + kSweep - 1) / kSweep; ++i) {
    const int x = x0 + kSweep * i;
    if (zin && x < n) (col + (int64_t)kSweep * i * n * n)[lo] = tile[x * pitch + zc];
  }
}

}  // namespace
}  // namespace scola
