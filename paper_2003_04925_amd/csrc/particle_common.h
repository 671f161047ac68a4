// Device helpers shared by the particle kernels of the forward step and of its adjoint:
// XCD-aware block numbering, wave and block reductions, and LDS window indexing.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace scola {
namespace {

// Logical block index: hardware dispatches consecutive workgroups round-robin over the 8
// XCDs, so logical = (b % 8) * (grid / 8) + b / 8 gives each XCD a contiguous run of
// logical blocks (whole boxes).
__device__ inline int logical_block(const BlockMap& m) {
  const int b = blockIdx.x;
  if (!m.xcd_remap) return b;
  const int per = gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

inline unsigned padded_grid(const BlockMap& m) {
  if (!m.xcd_remap) return (unsigned)m.count;
  return (unsigned)(((m.count + 7) / 8) * 8);
}

// Wave-wide min / max: DPP exchanges inside 16-lane rows, then the four row results are
// read into scalars; the result is uniform across the wave.
__device__ __forceinline__ int wave_min(int v) {
  v = min(v, lane_xor<1>(v));
  v = min(v, lane_xor<2>(v));
  v = min(v, lane_xor<4>(v));
  v = min(v, lane_xor<8>(v));
  return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}
__device__ __forceinline__ int wave_max(int v) {
  v = max(v, lane_xor<1>(v));
  v = max(v, lane_xor<2>(v));
  v = max(v, lane_xor<4>(v));
  v = max(v, lane_xor<8>(v));
  return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
             max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

constexpr int kWindow = 4096;   // LDS window entries per block (potential or mass)

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Lane-wise minimum of two pairs of unsigned 16-bit values packed in 32 bits.
__device__ __forceinline__ unsigned pk_min_u16(unsigned a, unsigned b) {
  return __builtin_bit_cast(unsigned, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

// Wave-wide minimum of a packed pair of unsigned 16-bit values (one DPP exchange per step
// moves both halves); the result is uniform across the wave.
__device__ __forceinline__ unsigned wave_min_u16x2(unsigned v) {
  v = pk_min_u16(v, (unsigned)lane_xor<1>((int)v));
  v = pk_min_u16(v, (unsigned)lane_xor<2>((int)v));
  v = pk_min_u16(v, (unsigned)lane_xor<4>((int)v));
  v = pk_min_u16(v, (unsigned)lane_xor<8>((int)v));
  return pk_min_u16(pk_min_u16(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
                    pk_min_u16(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

// Block-wide bounding box of per-thread integer ranges [lo, hi] (3 axes, values in
// [-16383, 16383]); threads with any == false do not count.  The six extrema are reduced
// as three packed pairs of 16-bit minima: lo + 2^14 and 2^14 - hi (0xffff marks "none").
// Must be called by all threads of the block.
__device__ inline void block_bounds(bool any, const int (&lo)[3], const int (&hi)[3],
                                    int* bounds) {
  constexpr int kOff = 1 << 14;
  if (threadIdx.x < 6) bounds[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -0x7fffffff;
  __syncthreads();
  const unsigned none = 0xffffffffu;
  const unsigned p0 = any ? (unsigned)(lo[0] + kOff) | ((unsigned)(lo[1] + kOff) << 16) : none;
  const unsigned p1 = any ? (unsigned)(lo[2] + kOff) | ((unsigned)(kOff - hi[0]) << 16) : none;
  const unsigned p2 = any ? (unsigned)(kOff - hi[1]) | ((unsigned)(kOff - hi[2]) << 16) : none;
  const unsigned r0 = wave_min_u16x2(p0), r1 = wave_min_u16x2(p1), r2 = wave_min_u16x2(p2);
  if ((threadIdx.x & 63) == 0 && (r0 & 0xffffu) != 0xffffu) {   // the wave has a range
    atomicMin(bounds + 0, (int)(r0 & 0xffffu) - kOff);
    atomicMin(bounds + 1, (int)(r0 >> 16) - kOff);
    atomicMin(bounds + 2, (int)(r1 & 0xffffu) - kOff);
    atomicMax(bounds + 3, kOff - (int)(r1 >> 16));
    atomicMax(bounds + 4, kOff - (int)(r2 & 0xffffu));
    atomicMax(bounds + 5, kOff - (int)(r2 >> 16));
  }
  __syncthreads();
}

// block_bounds plus the block-wide maximum of one int per thread, left in bounds[6] (the
// caller's array holds at least 7 entries).  Must be called by all threads of the block.
__device__ inline void block_bounds_max(bool any, const int (&lo)[3], const int (&hi)[3], int v,
                                        int* bounds) {
  if (threadIdx.x < 7) bounds[threadIdx.x] = threadIdx.x < 3 ? 0x7fffffff : -0x7fffffff;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int a = wave_min(any ? lo[c] : 0x7fffffff);
    const int b = wave_max(any ? hi[c] : -0x7fffffff);
    if ((threadIdx.x & 63) == 0) {
      atomicMin(bounds + c, a);
      atomicMax(bounds + 3 + c, b);
    }
  }
  const int m = wave_max(v);
  if ((threadIdx.x & 63) == 0) atomicMax(bounds + 6, m);
  __syncthreads();
}

// The LDS window of a block from the bounds left by block_bounds: nodes [l, l + w) per
// axis.  A block in which no thread contributed keeps the sentinels (lo > hi) and gets an
// empty window; the widths are formed only for a non-empty window, where they are at most
// M + 3, so the arithmetic cannot overflow.
struct BlockWindow {
  int lx, ly, lz, wx, wy, wz, vol;
  bool lds;   // fits in kWindow entries
};

__device__ inline BlockWindow block_window(const int* bounds) {
  BlockWindow w;
  w.lx = bounds[0];
  w.ly = bounds[1];
  w.lz = bounds[2];
  const bool empty = bounds[0] > bounds[3] || bounds[1] > bounds[4] || bounds[2] > bounds[5];
  w.wx = empty ? 0 : bounds[3] - bounds[0] + 1;
  w.wy = empty ? 0 : bounds[4] - bounds[1] + 1;
  w.wz = empty ? 0 : bounds[5] - bounds[2] + 1;
  w.vol = w.wx * w.wy * w.wz;
  w.lds = !empty && w.vol <= kWindow;
  return w;
}

// Row-major index (a * nb + b) * nc + c of a 3-D array with fewer than 2^24 entries and
// non-negative coordinates, with full-rate 24-bit multiplies.
__device__ __forceinline__ unsigned idx3(int a, int b, int c, int nb, int nc) {
  return __umul24(__umul24((unsigned)a, (unsigned)nb) + (unsigned)b, (unsigned)nc) + (unsigned)c;
}

// Row-major decomposition e -> (ex, ey, ez) of a window with rows wy x wz, using FP32
// reciprocals (exact for windows far below 2^20 entries) instead of integer division.
__device__ inline void window_coords(int e, int wz, int wyz, float inv_wz, float inv_wyz,
                                     int& ex, int& ey, int& ez) {
  ex = (int)(((float)e + 0.5f) * inv_wyz);
  const int r = e - ex * wyz;
  ey = (int)(((float)r + 0.5f) * inv_wz);
  ez = r - ey * wz;
}

// LDS windows of a block.  The fast form has a fixed geometry of kFw^3 nodes with
// compile-time pitches (x: kFw^2, y: kFw, z: 1): every stencil read and every deposit of a
// particle is one base address plus an immediate offset, and thread t owns the window
// column (y, z) = (t / kFw, t % kFw) when staging, clearing and flushing.  A block whose
// extent exceeds kFw nodes along some axis takes a window sized to its extent (runtime
// pitches, at most kWindow entries), and beyond that works on global memory.  All forms
// perform the same arithmetic, so they give identical results.
constexpr int kFw = 16, kFwY = kFw, kFwX = kFw * kFw;

// base + a byte offset below 2^32: a wave-uniform base and a 32-bit per-lane offset map to
// the scalar-base form of the global memory instructions
template <typename P>
__device__ __forceinline__ P* byte_offset(P* base, unsigned bytes) {
  using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + bytes);
}
static_assert(kFw * kFw * kFw == kWindow, "fixed window = LDS window");
static_assert(kFw * kFw == kBlock, "one window column per thread");

// Block-wide extent of the cells j0 of the particles with in == true: lo (minima) and hi
// (maxima) per axis, as wave-uniform scalars; any is false when no particle of the block is
// in.  Must be called by all threads of the block.
struct CellRange {
  int lo[3], hi[3];
  bool any;
};

__device__ __forceinline__ CellRange block_cells(bool in, const int (&j0)[3], int* bounds) {
  block_bounds(in, j0, j0, bounds);
  CellRange r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = __builtin_amdgcn_readfirstlane(bounds[a]);
    r.hi[a] = __builtin_amdgcn_readfirstlane(bounds[3 + a]);
  }
  r.any = r.lo[0] <= r.hi[0] && r.lo[1] <= r.hi[1] && r.lo[2] <= r.hi[2];
  return r;
}


// Block-wide extent of the cells j0 (as block_cells) and the block-wide maximum of one int
// per thread (v), all wave-uniform.  Must be called by all threads of the block.
__device__ __forceinline__ CellRange block_cells_max(bool in, const int (&j0)[3], int v,
                                                     int* bounds, int& vmax) {
  block_bounds_max(in, j0, j0, v, bounds);
  CellRange r;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r.lo[a] = __builtin_amdgcn_readfirstlane(bounds[a]);
    r.hi[a] = __builtin_amdgcn_readfirstlane(bounds[3 + a]);
  }
  vmax = __builtin_amdgcn_readfirstlane(bounds[6]);
  r.any = r.lo[0] <= r.hi[0] && r.lo[1] <= r.hi[1] && r.lo[2] <= r.hi[2];
  return r;
}

}  // namespace
}  // namespace scola
