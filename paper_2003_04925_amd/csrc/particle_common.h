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

// Wave-wide sum of an unsigned value (no wrap-around assumed), uniform across the wave.
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
  v += (unsigned)lane_xor<1>((int)v);
  v += (unsigned)lane_xor<2>((int)v);
  v += (unsigned)lane_xor<4>((int)v);
  v += (unsigned)lane_xor<8>((int)v);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
         __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
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

// LPT part of a particle's FP64 box coordinate (App. B): q - D1 Psi1 + D2 Psi2 for the
// lattice coordinate q; the residual displacement is added to the result.  The two fused
// multiply-adds are written out, so every kernel that forms the position of a particle at
// the same growth factors gets the same bits, and hence the same cell.
__device__ __forceinline__ double lpt_base(double q, double D1, double s1, double D2, double s2) {
  return fma(D2, s2, fma(-D1, s1, q));
}

// Row-major index (a * nb + b) * nc + c of a 3-D array with fewer than 2^24 entries and
// non-negative coordinates, with full-rate 24-bit multiplies.
__device__ __forceinline__ unsigned idx3(int a, int b, int c, int nb, int nc) {
  return __umul24(__umul24((unsigned)a, (unsigned)nb) + (unsigned)b, (unsigned)nc) + (unsigned)c;
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
// A raw buffer resource over `bytes` bytes at p (stride 0; word 3 = 32-bit data format, the
// gfx9 value).  Buffer loads and atomics address base + SGPR offset + 32-bit VGPR offset, so
// a block-uniform row offset costs no vector instruction, and accesses at or beyond `bytes`
// are discarded by the hardware (loads return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_of(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           0x00020000);
}

static_assert(kFw * kFw * kFw == kWindow, "fixed window = LDS window");
static_assert(kFw * kFw == kBlock, "one window column per thread");

// Block-wide extent of the cells j0 of the particles with in == true: lo (minima) and hi
// (maxima) per axis, as wave-uniform scalars; any is false when no particle of the block is
// in.  The six extrema travel as three packed pairs of 16-bit minima, j0 + 2^14 and
// 2^14 - j0 (cells lie in [-16383, 16383]; 0xffff marks "none"): each wave reduces its
// lanes with DPP exchanges and stores its three words in its own slot of `scratch`, and
// after one barrier every thread combines the slots of all waves.  No LDS atomics and no
// initialisation pass are needed.  Must be called by all threads of the block; `scratch`
// holds kCellScratch ints, and its previous contents must have been read before a barrier
// that precedes this call.
constexpr int kWaves = kBlock / 64;
constexpr int kCellScratch = 4 * kWaves;

struct CellRange {
  int lo[3], hi[3];
  bool any;
};

__device__ __forceinline__ void cells_to_slots(bool in, const int (&j0)[3], unsigned* s) {
  constexpr int kOff = 1 << 14;
  const unsigned none = 0xffffffffu;
  const unsigned p0 = in ? (unsigned)(j0[0] + kOff) | ((unsigned)(j0[1] + kOff) << 16) : none;
  const unsigned p1 = in ? (unsigned)(j0[2] + kOff) | ((unsigned)(kOff - j0[0]) << 16) : none;
  const unsigned p2 = in ? (unsigned)(kOff - j0[1]) | ((unsigned)(kOff - j0[2]) << 16) : none;
  const unsigned r0 = wave_min_u16x2(p0), r1 = wave_min_u16x2(p1), r2 = wave_min_u16x2(p2);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s[wv] = r0;
    s[kWaves + wv] = r1;
    s[2 * kWaves + wv] = r2;
  }
}

// Decodes the three packed words of cells_to_slots (after the block-wide minimum) into a
// CellRange; words 0xffffffff (no particle) give any == false.
__device__ __forceinline__ CellRange cells_decode(const unsigned (&q)[3]) {
  constexpr int kOff = 1 << 14;
  CellRange r;
  r.lo[0] = (int)(q[0] & 0xffffu) - kOff;
  r.lo[1] = (int)(q[0] >> 16) - kOff;
  r.lo[2] = (int)(q[1] & 0xffffu) - kOff;
  r.hi[0] = kOff - (int)(q[1] >> 16);
  r.hi[1] = kOff - (int)(q[2] & 0xffffu);
  r.hi[2] = kOff - (int)(q[2] >> 16);
  r.any = r.lo[0] <= r.hi[0] && r.lo[1] <= r.hi[1] && r.lo[2] <= r.hi[2];
  return r;
}

// Block-wide packed words from the wave slots, uniform across the block.
__device__ __forceinline__ void cells_from_slots(const unsigned* s, unsigned (&q)[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    unsigned m = s[i * kWaves];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) m = pk_min_u16(m, s[i * kWaves + w]);
    q[i] = __builtin_amdgcn_readfirstlane(m);
  }
}

// q receives the packed words of the extent, the form in which it is kept between launches.
__device__ __forceinline__ CellRange block_cells(bool in, const int (&j0)[3], int* scratch,
                                                 unsigned (&q)[3]) {
  unsigned* s = reinterpret_cast<unsigned*>(scratch);
  cells_to_slots(in, j0, s);
  __syncthreads();
  cells_from_slots(s, q);
  return cells_decode(q);
}

__device__ __forceinline__ CellRange block_cells(bool in, const int (&j0)[3], int* scratch) {
  unsigned q[3];
  return block_cells(in, j0, scratch, q);
}

// A block extent kept from an earlier launch and used in place of block_cells: each wave
// stores in slot 3 kWaves + wave whether every in-particle of the wave has its cell inside
// `cr`; after a barrier, hint_holds() tells every thread whether all waves agreed.
__device__ __forceinline__ void hint_to_slots(bool in, const int (&j0)[3], const CellRange& cr,
                                              int* scratch) {
  const bool ok = !in || (j0[0] >= cr.lo[0] && j0[0] <= cr.hi[0] && j0[1] >= cr.lo[1] &&
                          j0[1] <= cr.hi[1] && j0[2] >= cr.lo[2] && j0[2] <= cr.hi[2]);
  const int all = __all(ok);
  if ((threadIdx.x & 63) == 0) scratch[3 * kWaves + (threadIdx.x >> 6)] = all;
}

__device__ __forceinline__ bool hint_holds(const int* scratch) {
  int a = scratch[3 * kWaves];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) a &= scratch[3 * kWaves + w];
  return __builtin_amdgcn_readfirstlane(a) != 0;
}

// block_cells and the block-wide maximum of one int per thread (v), wave-uniform.
__device__ __forceinline__ CellRange block_cells_max(bool in, const int (&j0)[3], int v,
                                                     int* scratch, int& vmax) {
  unsigned* s = reinterpret_cast<unsigned*>(scratch);
  cells_to_slots(in, j0, s);
  const int m = wave_max(v);
  if ((threadIdx.x & 63) == 0) scratch[3 * kWaves + (threadIdx.x >> 6)] = m;
  __syncthreads();
  int mm = scratch[3 * kWaves];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) mm = max(mm, scratch[3 * kWaves + w]);
  vmax = __builtin_amdgcn_readfirstlane(mm);
  unsigned q[3];
  cells_from_slots(s, q);
  return cells_decode(q);
}

// Fixed-point CiC weights of the 8 corners (offset bits x = 4, y = 2, z = 1) of a particle
// at fractional offsets (fx, fy, fz), as integers of type I with `one` units per particle.
// The unit is split along x into round(fx one) and the rest, each of the two parts along y
// the same way, and each of the four parts along z.  Every split is exact in integers, so
// the eight weights are non-negative and sum to exactly one unit, with no remainder to
// place; each is within three units of its exact value.  F is the floating type the products
// are formed in (float for 2^21 units, double for 2^40): the integers stay below 2^24 and
// 2^53, and adding one half before truncation rounds the non-negative products.
template <typename I, typename F>
__device__ __forceinline__ void split_weights(F fx, F fy, F fz, I one, I (&w)[8]) {
  const I x1 = (I)fma(fx, (F)one, F(0.5));
  const I x[2] = {one - x1, x1};
  I xy[4];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const I hi = (I)fma(fy, (F)x[q], F(0.5));
    xy[2 * q] = x[q] - hi;
    xy[2 * q + 1] = hi;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const I hi = (I)fma(fz, (F)xy[q], F(0.5));
    w[2 * q] = xy[q] - hi;
    w[2 * q + 1] = hi;
  }
}

}  // namespace
}  // namespace scola
