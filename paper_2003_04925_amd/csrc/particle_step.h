// Device code of the fused particle step (CiC deposit, gradient and CiC interpolation, COLA
// kick and drift) as a device function of one logical block (see kernels_particles.hip).
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "particle_common.h"

namespace scola {

namespace {


// Integer type of one particle's fixed-point corner weights: 64-bit for the 2^40 units of
// FP64 plans, 32-bit for the 2^21 units of FP32 plans.
template <typename T>
using WeightT = typename std::conditional<MeshFixed<T>::bits == 40, long long, int>::type;

template <typename T>
__device__ __forceinline__ void mesh_weights(double fx, double fy, double fz,
                                             WeightT<T> (&w)[8]) {
  if constexpr (MeshFixed<T>::bits == 40)
    split_weights<long long, double>(fx, fy, fz, 1ll << 40, w);
  else
    split_weights<int, float>((float)fx, (float)fy, (float)fz, 1 << MeshFixed<T>::bits, w);
}

// Corner range of one particle's CiC footprint restricted to interior nodes [1, n]:
// returns false when the particle deposits nothing (outside the box, or NaN).
__device__ inline bool deposit_footprint(int M, double ux, double uy, double uz, int (&j0)[3],
                                         double (&f)[3]) {
  const double hi = (double)M + 1.0;
  if (!(ux >= -1.0 && ux < hi && uy >= -1.0 && uy < hi && uz >= -1.0 && uz < hi))
    return false;
  const double u[3] = {ux, uy, uz};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double fl = floor(u[c]);
    j0[c] = (int)fl;
    f[c] = u[c] - fl;
  }
  return true;
}


// B^sCOLA for the 256 particles of one block (one Lagrangian brick): CiC of every particle
// onto interior nodes [1, M-1]^3 of its box, privatised in an LDS window that covers the
// block's Eulerian footprint, then one global atomic per touched interior node.  Integer
// sums make every window form give identical results.  The block's packed cell extent is
// stored at hint_out (words 0-2) for the force pass at the same positions.  The mass a
// particle drops is one unit minus what it keeps (the eight weights sum to exactly one
// unit).  FP32 plans store the block's total (at most 256 x 2^21 units) in word 3 of
// hint_out, for the Poisson pass that consumes this deposit to fold into the box's counter,
// and return 0; FP64 plans store 0 there and return this thread's dropped mass.  Must be
// called by all threads of the block.
template <typename T>
__device__ __forceinline__ long long deposit_block(typename MeshFixed<T>::rho_t* __restrict__ rho, int M,
                                          bool active, double ux, double uy, double uz,
                                          typename MeshFixed<T>::window_t* win, int* bounds,
                                          uint4* hint_out) {
  using W = typename MeshFixed<T>::window_t;
  using Rho = typename MeshFixed<T>::rho_t;
  const int n = M - 1;
  int j0[3] = {0, 0, 0};
  double f[3] = {0, 0, 0};
  const bool in = active && deposit_footprint(M, ux, uy, uz, j0, f);
  WeightT<T> w[8];
  if (in) mesh_weights<T>(f[0], f[1], f[2], w);
  // which of the two corner planes along each axis are interior nodes
  bool inner[3][2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    inner[c][0] = j0[c] >= 1 && j0[c] <= n;
    inner[c][1] = j0[c] >= 0 && j0[c] <= n - 1;
  }
  WeightT<T> kept = 0;
  if (in) {
#pragma unroll
    for (int c = 0; c < 8; ++c)
      if (inner[0][(c >> 2) & 1] && inner[1][(c >> 1) & 1] && inner[2][c & 1]) kept += w[c];
  }
  long long dropped = active ? (1ll << MeshFixed<T>::bits) - (long long)kept : 0;
  constexpr bool kBlockDrop = MeshFixed<T>::bits < 32;
  if constexpr (kBlockDrop) {
    // the wave's dropped mass in the slot that block_cells leaves free (read after its
    // barrier): no atomics on the box's counter, whose word all blocks of the box share
    const unsigned d = wave_sum((unsigned)dropped);
    if ((threadIdx.x & 63) == 0) bounds[3 * kWaves + (threadIdx.x >> 6)] = (int)d;
    dropped = 0;
  }
  // the whole LDS window (every form below uses at most kWindow entries) is cleared before
  // the barrier of the extent reduction, which then also orders the clearing before the
  // accumulation; the caller's last use of the window ended at a barrier
  {
    // 16-byte stores (the window is 16-byte aligned and a multiple of kBlock x 16 bytes)
    constexpr int kClear = kWindow * (int)sizeof(W) / 16 / kBlock;
    static_assert(kClear * 16 * kBlock == kWindow * (int)sizeof(W), "whole window");
    uint4* const w4 = reinterpret_cast<uint4*>(win);
#pragma unroll
    for (int k = 0; k < kClear; ++k) w4[threadIdx.x + kBlock * k] = make_uint4(0u, 0u, 0u, 0u);
  }
  unsigned q[3];
  const CellRange cr = block_cells(in, j0, bounds, q);
  if (threadIdx.x == 0) {
    unsigned bd = 0u;
    if constexpr (kBlockDrop) {
#pragma unroll
      for (int w = 0; w < kWaves; ++w) bd += (unsigned)bounds[3 * kWaves + w];
    }
    *hint_out = make_uint4(q[0], q[1], q[2], bd);
  }
  if (!cr.any) return dropped;
  // the corners of the block's particles span [min j0, max j0 + 1] per axis
  const int ox = cr.lo[0], oy = cr.lo[1], oz = cr.lo[2];
  const int ex = cr.hi[0] - ox + 2, ey = cr.hi[1] - oy + 2, ez = cr.hi[2] - oz + 2;
  if (ex <= kFw && ey <= kFw && ez <= kFw) {
    const int t = threadIdx.x, ty = t / kFw, tz = t % kFw;
    if (in) {
      // all eight corners go to the window; only interior nodes are flushed
      W* wp = win + (j0[0] - ox) * kFwX + (j0[1] - oy) * kFwY + (j0[2] - oz);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        atomicAdd(wp + ((c >> 2) & 1) * kFwX + ((c >> 1) & 1) * kFwY + (c & 1), (W)w[c]);
    }
    __syncthreads();
    const int ny = oy + ty, nz = oz + tz;
    if (ty < ey && tz < ez && ny >= 1 && ny <= n && nz >= 1 && nz <= n) {
      const int xa = max(1 - ox, 0), xb = min(n + 1 - ox, ex);   // interior x planes
      const unsigned gcol = (unsigned)(((ny - 1) * n + (nz - 1)) * (int)sizeof(Rho));
      if constexpr (sizeof(Rho) == 4) {
        // 32-bit words: buffer atomics over the box's mesh, the plane a scalar offset; the
        // block-uniform plane range [xa, xb) in groups of four (reads first, then atomics),
        // so the planes beyond the block's extent cost nothing
        const __amdgpu_buffer_rsrc_t rs = buffer_of(rho, (unsigned)(n * n * n * (int)sizeof(Rho)));
        for (int x0 = xa; x0 < xb; x0 += 4) {
          Rho v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) v[u] = x0 + u < xb ? win[t + kFwX * (x0 + u)] : Rho(0);
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (v[u] != 0)
              __builtin_amdgcn_raw_ptr_buffer_atomic_add_i32(
                  (int)v[u], rs, gcol, (ox - 1 + x0 + u) * (n * n) * (int)sizeof(Rho), 0);
        }
      } else {
        Rho v[kFw];
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi)
          v[xi] = (xi >= xa && xi < xb) ? win[t + kFwX * xi] : Rho(0);
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi)
          if (v[xi] != 0)
            atomicAdd(byte_offset(rho + (int64_t)(ox - 1 + xi) * (n * n), gcol), v[xi]);
      }
    }
    return dropped;
  }
  // sized window over the interior nodes the block touches
  const int lx = max(ox, 1), ly = max(oy, 1), lz = max(oz, 1);
  const int hx = min(cr.hi[0] + 1, n), hy = min(cr.hi[1] + 1, n), hz = min(cr.hi[2] + 1, n);
  if (lx > hx || ly > hy || lz > hz) return dropped;   // no interior corner at all
  const int wx = hx - lx + 1, wy = hy - ly + 1, wz = hz - lz + 1;
  const int wyz = wy * wz, vol = wx * wyz;
  const bool use_lds = vol <= kWindow;
  if (in) {
    // window index of corner (0, 0, 0); interior corners add dx wyz + dy wz + dz
    const int base = ((j0[0] - lx) * wy + (j0[1] - ly)) * wz + (j0[2] - lz);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
      if (inner[0][dx] && inner[1][dy] && inner[2][dz] && w[c] != 0) {
        if (use_lds)
          atomicAdd(win + (base + dx * wyz + dy * wz + dz), (W)w[c]);
        else
          atomicAdd(rho + idx3(j0[0] + dx - 1, j0[1] + dy - 1, j0[2] + dz - 1, n, n), (Rho)w[c]);
      }
    }
  }
  if (use_lds) {
    __syncthreads();
    // flush: each thread takes a (y, z) column of the window and walks it along x
    const float inv_wz = 1.0f / (float)wz;
    const unsigned gstep = (unsigned)(n * n);
    for (int pos = threadIdx.x; pos < wyz; pos += blockDim.x) {
      const int ey2 = (int)(((float)pos + 0.5f) * inv_wz), ez2 = pos - ey2 * wz;
      unsigned widx = (unsigned)pos;
      unsigned gidx = idx3(lx - 1, ly + ey2 - 1, lz + ez2 - 1, n, n);
      for (int x = 0; x < wx; ++x, widx += (unsigned)wyz, gidx += gstep) {
        const Rho v = win[widx];
        if (v != 0) atomicAdd(rho + gidx, v);
      }
    }
  }
  return dropped;
}

// grad^sCOLA + B-bar^sCOLA at one particle: the central-difference gradient of the padded
// potential at the CiC corners j0 + {0, 1} that lie in [0, M] (others carry zero weight),
// interpolated with the weights fr.  `at(kx, ky, kz)` returns the potential at node
// j0 - 1 + k (k in 0..3 per axis; a finite stand-in where only zero weights use it).
// Along each axis, corner j0 differences nodes j0 + 1 and j0 - 1, corner j0 + 1 nodes
// j0 + 2 and j0: 32 distinct nodes for the three components.
template <typename T, typename At>
__device__ __forceinline__ void gather_force(int M, const int (&j0)[3], const T (&fr)[3], At at,
                                    T (&g)[3]) {
  T w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a][0] = j0[a] >= 0 ? T(1) - fr[a] : T(0);
    w[a][1] = j0[a] + 1 <= M ? fr[a] : T(0);
  }
  T gx = 0, gy = 0, gz = 0;
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      gx += w[1][p] * w[2][q] *
            (w[0][0] * (at(2, 1 + p, 1 + q) - at(0, 1 + p, 1 + q)) +
             w[0][1] * (at(3, 1 + p, 1 + q) - at(1, 1 + p, 1 + q)));
      gy += w[0][p] * w[2][q] *
            (w[1][0] * (at(1 + p, 2, 1 + q) - at(1 + p, 0, 1 + q)) +
             w[1][1] * (at(1 + p, 3, 1 + q) - at(1 + p, 1, 1 + q)));
      gz += w[0][p] * w[1][q] *
            (w[2][0] * (at(1 + p, 1 + q, 2) - at(1 + p, 1 + q, 0)) +
             w[2][1] * (at(1 + p, 1 + q, 3) - at(1 + p, 1 + q, 1)));
    }
  g[0] = T(0.5) * gx;
  g[1] = T(0.5) * gy;
  g[2] = T(0.5) * gz;
}

// gather_force with the four (p, q) lines of the stencil in a rolled loop: the same
// arithmetic in the same order, for the rarely taken sized-window and global-memory forms,
// which then hold few values in registers and do not set the kernel's register budget.
template <typename T, typename At>
__device__ __forceinline__ void gather_force_rolled(int M, const int (&j0)[3], const T (&fr)[3],
                                                 At at, T (&g)[3]) {
  T w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a][0] = j0[a] >= 0 ? T(1) - fr[a] : T(0);
    w[a][1] = j0[a] + 1 <= M ? fr[a] : T(0);
  }
  T gx = 0, gy = 0, gz = 0;
#pragma unroll 1
  for (int pq = 0; pq < 4; ++pq) {
    const int p = pq >> 1, q = pq & 1;
    const T wxp = p ? w[0][1] : w[0][0], wyp = p ? w[1][1] : w[1][0];
    const T wyq = q ? w[1][1] : w[1][0], wzq = q ? w[2][1] : w[2][0];
    gx += wyp * wzq *
          (w[0][0] * (at(2, 1 + p, 1 + q) - at(0, 1 + p, 1 + q)) +
           w[0][1] * (at(3, 1 + p, 1 + q) - at(1, 1 + p, 1 + q)));
    gy += wxp * wzq *
          (w[1][0] * (at(1 + p, 2, 1 + q) - at(1 + p, 0, 1 + q)) +
           w[1][1] * (at(1 + p, 3, 1 + q) - at(1 + p, 1, 1 + q)));
    gz += wxp * wyq *
          (w[2][0] * (at(1 + p, 1 + q, 2) - at(1 + p, 1 + q, 0)) +
           w[2][1] * (at(1 + p, 1 + q, 3) - at(1 + p, 1 + q, 1)));
  }
  g[0] = T(0.5) * gx;
  g[1] = T(0.5) * gy;
  g[2] = T(0.5) * gz;
}

// Direct-to-LDS staging of the fixed potential window placed from a kept extent cr (FP32
// plans): for each of the window's x planes, every lane of a wave loads the potential at
// its window column (y, z) = (t / kFw, t % kFw), coordinates clamped into the padded grid,
// and the load itself writes the value to win[t + kFwX x] (the 64 lanes of a wave fill 64
// consecutive words, which is the window's layout).  No registers hold the values, so the
// loads can be issued before the block's particles arrive.  Nodes outside the padded grid
// (one layer at most) get finite stand-ins that only zero-weight corners read.  Returns
// false, having issued nothing, for FP64 plans and for extents beyond the fixed window.
template <typename T>
__device__ __forceinline__ bool stage_window_direct(const T* __restrict__ phi, int M,
                                                    const CellRange& cr, T* win) {
  if constexpr (sizeof(T) != 4) {
    return false;
  } else {
    const int ox = cr.lo[0] - 1, oy = cr.lo[1] - 1, oz = cr.lo[2] - 1;
    const int ex = cr.hi[0] - ox + 3, ey = cr.hi[1] - oy + 3, ez = cr.hi[2] - oz + 3;
    if (!(cr.any && ex <= kFw && ey <= kFw && ez <= kFw)) return false;
    const int Mp = M + 3, Mp2 = Mp * Mp;
    const int t = threadIdx.x, ty = t / kFw, tz = t % kFw;
    if (ty < ey && tz < ez) {
      const int ny = min(max(oy + ty, -1), M + 1), nz = min(max(oz + tz, -1), M + 1);
      const unsigned gcol = (unsigned)(((ny + 1) * Mp + (nz + 1)) * (int)sizeof(T));
      // the wave's first window word, a wave-uniform value held in a scalar register (the
      // LDS destination of these loads is a scalar base)
      T* const wave_base = win + __builtin_amdgcn_readfirstlane(t & ~63);
      // the box's padded potential as a buffer: plane nx + 1 is a scalar offset, the column
      // the lane's 32-bit offset
      const __amdgpu_buffer_rsrc_t rs = buffer_of(phi, (unsigned)(Mp2 * Mp * (int)sizeof(T)));
#pragma unroll
      for (int xi = 0; xi < kFw; ++xi)
        if (xi < ex) {
          const int nx = min(max(ox + xi, -1), M + 1);
          __builtin_amdgcn_raw_ptr_buffer_load_lds(
              rs, (__attribute__((address_space(3))) void*)(wave_base + kFwX * xi), 4, gcol,
              (nx + 1) * Mp2 * (int)sizeof(T), 0, 0);
        }
    }
    return true;
  }
}

// Force at u for the 256 particles of a block: the potential nodes the block's stencils
// touch are staged once in LDS (each thread loads window columns along x) and gathered
// from there; a block whose footprint exceeds the sized window gathers from global
// memory.  The window is placed from the block's cell extent.  With `hinted`, the extent
// hc kept by the deposit of the same positions is checked (every particle's cell inside
// it, one vote per wave) and used in place of the reduction; `staged` says that the fixed
// window placed from hc is already on its way into LDS (stage_window_direct).  A stale
// hint fails the check, and the block reduces its extent and stages as usual.  Any window
// that covers every stencil gives the same force, so the hint changes no result.  Must be
// called by all threads of the block.
template <typename T>
__device__ __forceinline__ void block_force(const T* __restrict__ phi, int M, double ux, double uy,
                                   double uz, T* win, int* bounds, bool hinted,
                                   const CellRange& hc, bool staged, T (&g)[3]) {
  g[0] = g[1] = g[2] = T(0);
  const double hiu = (double)M + 1.0;
  const bool in = ux >= -1.0 && ux < hiu && uy >= -1.0 && uy < hiu && uz >= -1.0 && uz < hiu;
  const double u[3] = {ux, uy, uz};
  int j0[3] = {0, 0, 0};
  T fr[3] = {T(0), T(0), T(0)};
  if (in) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double fl = floor(u[a]);
      j0[a] = (int)fl;
      fr[a] = (T)(u[a] - fl);
    }
  }
  const int Mp = M + 3, Mp2 = Mp * Mp;
  CellRange cr = hc;
  bool held = false;
  if (hinted) {
    hint_to_slots(in, j0, cr, bounds);
    // the direct-to-LDS loads of this wave must have landed before the barrier releases the
    // other waves to read them: the barrier's workgroup fence does not wait for them
    if (staged) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    held = hint_holds(bounds);
  }
  if (!held) cr = block_cells(in, j0, bounds);
  if (cr.any) {
    // the stencils of the block's particles span [min j0 - 1, max j0 + 2] per axis
    const int ox = cr.lo[0] - 1, oy = cr.lo[1] - 1, oz = cr.lo[2] - 1;
    const int ex = cr.hi[0] - ox + 3, ey = cr.hi[1] - oy + 3, ez = cr.hi[2] - oz + 3;
    if (ex <= kFw && ey <= kFw && ez <= kFw) {
      if (!(held && staged)) {
        const int t = threadIdx.x, ty = t / kFw, tz = t % kFw;
        const int ny = oy + ty, nz = oz + tz;
        // window nodes outside the padded grid [-1, M+1] (one layer at most) are zero; only
        // zero-weight corners read them
        const bool col =
            ty < ey && tz < ez && ny >= -1 && ny <= M + 1 && nz >= -1 && nz <= M + 1;
        const int xa = max(-1 - ox, 0), xb = min(M + 2 - ox, ex);
        // all loads of the column are issued before the first LDS store
        const unsigned gcol = col ? (unsigned)(((ny + 1) * Mp + (nz + 1)) * (int)sizeof(T)) : 0u;
        T v[kFw];
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi) v[xi] = T(0);
        if (col) {
#pragma unroll
          for (int xi = 0; xi < kFw; ++xi)
            if (xi >= xa && xi < xb) v[xi] = *byte_offset(phi + (int64_t)(ox + 1 + xi) * Mp2, gcol);
        }
#pragma unroll
        for (int xi = 0; xi < kFw; ++xi)
          if (xi < ex) win[t + kFwX * xi] = v[xi];
        __syncthreads();
      }
      if (in) {
        const T* wp = win + (j0[0] - 1 - ox) * kFwX + (j0[1] - 1 - oy) * kFwY + (j0[2] - 1 - oz);
        gather_force<T>(M, j0, fr,
                        [&](int kx, int ky, int kz) { return wp[kx * kFwX + ky * kFwY + kz]; }, g);
      }
    } else if (ex * ey * ez <= kWindow) {
      // window sized to the extent, laid out like the fixed one with runtime pitches
      // (x: ey ez, y: ez): nodes outside the padded grid are zero, as in the fixed form, so
      // the stencil reads need no clamping
      const int eyz = ey * ez;
      const float inv_ez = 1.0f / (float)ez;
      for (int pos = threadIdx.x; pos < eyz; pos += blockDim.x) {
        const int ey2 = (int)(((float)pos + 0.5f) * inv_ez), ez2 = pos - ey2 * ez;
        const int ny = oy + ey2, nz = oz + ez2;
        const bool col = ny >= -1 && ny <= M + 1 && nz >= -1 && nz <= M + 1;
        const int xa = max(-1 - ox, 0), xb = col ? min(M + 2 - ox, ex) : 0;
        const int gcol = (ny + 1) * Mp + (nz + 1);
#pragma unroll 4
        for (int x = 0; x < ex; ++x)
          win[pos + x * eyz] = x >= xa && x < xb ? phi[(int64_t)(ox + 1 + x) * Mp2 + gcol] : T(0);
      }
      __syncthreads();
      if (in) {
        const T* wp = win + ((j0[0] - 1 - ox) * ey + (j0[1] - 1 - oy)) * ez + (j0[2] - 1 - oz);
        gather_force_rolled<T>(M, j0, fr, [&](int kx, int ky, int kz) {
          return wp[kx * eyz + ky * ez + kz];
        }, g);
      }
    } else if (in) {
      // global memory; stencil coordinates are clamped into [-1, M+1], which changes only
      // reads that carry zero weight
      auto cl = [&](int v) { return min(max(v, -1), M + 1); };
      gather_force_rolled<T>(M, j0, fr, [&](int kx, int ky, int kz) {
        return phi[idx3(cl(j0[0] - 1 + kx) + 1, cl(j0[1] - 1 + ky) + 1,
                        cl(j0[2] - 1 + kz) + 1, Mp, Mp)];
      }, g);
    }
  }
  __syncthreads();   // every thread is done with `bounds` and the window before reuse
}

// Weights c_k (k = 1..NG) of the central first difference of order 2 NG,
// sum_k c_k (f(i+k) - f(i-k)): (1/2), (2/3, -1/12), (3/4, -3/20, 1/60).
template <int NG>
__device__ __forceinline__ constexpr double grad_weight(int k) {
  return NG == 1 ? 0.5
       : NG == 2 ? (k == 1 ? 2.0 / 3.0 : -1.0 / 12.0)
                 : (k == 1 ? 0.75 : k == 2 ? -0.15 : 1.0 / 60.0);
}

// grad^sCOLA + B-bar^sCOLA at one particle with the gradient of order 2 NG (NG > 1): at each
// CiC corner c in [0, M] (others carry zero weight) the component along axis a is
// sum_k c_k (Phi(c + k e_a) - Phi(c - k e_a)); `at(kx, ky, kz)` returns the potential at
// node j0 - NG + k (k in 0..2 NG + 1 per axis; a finite stand-in where only zero weights
// use it).
template <typename T, int NG, typename At>
__device__ __forceinline__ void gather_force_wide(int M, const int (&j0)[3], const T (&fr)[3],
                                                  At at, T (&g)[3]) {
  T w[3][2];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w[a][0] = j0[a] >= 0 ? T(1) - fr[a] : T(0);
    w[a][1] = j0[a] + 1 <= M ? fr[a] : T(0);
  }
  T gx = 0, gy = 0, gz = 0;
#pragma unroll 1
  for (int c = 0; c < 8; ++c) {
    const int dx = (c >> 2) & 1, dy = (c >> 1) & 1, dz = c & 1;
    const T wc = w[0][dx] * w[1][dy] * w[2][dz];
    const int X = NG + dx, Y = NG + dy, Z = NG + dz;
    T sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 1; k <= NG; ++k) {
      const T ck = (T)grad_weight<NG>(k);
      sx += ck * (at(X + k, Y, Z) - at(X - k, Y, Z));
      sy += ck * (at(X, Y + k, Z) - at(X, Y - k, Z));
      sz += ck * (at(X, Y, Z + k) - at(X, Y, Z - k));
    }
    gx += wc * sx;
    gy += wc * sy;
    gz += wc * sz;
  }
  g[0] = gx;
  g[1] = gy;
  g[2] = gz;
}

// Force at u for the 256 particles of a block at gradient order 2 NG (NG > 1) on the padded
// potential [-NG, M + NG]^3: the block's stencil nodes [min j0 - NG, max j0 + 1 + NG] are
// staged in an LDS window sized to that extent when it fits, else gathered from global
// memory; coordinates are clamped into the padded grid, which changes only reads that
// carry zero weight.  Must be called by all threads of the block.
template <typename T, int NG>
__device__ __forceinline__ void block_force_wide(const T* __restrict__ phi, int M, double ux,
                                                 double uy, double uz, T* win, int* bounds,
                                                 T (&g)[3]) {
  g[0] = g[1] = g[2] = T(0);
  const double hiu = (double)M + 1.0;
  const bool in = ux >= -1.0 && ux < hiu && uy >= -1.0 && uy < hiu && uz >= -1.0 && uz < hiu;
  const double u[3] = {ux, uy, uz};
  int j0[3] = {0, 0, 0};
  T fr[3] = {T(0), T(0), T(0)};
  if (in) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double fl = floor(u[a]);
      j0[a] = (int)fl;
      fr[a] = (T)(u[a] - fl);
    }
  }
  const int Mp = M + 1 + 2 * NG;
  auto cl = [&](int v) { return min(max(v, -NG), M + NG) + NG; };   // padded index
  const CellRange cr = block_cells(in, j0, bounds);
  if (cr.any) {
    const int ox = cr.lo[0] - NG, oy = cr.lo[1] - NG, oz = cr.lo[2] - NG;
    const int wx = cr.hi[0] - cr.lo[0] + 2 + 2 * NG, wy = cr.hi[1] - cr.lo[1] + 2 + 2 * NG,
              wz = cr.hi[2] - cr.lo[2] + 2 + 2 * NG;
    const int wyz = wy * wz;
    if (wx * wyz <= kWindow) {
      for (int pos = threadIdx.x; pos < wyz; pos += blockDim.x) {
        const int ey = pos / wz, ez = pos - ey * wz;
        const int64_t col = (int64_t)cl(oy + ey) * Mp + cl(oz + ez);
        for (int x = 0; x < wx; ++x) win[x * wyz + pos] = phi[(int64_t)cl(ox + x) * Mp * Mp + col];
      }
      __syncthreads();
      if (in) {
        const int bx = j0[0] - NG - ox, by = j0[1] - NG - oy, bz = j0[2] - NG - oz;
        gather_force_wide<T, NG>(M, j0, fr, [&](int kx, int ky, int kz) {
          return win[((bx + kx) * wy + by + ky) * wz + bz + kz];
        }, g);
      }
    } else if (in) {
      gather_force_wide<T, NG>(M, j0, fr, [&](int kx, int ky, int kz) {
        return phi[((int64_t)cl(j0[0] - NG + kx) * Mp + cl(j0[1] - NG + ky)) * Mp +
                   cl(j0[2] - NG + kz)];
      }, g);
    }
  }
  __syncthreads();   // every thread is done with `bounds` and the window before reuse
}

// The fused particle step of logical block L (< m.count): called by k_particles below and by
// the persistent step kernel.
template <typename T, int MODE, int NG = 1>
__device__ __forceinline__ void particles_block(const ParticleArgs<T>& a, const BlockMap& m,
                                                int L) {
  const int b = m.base + L;
  const int ti = m.tile[b];
  const TileDesc t = a.tiles[ti];
  const int M = t.M;
  const int local = m.local[b];          // the block's brick of 4 x 8 x 8 lattice sites
  const int tid = threadIdx.x;
  // the brick's first particle (block-uniform): every particle stream of the block is a
  // uniform base plus the thread's 32-bit offset, so the address arithmetic stays scalar
  const int64_t p0 = t.p_off + (int64_t)local * kBlock;
  const int64_t P = a.P;
  // the block's cell extent as the previous deposit of these positions left it
  uint4* const hint = a.cells + (t.p_off / kBlock + local);
  constexpr bool kForce = MODE != kDepositOnly && MODE != kInit;
  uint4 h = make_uint4(0u, 0u, 0u, 0u);
  // the kept extents place the fixed window of the order-2 gradient only
  const bool use_hints = NG == 1 && a.use_hints != 0;
  if (kForce && use_hints) h = *hint;
  // lattice site: the brick's corner from the uniform brick index, the thread's place in the
  // brick from its index (the layout of brick_site)
  const int nb = M >> 3;
  const int i = (local / (nb * nb)) * 4 + (tid >> 6);
  const int j = ((local / nb) % nb) * 8 + ((tid >> 3) & 7);
  const int k = (local % nb) * 8 + (tid & 7);
  const double q[3] = {i + 0.5, j + 0.5, k + 0.5};
  double s1[3], s2[3];
  T xr[3], pr[3];
  const T* ps1[3];
  const T* ps2[3];
  T* pxr[3];
  T* pxo[3];
  T* ppr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    ps1[c] = a.psi1 + (c * P + p0);
    ps2[c] = a.psi2 + (c * P + p0);
    pxr[c] = a.xres + (c * P + p0);
    pxo[c] = a.xout + (c * P + p0);
    ppr[c] = a.pres + (c * P + p0);
  }
  // the particle streams are touched once per step: non-temporal loads and stores keep
  // them from competing for cache lines with the box's mass mesh (the target of the
  // deposit's atomics) and potential, which neighbouring blocks reuse.  `fresh` (uniform):
  // L- leaves x_res = p_res = 0 unwritten and the first step takes them as zero
  const bool fresh = a.sc.fresh != 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s1[c] = (double)__builtin_nontemporal_load(ps1[c] + tid);
    s2[c] = (double)__builtin_nontemporal_load(ps2[c] + tid);
    if (MODE == kInit) {
      // operator L- (App. B): at t_0 the particles sit on their LPT trajectory and the
      // residual momentum is zero
      xr[c] = T(0);
      if (!fresh) {
        pxr[c][tid] = T(0);
        ppr[c][tid] = T(0);
      }
    } else {
      xr[c] = fresh ? T(0) : __builtin_nontemporal_load(pxr[c] + tid);
    }
  }
  // one LDS window, first for the potential (kWindow T values), then for the block's mass
  // (kWindow fixed-point accumulators)
  __shared__ __align__(16) unsigned long long win[kWindow * sizeof(T) / 8];
  __shared__ int bounds[kCellScratch];
  // the potential window placed from the kept extent is requested while the particle
  // streams are still in flight
  const bool hinted = kForce && use_hints;
  CellRange hc;
  bool staged = false;
  if (hinted) {
    const unsigned hq[3] = {(unsigned)__builtin_amdgcn_readfirstlane(h.x),
                            (unsigned)__builtin_amdgcn_readfirstlane(h.y),
                            (unsigned)__builtin_amdgcn_readfirstlane(h.z)};
    hc = cells_decode(hq);
    staged = stage_window_direct<T>(a.phi + t.h_off, M, hc, reinterpret_cast<T*>(win));
  }
  const StepScalars sc = a.sc;
  double u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u[c] = lpt_base(q[c], sc.D1, s1[c], sc.D2, s2[c]) + (double)xr[c];
  if (kForce) {
#pragma unroll
    for (int c = 0; c < 3; ++c) pr[c] = fresh ? T(0) : __builtin_nontemporal_load(ppr[c] + tid);
    // the LPT terms of the kick and of the next position are formed before the force, so
    // Psi1 and Psi2 are not held across it
    const double d2 = sc.D2 - sc.D1 * sc.D1;
    T lpt[3];
    double un[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lpt[c] = (T)(sc.D1 * s1[c] - d2 * s2[c]);
      un[c] = lpt_base(q[c], sc.D1n, s1[c], sc.D2n, s2[c]);
      // formed here: the compiler would otherwise sink them past the force and keep
      // Psi1, Psi2 and q alive across it
      asm volatile("" : "+v"(lpt[c]), "+v"(un[c]));
    }
    T g[3];
    if constexpr (NG == 1)
      block_force<T>(a.phi + t.h_off, M, u[0], u[1], u[2], reinterpret_cast<T*>(win), bounds,
                     hinted, hc, staged, g);
    else
      block_force_wide<T, NG>(a.phi + t.h_off, M, u[0], u[1], u[2], reinterpret_cast<T*>(win),
                              bounds, g);
#pragma unroll
    for (int c = 0; c < 3; ++c) pr[c] += (T)sc.beta * (g[c] - lpt[c]);
    if (MODE == kFinalKick) {
#pragma unroll
      for (int c = 0; c < 3; ++c) ppr[c][tid] = pr[c] + (T)(sc.c1 * s1[c] + sc.c2 * s2[c]);
      return;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xr[c] += (T)sc.alpha * pr[c];
      __builtin_nontemporal_store(xr[c], pxo[c] + tid);
      __builtin_nontemporal_store(pr[c], ppr[c] + tid);
    }
    if (MODE == kStepNoDeposit) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c] = un[c] + (double)xr[c];
  }
  if constexpr (MeshFixed<T>::bits < 32) {
    // FP32: the block's dropped mass travels in its hint (folded by the Poisson pass)
    deposit_block<T>(a.rho + t.g_off, M, true, u[0], u[1], u[2],
                     reinterpret_cast<typename MeshFixed<T>::window_t*>(win), bounds, hint);
  } else {
    __shared__ unsigned long long block_drop;
    if (threadIdx.x == 0) block_drop = 0ull;
    const long long drop =
        deposit_block<T>(a.rho + t.g_off, M, true, u[0], u[1], u[2],
                         reinterpret_cast<typename MeshFixed<T>::window_t*>(win), bounds, hint);
    // one atomic per block on the box's counter, which all blocks of the box share
    if (drop != 0) atomicAdd(&block_drop, (unsigned long long)drop);
    __syncthreads();
    if (threadIdx.x == 0 && block_drop != 0ull) atomicAdd(a.dropped + ti, block_drop);
  }
  // FP32 plans count the deposits of every box (its first block, once per launch) for the
  // mass identity that detects a wrapped 32-bit node (see the Poisson pass)
  if constexpr (MeshFixed<T>::bits < 32)
    if (threadIdx.x == 0 && local == 0) atomicAdd(a.deposits + ti, 1ull);
}

}  // namespace
}  // namespace scola
