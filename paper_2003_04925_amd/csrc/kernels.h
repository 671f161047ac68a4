// Launch interfaces of the tiled-sCOLA kernels (host side of the HIP library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

namespace scola {

// Block map of one batched launch: block b works on tile blk_tile[b], local unit
// blk_local[b] (a particle block of 256, a plane, or a pencil chunk).  Blocks of one tile
// are contiguous, so a per-tile launch is a sub-range [base, base + count).
struct BlockMap {
  const int* tile = nullptr;
  const int* local = nullptr;
  int base = 0;
  int count = 0;
  int xcd_remap = 1;       // spread consecutive logical blocks over one XCD (see kernels)
};

struct SetupArgs {
  const double* white_noise;
  double2* cbuf;
  double* phi1;
  double* phi2;
  int N;
  double L, amplitude, ns, Om, Ob, h, Tcmb, growth2;
};

struct BoxSetupArgs {
  const TileDesc* tiles;
  int n_tiles;
  const int* blk_tile;
  const int* blk_first;
  int n_blocks;
  const double* phi1;
  const double* phi2;
  double* psi1;
  double* psi2;
  double* bc0;
  int N;
  int64_t P;
};

template <typename T>
struct MeshArgs {
  const TileDesc* tiles;
  unsigned long long* rho;  // fixed-point mass (int64 two's complement)
  T* work;
  T* phi;
  const double* bc0;
  const void* twiddles;     // complex T, per M: 2M entries W_{2M}^m
  const T* eigen;           // per M: lambda_l, l = 1..M-1 (FDA-2, unit spacing)
  double D1_bc;
};

template <typename T>
struct ParticleArgs {
  const TileDesc* tiles;
  const double* psi1;
  const double* psi2;
  T* xres;
  T* pres;
  const T* phi;
  unsigned long long* rho;
  unsigned long long* dropped;
  int64_t P;
  StepScalars sc;
};

template <typename T>
struct OutputArgs {
  const TileDesc* tiles;
  const double* psi1;
  const double* psi2;
  const T* xres;
  const T* pres;
  T* pos;
  T* mom;
  unsigned long long* grid;
  int64_t P;
  int Np, N_out;
  double D1, D2, cell, L;
};

enum ParticleMode { kDepositOnly = 0, kStep = 1, kStepNoDeposit = 2, kFinalKick = 3, kInit = 4 };

hipError_t launch_setup_potentials(const SetupArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_setup_boxes(const BoxSetupArgs& a, T* xres, T* pres, hipStream_t s);

// One size class (all blocks of the maps belong to boxes with this M).
template <typename T>
hipError_t launch_poisson(const MeshArgs<T>& a, int M, const BlockMap& p1, const BlockMap& p2,
                          const BlockMap& p3, hipStream_t s);
template <typename T>
hipError_t launch_particles(const ParticleArgs<T>& a, int mode, const BlockMap& m,
                            hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_output(const OutputArgs<T>& a, const BlockMap& m, bool density,
                         T* density_out, hipStream_t s);

constexpr int kPencilChunk = 32;   // z-columns per block of the x-pencil pass

}  // namespace scola
