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
  int ng = 1;               // finite differences of order 2 ng
};

struct BoxSetupArgs {
  const TileDesc* tiles;
  int n_tiles;
  const int* blk_tile;
  const int* blk_first;
  int n_blocks;
  const double* phi1;
  const double* phi2;
  void* psi1;               // [3][P] in the plan precision
  void* psi2;
  double* bc0;
  int N;                    // LPT grid nodes per side
  int64_t P;
  int ng = 1;               // finite differences of order 2 ng; Phi_BC^0 on [-ng, M+ng]^3
  int Np = 0;               // lattice particles per side (a multiple of N)
};

template <typename T>
struct MeshArgs {
  const TileDesc* tiles;
  typename MeshFixed<T>::rho_t* rho;   // fixed-point mass
  unsigned long long* alarm;           // count of FP32-plan node visits finding >= 2^31 units
  unsigned long long* kept;            // FP32 plans: per tile, the mass the passes found
  // FP32 plans: the per-tile dropped mass, and the particle bricks' hints (four words per
  // brick of 256 particles), whose word 3 holds the mass the brick's last deposit dropped
  // until the pass consuming that deposit folds it into `dropped` and clears it
  unsigned long long* dropped;
  unsigned* hints;
  T* work;
  T* phi;
  const double* bc0;
  const void* twiddles;     // complex T, per M: 2M entries W_{2M}^m
  const T* eigen;           // per M: lambda_l, l = 1..M-1 (FDA of the plan order, unit spacing)
  // FP32 plans, per M: the DST-I sine matrix S[j][k] = sin(pi (j+1)(k+1) / M), j, k < M - 1,
  // as FP16 halves hi then lo (M rows of 32 ceil(M / 32) values each, zero-padded)
  const void* sine;
  double D1_bc;
  // order 2, forward solves of an evolution: bit 1, the third pass leaves each interior x
  // plane's boundary-source perimeter terms (the first pass's sums of Phi_BC^0 at the
  // face-layer neighbours, FP64) at the start of that plane of `work`, which it has
  // consumed; bit 0, the first pass of the next solve reads them there (one contiguous run)
  // instead of gathering them from Phi_BC^0, whose z-face values lie one per cache line
  int bc_handoff = 0;
  // adjoint solve only: the source is read from `work`, the result written to lam_rho, and
  // the boundary-source transpose accumulated into lam_bc0
  T* lam_rho = nullptr;
  double* lam_bc0 = nullptr;
  // consistency tests of Sec. 4.3 (forward solve only): when set, the density contrast of
  // the interior nodes (ov_delta) and/or the potential of the face layers and the shell
  // (ov_phi, in place of D1_bc Phi_BC^0) are taken from full-box periodic fields [N^3] at
  // the nodes' global positions (box origin + node, wrapped)
  const T* ov_delta = nullptr;
  const T* ov_phi = nullptr;
  int ov_N = 0;
  int ng = 1;                          // ghost layers: finite differences of order 2 ng
};

template <typename T>
struct ParticleArgs {
  const TileDesc* tiles;
  const T* psi1;            // [3][P] in the plan precision
  const T* psi2;
  T* xres;
  T* xout;                  // x_res after the drift: xres itself, or another buffer
  T* pres;
  const T* phi;
  typename MeshFixed<T>::rho_t* rho;
  unsigned long long* dropped;
  unsigned long long* deposits;   // FP32 plans: deposits per tile (for the mass identity)
  // per brick of 256 particles: the packed cell extent of its last deposit (words 0-2),
  // written by every depositing launch and, with use_hints, tried by the force pass before
  // it reduces the extent itself (a stale entry costs time, never a result); word 3 holds,
  // in FP32 plans, the mass the deposit dropped until the Poisson pass folds it
  uint4* cells;
  int use_hints;
  int64_t P;
  StepScalars sc;
  int ng = 1;               // ghost layers of the padded potential (gradient of order 2 ng)
};

template <typename T>
struct OutputArgs {
  const TileDesc* tiles;
  const T* psi1;            // [3][P] in the plan precision
  const T* psi2;
  const T* xres;
  const T* pres;
  T* pos;
  T* mom;
  unsigned long long* grid;
  int64_t P;
  int Np, N_out;
  double D1, D2, cell, L;
};

// Arrays and scalars of one reverse step (or of the output transpose).
template <typename T>
struct AdjointArgs {
  const TileDesc* tiles;
  const T* psi1;            // [3][P] in the plan precision
  const T* psi2;
  T* lam_x;                 // adjoint of x_res, [3][P]
  T* lam_p;                 // adjoint of p_res, [3][P]
  T* lam_psi1;              // accumulated adjoint of Psi1, [3][P] (plan precision)
  T* lam_psi2;              // accumulated adjoint of Psi2, [3][P]
  int64_t P, H;
  // gather half: force positions of step g (x_res at that time), its potential and the
  // adjoint of its deposited mass; lam_g = beta_g lam_p
  const T* xg;
  const T* phi;             // [H]
  const T* lam_rho;         // [G]
  double beta_g, D1g, D2g;
  // scatter half: kick/drift coefficients of step k and its force positions; the
  // transposed interpolation lands in `work` (interior nodes, zeroed) and lam_bc0 (shell)
  const T* xs;
  T* work;                  // [G]
  double* lam_bc0;          // [H]
  double alpha, beta, D1, D2;
};

enum ParticleMode { kDepositOnly = 0, kStep = 1, kStepNoDeposit = 2, kFinalKick = 3, kInit = 4 };

hipError_t launch_setup_potentials(const SetupArgs& a, hipStream_t s);
template <typename T>
hipError_t launch_setup_boxes(const BoxSetupArgs& a, T* xres, T* pres, hipStream_t s);

// One size class (all blocks of the maps belong to boxes with this M).  adjoint: solve
// Delta lam = work with zero boundary values (the Dirichlet operator is symmetric), write
// lam_rho, and add -D1_bc C^T lam to lam_bc0 (C maps face values onto the first interior
// layer in delta' = delta - Delta Phi_BCs).
template <typename T>
hipError_t launch_poisson(const MeshArgs<T>& a, int M, const BlockMap& p1, const BlockMap& p2,
                          const BlockMap& p3, hipStream_t s, bool adjoint = false);
template <typename T>
// occ: waves per SIMD the kernel's registers are held to (6 or 8)
hipError_t launch_particles(const ParticleArgs<T>& a, int mode, const BlockMap& m, int occ,
                            hipStream_t s);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_zero_u32(unsigned* p, int64_t n, hipStream_t s);
// Folds word 3 of the bricks' hints (FP32 deposits' dropped mass) of tiles [0, n_tiles)
// into dropped[tile] and clears it: for a deposit that no Poisson pass consumes.
hipError_t launch_fold_drops(const TileDesc* tiles, int n_tiles, unsigned* hints,
                             unsigned long long* dropped, hipStream_t s);
template <typename T>
hipError_t launch_output(const OutputArgs<T>& a, const BlockMap& m, bool density,
                         T* density_out, hipStream_t s);

template <typename T>
hipError_t launch_adj_output(const AdjointArgs<T>& a, const BlockMap& m, const T* lam_dens,
                             int Np, int N_out, hipStream_t s);
// One fused particle pass of the reverse sweep: the gather half of step g (after that
// step's adjoint Poisson solve) and/or the scatter half of step k = g - 1.
template <typename T>
hipError_t launch_adj_step(const AdjointArgs<T>& a, const BlockMap& part, bool gather,
                           bool scatter, hipStream_t s);
template <typename T>
hipError_t launch_adj_setup_scatter(const BoxSetupArgs& b, const T* lam_psi1,
                                    const T* lam_psi2, double* lam_psig,
                                    const double* lam_bc0, double* lam_phi1, hipStream_t s);
hipError_t launch_adj_phi_from_psi(const double* lam_psig, double* lam_phi1, double2* cbuf,
                                   int N, hipStream_t s);
hipError_t launch_adj_source(const double* phi1, const double* lam_s, double* f6,
                             double* lam_phi1, int N, hipStream_t s);
hipError_t launch_real_to_complex(const double* in, double2* out, int64_t n, hipStream_t s);
// FP64 set-up pieces reused by the adjoint
hipError_t fft3d_forward(double2* c, int N, hipStream_t s);
hipError_t fft3d_inverse(double2* c, int N, hipStream_t s);
hipError_t launch_ic_filter(const SetupArgs& a, hipStream_t s);
hipError_t launch_inverse_laplacian(double2* c, int N, int ng, hipStream_t s);
hipError_t launch_take_real(const double2* c, double* out, double scale, int64_t n, hipStream_t s);

// Monolithic periodic tCOLA of the full box (N^3 particles in lattice order, [3][N^3]
// component arrays, a periodic N^3 node grid).
template <typename T>
struct TcolaArgs {
  const T* psi1;            // [3][N^3] in the plan precision
  const T* psi2;
  T* xres;
  T* pres;
  unsigned long long* rho;   // [N^3] fixed-point mass, 2^40 units per particle
  const T* phi;              // [N^3] periodic potential
  int N;
  StepScalars sc;
  int ng = 1;               // finite differences of order 2 ng
};

template <typename T>
hipError_t launch_tcola_setup(const TcolaArgs<T>& a, const double* phi1, const double* phi2,
                              hipStream_t s);
template <typename T>
hipError_t launch_tcola_particles(const TcolaArgs<T>& a, int mode, hipStream_t s);
// rec_delta / rec_phi: optional N^3 arrays receiving this solve's delta and potential
template <typename T>
hipError_t launch_tcola_poisson(const TcolaArgs<T>& a, double2* cbuf, T* phi, T* rec_delta,
                                T* rec_phi, hipStream_t s);
template <typename T>
hipError_t launch_tcola_output(const TcolaArgs<T>& a, T* pos, T* mom, unsigned long long* grid,
                               T* density, int N_out, double cell, double L, hipStream_t s);

// One KDK step of one box class (kStep particle pass + the next force's Poisson passes) as
// one persistent cooperative launch (FP32 plans).  barrier: two device words, the arrival
// counter (cleared by the launcher) and a sticky flag set if a bounded barrier wait gave
// up; grid_out receives the grid size used.
template <typename T>
hipError_t launch_step_persistent(const ParticleArgs<T>& pa, const MeshArgs<T>& ma, int M,
                                  const BlockMap& mp, const BlockMap& m1, const BlockMap& m2,
                                  const BlockMap& m3, unsigned* barrier, hipStream_t s,
                                  int* grid_out);

constexpr int kPencilChunk = 32;       // z-columns per block of the x-pencil pass (FFT)
constexpr int kPencilChunkMfma = 64;   // the same for FP32 plans (matrix-core pass)
template <typename T>
__host__ __device__ constexpr int pencil_chunk() {
  return sizeof(T) == 4 ? kPencilChunkMfma : kPencilChunk;
}

}  // namespace scola
