/*
 * scola.h -- C ABI of the MI355X tiled-sCOLA engine (libscola.so).
 *
 * Method: Leclercq et al., "Perfectly parallel cosmological simulations using spatial
 * comoving Lagrangian acceleration" (arXiv:2003.04925).  A periodic cube of side L holding
 * N_p^3 particles on a Lagrangian lattice is split into cubic tiles (Sec. 3.2, B.1); every
 * tile plus a buffer of particles forms an sCOLA box that is evolved on its own through
 * COLA kick-drift steps (Sec. 3.4, App. A-B) with a Dirichlet Poisson solver by DST-I whose
 * boundary potential is the linearly evolving full-box LPT potential (Sec. 3.4.2 eq. LEP,
 * App. C).  The core particles' final positions and momenta and their CiC density are the
 * outputs (Sec. 3.2, B.2).
 *
 * Conventions shared by every entry point
 *  - Every call returns scola_status (0 = SCOLA_OK, < 0 = error).  On error nothing has been
 *    launched unless stated otherwise, and scola_last_error() holds a message (per thread).
 *  - Pointers named d_* are device pointers (HIP, the device current when the plan was
 *    created).  The caller owns them and every workspace; the plan owns its host tables
 *    and a few small device tables (tile table, block maps, twiddles, eigenvalues).
 *  - Work is enqueued on the given stream and is asynchronous; the call returns once it is
 *    enqueued.  Calls on one plan must not overlap in time (the plan holds the step state).
 *  - 3-D arrays are C order [x][y][z] (z fastest).  Component arrays are [3][n].
 *  - Lengths inside the workspace are in lattice cells (Delta q = L / N_p); outputs are in
 *    Mpc/h.  Time is the scale factor a; H0 = 1.
 *  - Box layout: a box of M = core_n + 2 buffer particles per side holds its particles at
 *    local positions i + 1/2; PM nodes sit at integer local positions, the Dirichlet problem
 *    has M - 1 unknowns per side and the potential is padded to [-g, M+g], g = N_ghost =
 *    fda_order / 2 (Sec. 3: 1, 2, 3 at finite-difference order 2, 4, 6).  M is one of 16,
 *    32, 48, ..., 128 (see scola_tile).
 */
#ifndef SCOLA_H
#define SCOLA_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SCOLA_OK = 0,
  SCOLA_EINVAL = -1,       /* an argument is out of range or inconsistent */
  SCOLA_ENOMEM = -2,       /* host or plan-owned device allocation failed */
  SCOLA_EDEVICE = -3,      /* a HIP call failed (launch, copy, event) */
  SCOLA_ESTATE = -4,       /* call order violated (e.g. evolve before setup) */
  SCOLA_EUNSUPPORTED = -5, /* valid request outside what the library implements */
  SCOLA_EOVERFLOW = -6     /* a fixed-point mesh value left its range (see scola_mass_alarm) */
} scola_status;

enum { SCOLA_FP32 = 0, SCOLA_FP64 = 1 };           /* particle/mesh arithmetic */
enum { SCOLA_BATCHED = 0, SCOLA_PER_TILE = 1 };    /* all tiles per launch, or one tile */
enum { SCOLA_MODIFIED = 0, SCOLA_STANDARD = 1 };   /* COLA time factors of App. B */

/* Flat LambdaCDM (Sec. 4: Planck 2015 values; Omega_L = 1 - Omega_m). */
typedef struct {
  double Omega_m, Omega_b, h, n_s, sigma8, T_cmb;
} scola_cosmology;

/* One tile (Sec. 3.2, B.1): core particles [core_lo, core_lo + core_n) per axis of the
 * global lattice (indices, wrapped mod N_p), surrounded by `buffer` particles per side.
 * mesh[a]: PM cells per side of the box's mesh along axis a (Sec. 3.2 B.1: N_g).  0 means
 * M = core_n + 2 buffer, the particles per side of the box, which is the only mesh the
 * library implements (the PM node spacing then equals the lattice spacing); any other value
 * is refused with SCOLA_EUNSUPPORTED.
 * Admitted box sizes: M = 16 R for R = 1..8, i.e. {16, 32, 48, 64, 80, 96, 112, 128}: the
 * particles of a box are stored in bricks of 4 x 8 x 8, and every 1-D sine transform of the
 * Poisson solve is a product with 16-row sine-matrix tiles (FP32 plans) or an FFT of 16 R
 * points on 16 lanes (FP64 plans).  These are the members of
 * 2^a {1, 3, 5, 7} that are multiples of 16 up to 128; other sizes of that form (24, 40, 56,
 * 192, 256, ...) are refused with SCOLA_EUNSUPPORTED. */
typedef struct {
  int32_t core_lo[3];
  int32_t core_n;
  int32_t buffer;
  int32_t mesh[3];
  double a_f;              /* final scale factor of this tile (Sec. 5.1, light cones: tiles
                              need not share one final time): 0 -> cfg.a_f, else > a_i.  Each
                              tile takes cfg.n_steps steps linearly spaced from a_i to its a_f;
                              tiles of one box size and final time share launches.  The reverse
                              mode needs one final time for all tiles (else SCOLA_EUNSUPPORTED). */
} scola_tile;

/* Run parameters (Sec. 3, Sec. 4). */
typedef struct {
  double L;                /* box side, Mpc/h, > 0 */
  int32_t Np;              /* particles per side; power of two in [8, 1024] */
  int32_t N_lpt;           /* LPT grid nodes per side (Sec. 3.1, A.1: N): 0 -> N_p (the nodes
                              coincide with the particles), or a power-of-two divisor of N_p of
                              at least 8, e.g. N_p / 2 as in Sec. 4 (node m at the cell centre
                              (m + 1/2) L / N; Psi differenced on the grid and interpolated by
                              CiC to the particles, Sec. 3.3 C.2; Phi_BC^0 interpolated by CiC
                              to the PM nodes); anything else SCOLA_EINVAL.  The white noise
                              lives on this grid.  scola_backward and scola_tcola_forward are
                              built for N_lpt = N_p (SCOLA_EUNSUPPORTED otherwise) */
  int32_t N_out;           /* output density grid per side (0 -> N_p) */
  int32_t fda_order;       /* finite-difference order of every Laplacian and gradient (Sec. 3;
                              App. C.1-C.2): 2, 4 or 6 (0 -> 2, the order of Sec. 4's runs),
                              else SCOLA_EINVAL.  Order 2 g uses g ghost layers: Phi_BCs on the
                              g layers outside the interior, the potential padded by g.  At
                              orders 4 and 6 the sine transform solves the wide stencil with
                              the unknown continued antisymmetrically past each face, as
                              App. C.2's eigenvalues imply.  scola_backward and the persistent
                              step are built for order 2 (SCOLA_EUNSUPPORTED otherwise) */
  int32_t n_steps;         /* KDK steps, linearly spaced in a (Sec. 4), >= 1 */
  double a_i, a_f;         /* initial / final scale factor, 0 < a_i < a_f */
  double n_lpt;            /* exponent of u(a) = a^n_LPT in the modified time factors (App. B);
                              0 -> -2.5, the paper's value; must be finite */
  int32_t discretisation;  /* SCOLA_MODIFIED (App. B, modified time factors with n_lpt) or
                              SCOLA_STANDARD (App. B eq. alpha-beta-standard: integrals of
                              the drift and kick prefactors) */
  int32_t precision;       /* SCOLA_FP32 or SCOLA_FP64 */
  int32_t schedule;        /* SCOLA_BATCHED or SCOLA_PER_TILE */
  int32_t want_momenta;    /* nonzero: evaluate the last force and apply the final half
                              kick and L+ (App. B) so momenta are available */
  int32_t checkpoint_every;/* 0: forward only.  c > 0: the forward stores (x_res, p_res)
                              before steps 0, c, 2c, ... and scola_backward is available
                              (it recomputes each segment of c steps) */
} scola_config;

typedef struct scola_plan scola_plan;

/* Byte offsets of the arrays held in the caller's workspace (for inspection and for
 * operator-level calls).  P = total box particles, G = sum (M-1)^3, H = sum (M+1+2g)^3
 * (g = fda_order / 2), N = N_p, R = real type of the plan (float or double). */
typedef struct {
  size_t psi1, psi2;       /* R [3][P]: Psi1 = grad phi1, Psi2 = grad phi2 (cells), differenced
                              in FP64 and stored in the plan precision R */
  size_t x_res, p_res;     /* R [3][P]: COLA residual position and momentum (cells) */
  size_t rho;              /* fixed-point CiC mass, 2^fixed_bits units per particle: int64 [G]
                              (FP64 plans) or uint32 [G] (FP32 plans; a node holds at most
                              2048 particles, see `dropped`); size rounded up to 8 bytes */
  size_t work;             /* R [G]: sine-space scratch of the Poisson solve */
  size_t phi;              /* R [H]: potential on the padded node grid [-g, M+g]^3 */
  size_t bc0;              /* double [H]: Phi_BC^0 (LEP boundary potential at D1 = 1) */
  size_t dropped;          /* int64 [3 n_tiles + 1], counters since the last reset: the
                              fixed-point mass dropped by the deposits, per tile; the number of
                              node visits by the Poisson pass that found >= 2^31 units on an
                              FP32-plan node (1024 particles, within a factor 2 of the 32-bit
                              range); then, FP32 plans only, per tile the mass the Poisson
                              passes found and per tile the number of deposits (mass identity:
                              found + dropped = deposits x M^3 x 2^21 units unless a node's
                              32-bit mass wrapped, which loses exactly 2^32 units).
                              scola_evolve and scola_op_deposit reset all; scola_mass_alarm
                              evaluates them. */
  size_t cells;            /* uint32 [P / 256][4]: per brick of 256 particles (lattice order
                              within a box), words 0-2: the block cell extent of its last
                              deposit, packed; the force pass of the next step tries it before
                              reducing the extent itself.  Any content there is valid: a stale
                              entry costs time and changes no result.  Word 3, FP32 plans: the
                              mass the brick's last deposit dropped, which the Poisson pass
                              consuming that deposit (within scola_op_deposit and
                              scola_op_step, the call itself) adds to `dropped` and clears; it
                              is 0 between calls, and a value written there is counted as
                              dropped mass by the next Poisson pass. */
  size_t phi1, phi2;       /* double [N^3]: Lagrangian potentials (Sec. 3.1, A.2) */
  size_t cbuf;             /* double2 [N^3]: FFT scratch */
  size_t outgrid;          /* int64 [N_out^3]: fixed-point output density */
  /* reverse mode (all 0 when cfg.checkpoint_every == 0); c = checkpoint_every */
  size_t ckpt;             /* R [ceil(n_steps/c)][6][P]: (x_res, p_res) before steps 0, c, ... */
  size_t seg_x;            /* R [c+1][3][P]: ring of x_res per step (slot = step mod (c+1))
                              for the segment being reversed and the first step after it */
  size_t seg_phi;          /* R [c+1][H]: ring of the potentials of the same steps */
  size_t lam_x, lam_p;     /* R [3][P]: adjoints of x_res and p_res */
  size_t lam_psi1, lam_psi2; /* R [3][P]: accumulated adjoints of Psi1, Psi2 */
  size_t lam_rho;          /* R [G]: adjoint of the deposited mass */
  size_t lam_bc0;          /* double [H]: accumulated adjoint of Phi_BC^0 */
  size_t adj_grid;         /* double [14][N^3]: set-up adjoint fields */
  size_t total;            /* workspace size in bytes */
  int64_t n_particles;     /* P */
  int64_t n_nodes;         /* G */
  int64_t n_padded;        /* H */
  int32_t fixed_bits;      /* one particle's mass in rho: 2^40 (FP64 plans) or 2^21 (FP32) */
} scola_layout;

#define SCOLA_FIXED_BITS 40  /* output-density CiC weights are accumulated as round(w 2^40) */

/* Fill out[0 .. tiles_per_side^3) with the uniform tiling of Sec. 3.2 (B.1): cores of
 * N_p / tiles_per_side particles, order x-major.  Np must be a multiple of tiles_per_side.
 * capacity = number of elements of out. */
scola_status scola_uniform_tiling(int32_t Np, int32_t tiles_per_side, int32_t buffer,
                                  scola_tile* out, int32_t capacity);

/* Validate the configuration and build a plan: host FP64 scalars (growth factors D1, D2
 * of App. A eqs. VD1/VD2 normalised to D1(a_i) = 1; modified time factors of App. B with
 * n_LPT = -2.5; sigma_8 normalisation of the Eisenstein-Hu no-wiggle spectrum) and the
 * device tile table.  The tiles must cover the lattice exactly once.  *out receives the
 * plan (NULL on error).  The current HIP device becomes the plan's device. */
scola_status scola_plan_create(const scola_config* cfg, const scola_cosmology* cosmo,
                               const scola_tile* tiles, int32_t n_tiles, scola_plan** out);

scola_status scola_plan_destroy(scola_plan* plan);

/* Bytes of device workspace the caller must provide (256-byte aligned base). */
scola_status scola_workspace_size(const scola_plan* plan, size_t* bytes);
scola_status scola_workspace_layout(const scola_plan* plan, scola_layout* out);

/* The whole run: scola_setup, scola_evolve, scola_output.  tile_subset (host array of
 * n_subset tile indices, or NULL for all) restricts the evolution and outputs to those
 * tiles (Sec. 5.1, node failures: any tile can be recomputed alone, with bitwise the same
 * result as in the full run); other tiles' output entries are left untouched and the
 * density is not produced (d_density must then be NULL).
 * d_white_noise: double [N_lpt^3] unit white noise on the LPT grid (Sec. 3.1, A.1).
 * d_pos: R [3][N_p^3] final positions in [0, L) Mpc/h at the global lattice index.
 * d_mom: R [3][N_p^3] final momenta p = dx/da / drift_prefactor (Mpc/h, H0 = 1), or NULL;
 *        requires cfg.want_momenta.
 * d_density: R [N_out^3] CiC density contrast of the core particles (Sec. 4.1), or NULL. */
scola_status scola_forward(scola_plan* plan, const double* d_white_noise, void* d_pos,
                           void* d_mom, void* d_density, const int32_t* tile_subset,
                           int32_t n_subset, void* d_workspace, hipStream_t stream);

/* Size of the library's static device workspace (per GPU) used by scola_forward_noalloc. */
#define SCOLA_STATIC_WORKSPACE_BYTES (128u << 20)

/* scola_forward for callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): the same set-up, evolution and outputs
 * over all tiles, with the workspace taken from a static device array of the library
 * (SCOLA_STATIC_WORKSPACE_BYTES = 128 MiB per GPU, held from the first call on a GPU until
 * the process ends) instead of the caller's.  The call allocates nothing (no hipMalloc,
 * stream, event or graph): it runs eagerly on `stream` with one box group.  Outputs are as
 * for scola_forward with tile_subset = NULL.
 * Errors: SCOLA_EINVAL if the plan's workspace (scola_workspace_size) exceeds the static
 * size, if white noise is NULL, if d_mom is given without cfg.want_momenta, or if the
 * current device is not the plan's.  Every call on a GPU uses that GPU's one static array
 * and overwrites what the previous call left there, so calls that overlap in time on one
 * GPU (on different streams or from different threads or plans) race and must be
 * serialised by the caller.  The reverse mode is not available from this workspace, and
 * the call-order state of caller workspaces is left as it was. */
scola_status scola_forward_noalloc(scola_plan* plan, const double* d_white_noise, void* d_pos,
                                   void* d_mom, void* d_density, hipStream_t stream);

/* Reverse mode of scola_forward for a loss on the output density: given d loss / d delta_out
 * (R [N_out^3], device), writes d loss / d white noise (double [N_lpt^3], device).  Needs a
 * plan with checkpoint_every > 0 and a preceding scola_forward over all tiles on the same
 * workspace (else SCOLA_ESTATE).  Segments of checkpoint_every steps are recomputed from
 * the checkpoints, then reversed step by step: transpose of the drift and kick, of the
 * gradient-then-CiC-interpolation chain (one scalar scatter per particle onto the padded
 * nodes), the same Dirichlet DST solve (the FDA-2 Dirichlet Laplacian is symmetric) and of
 * the deposit; finally the FP64 transposes of Phi_BC^0, Psi = D phi, the second-order
 * source and the initial-condition filter.
 * The particle state left in the workspace afterwards is that of the first segment;
 * run scola_evolve again before scola_output. */
scola_status scola_backward(scola_plan* plan, const void* d_grad_density,
                            double* d_grad_white_noise, void* d_workspace,
                            hipStream_t stream);

/* Steps A.1-A.2 and C.1-C.3 (Sec. 3.1, 3.3) in FP64: white noise -> delta_i via the
 * Eisenstein-Hu spectrum (convolution approach), phi1 and phi2 with the FDA kernel,
 * Psi1 and Psi2 for every box particle and Phi_BC^0 on every box's padded shell.  Also
 * resets x_res = p_res = 0 (operator L-, App. B). */
scola_status scola_setup(scola_plan* plan, const double* d_white_noise, void* d_workspace,
                         hipStream_t stream);

/* Step D (Sec. 3.4): the KDK operator E~ of App. B for every tile of tile_subset (NULL =
 * all), starting with L- (x_res = p_res = 0 at a_i), so it can be repeated on the state
 * left by scola_setup.  With cfg.want_momenta the final half kick and L+ are applied and
 * p_res then holds the full momentum p. */
scola_status scola_evolve(scola_plan* plan, const int32_t* tile_subset, int32_t n_subset,
                          void* d_workspace, hipStream_t stream);

/* The consistency tests of Sec. 4.3 (eqs. test_setup1-4): scola_evolve over all tiles in
 * which the density contrast of every box's interior nodes (d_delta) and/or the potential
 * of its face layers and shell (d_phi, in place of the linearly evolving D1 Phi_BC^0) are
 * taken at every force evaluation from full-box periodic fields, such as the record of
 * scola_tcola_forward: R [n_force][N_p^3], evaluation k at t_k, read at the nodes' global
 * positions (box origin + node, wrapped).  Either pointer may be NULL (both NULL is the
 * method itself, eq. test_setup1).  With both, every box reproduces the periodic tCOLA run
 * in its core to round-off (eq. test_setup4).  Runs eagerly on `stream` with one box group;
 * needs scola_setup on the workspace (else SCOLA_ESTATE). */
scola_status scola_evolve_overrides(scola_plan* plan, const void* d_delta, const void* d_phi,
                                    void* d_workspace, hipStream_t stream);

/* Launch schedule (not a quantity of the paper; results are bitwise identical under every
 * schedule).  Boxes are grouped into classes of equal size M and final scale factor
 * (ascending M); every class has its own launches of the fused particle kernel and of the
 * Poisson passes.  Per class:
 *   waves_per_simd       6 or 8: register budget the fused particle kernel is compiled for
 *                        (6 = 80 registers, 8 = 64; FP64 plans need more than 64 and run
 *                        at the occupancy their registers allow);
 *   xcd_remap_particles  1: blocks numbered so each of the 8 XCDs takes a contiguous run of
 *                        whole boxes (their meshes stay in one L2); 0: hardware order;
 *   xcd_remap_mesh       the same for the three Poisson passes.
 * Defaults {6, 1, 1}.  scola_plan_tune times the choices per class on the workspace's
 * particles (after scola_setup, else SCOLA_ESTATE) with `reps` launches each (1..1000) and
 * keeps the fastest; it leaves the set-up fields (Psi, Phi_BC^0) untouched, clears its
 * deposits, and synchronises the stream (call it before scola_evolve, never inside a timed
 * or captured region).  Its timed evolutions leave x_res and p_res at the end of an
 * evolution; scola_evolve starts from L- whatever they hold, so runs after tuning are
 * bitwise those without it.  scola_plan_schedule copies the schedule of every class into out (capacity
 * entries at least; out may be NULL to query *n_classes).  scola_plan_set_schedule sets it
 * (same classes, same order). */
typedef struct {
  int32_t M;
  int32_t waves_per_simd;
  int32_t xcd_remap_particles;
  int32_t xcd_remap_mesh;
} scola_class_schedule;

scola_status scola_plan_tune(scola_plan* plan, void* d_workspace, hipStream_t stream,
                             int32_t reps);
/* Concurrent box groups of the batched evolution (1, 2 or 4, default 1): with G > 1, the
 * tiles of every size class are split in G equal shares that advance at the same time, one
 * on `stream` and the others on plan-owned streams that fork from and join back to `stream`
 * with events, so one share's Poisson passes overlap another share's particle kernel.
 * Results are bitwise independent of G.  scola_plan_tune also chooses G, together with
 * waves_per_simd (one value for all classes) and whether the Poisson numbering chosen per
 * class is kept or flipped in every class, by timing whole evolutions each way (a choice
 * that is fastest for one kernel alone can lose when the groups share the GPU). */
scola_status scola_plan_concurrency(const scola_plan* plan, int32_t* groups);
scola_status scola_plan_set_concurrency(scola_plan* plan, int32_t groups);
scola_status scola_plan_schedule(const scola_plan* plan, scola_class_schedule* out,
                                 int32_t capacity, int32_t* n_classes);
scola_status scola_plan_set_schedule(scola_plan* plan, const scola_class_schedule* in,
                                     int32_t n_classes);

/* hipGraph replay of scola_evolve (enabled by default).  With the batched schedule over all
 * tiles, the second call of scola_evolve on a workspace records the whole evolution (every
 * kernel launch and checkpoint copy) as one graph on a plan-owned capture stream, and that
 * and every later call launch the graph on `stream`.  The graph is rebuilt after a change
 * of workspace or schedule.  enable = 0 drops it and runs every call eagerly. */
scola_status scola_plan_set_graph(scola_plan* plan, int32_t enable);

/* One persistent launch per KDK step (the batching pattern of a single fused launch per
 * step): with enable != 0, every step of the batched evolution that deposits runs, per
 * class, the fused particle step of all bricks and the three Poisson passes of the next
 * force in ONE cooperative launch whose grid is the number of workgroups resident at once,
 * the phases separated by grid-wide barriers (bounded waits; a cooperative launch fails
 * rather than oversubscribe, so no wait can deadlock).  Results are bitwise those of the
 * default schedule.  Runs eagerly (no hipGraph) on one box group; FP32 batched plans only
 * (SCOLA_EUNSUPPORTED for FP64, SCOLA_EINVAL for the per-tile schedule).  It is slower than
 * the default (the kernel carries the register and LDS needs of its heaviest phase into all
 * of them), so the default is off.
 * scola_plan_persistent reports the setting, the grid of the last persistent launch and the
 * sticky count of barrier waits that gave up (always 0 unless something is wrong); it
 * synchronises `stream`. */
scola_status scola_plan_set_persistent(scola_plan* plan, int32_t enable);
scola_status scola_plan_persistent(const scola_plan* plan, hipStream_t stream, int32_t* enabled,
                                   int32_t* grid, int32_t* barrier_failures);

/* Step B.2 (Sec. 3.2): core particles' positions/momenta to global lattice order, and the
 * periodic CiC density of the core particles on N_out^3 nodes (all tiles must have been
 * evolved for the density).  Any output pointer may be NULL. */
scola_status scola_output(scola_plan* plan, void* d_pos, void* d_mom, void* d_density,
                          const int32_t* tile_subset, int32_t n_subset,
                          void* d_workspace, hipStream_t stream);

/* Operator-level entry points on the workspace state (used by the parity tests; the
 * forward pass is built from the same kernels).
 *
 * scola_op_deposit: B^sCOLA (Sec. 3.4.1) -- clears rho and deposits every box particle at
 *   u = q - D1 Psi1 + D2 Psi2 + x_res onto interior nodes [1, M-1]^3; mass that would land
 *   elsewhere is dropped and counted in `dropped`.
 * scola_op_poisson: App. C -- delta = rho / 2^fixed_bits - 1, delta' = delta - Delta Phi_BCs with
 *   Phi_BCs = D1_bc Phi_BC^0, forward DST-I, division by the FDA eigenvalues, inverse
 *   DST-I; writes phi on [-g, M+g]^3 with the shell set to D1_bc Phi_BC^0 (Sec. 3.4.2).
 *   rho is left zeroed for the next deposit.
 * scola_op_step: one fused kick-drift (App. B eqs. K_COLA, D_COLA with the sCOLA kick of
 *   App. A eq. kick-scola): gradient of phi and CiC interpolation at
 *   u = q - D1 Psi1 + D2 Psi2 + x_res, p_res += beta (g - D1 Psi1 + (D2 - D1^2) Psi2),
 *   x_res += alpha p_res, then (if deposit) deposit at u' = q - D1n Psi1 + D2n Psi2 +
 *   x_res into rho (which must be zero, as scola_op_poisson leaves it).
 * scola_op_final_kick: the last half kick (same as the kick above) followed by L+:
 *   p_res <- p_res + c1 Psi1 + c2 Psi2. */
scola_status scola_op_deposit(scola_plan* plan, double D1, double D2, void* d_workspace,
                              hipStream_t stream);
scola_status scola_op_poisson(scola_plan* plan, double D1_bc, void* d_workspace,
                              hipStream_t stream);
scola_status scola_op_step(scola_plan* plan, double beta, double alpha, double D1, double D2,
                           double D1n, double D2n, int32_t deposit, void* d_workspace,
                           hipStream_t stream);
scola_status scola_op_final_kick(scola_plan* plan, double beta, double D1, double D2,
                                 double c1, double c2, void* d_workspace, hipStream_t stream);

/* Host FP64 scalar tables of the plan.
 * scola_step_table: n_steps rows of 8 doubles
 *   {a_D, beta, alpha, D1(a_D), D2(a_D), D1(a_next), D2(a_next), a_next}
 *   (App. B: step k kicks from t_{k-1/2} (t_0 for k = 0) to t_{k+1/2} with the force at
 *   t_k, then drifts from t_k to t_{k+1}); then one row for the final half kick
 *   {a_f, beta, D1, D2, c1, c2, 0, 0} with c1, c2 the L+ coefficients.
 *   rows_capacity >= n_steps + 1.
 * scola_power_spectrum: P_lin(k, a = 1) in (Mpc/h)^3 at the n given k (h/Mpc), host
 *   arrays, as used by scola_setup (before the growth scaling to a_i). */
scola_status scola_step_table(const scola_plan* plan, double* rows, int32_t rows_capacity);
scola_status scola_power_spectrum(const scola_plan* plan, const double* k, double* out,
                                  int32_t n);

/* Host-only versions of the two tables above, without a plan or a device (same numbers
 * as the plan computes): rows as in scola_step_table for cfg->n_steps steps; P_lin(k, 1). */
scola_status scola_schedule_table(const scola_config* cfg, const scola_cosmology* cosmo,
                                  double* rows, int32_t rows_capacity);
scola_status scola_linear_power(const scola_cosmology* cosmo, const double* k, double* out,
                                int32_t n);

/* Monolithic periodic tCOLA of the plan's full box (Sec. 2.2, App. A eqs. drift-cola and
 * kick-tcola, App. B): the N_p^3 particles evolved together with a periodic PM grid of N_p^3
 * nodes (one per lattice cell, at integer positions of the lattice coordinate whose particles
 * sit at i + 1/2), periodic CiC deposit and interpolation, the Poisson equation with the
 * plan's finite-difference order solved by FFT (FP64 transforms), the central-difference
 * gradient of the same order, and the plan's KDK schedule and
 * precision; the tiling of the plan is not used.  It is the reference of the sCOLA accuracy
 * study (Sec. 4.2) and the source of the true density and potential of the consistency tests
 * (Sec. 4.3).
 * d_workspace: at least scola_tcola_workspace_size bytes, 256-byte aligned (independent of
 *   the sCOLA workspace).
 * d_pos, d_mom, d_density: as for scola_forward (each may be NULL; d_mom needs
 *   cfg.want_momenta).
 * d_record_delta, d_record_phi: NULL, or R [n_force][N_p^3] arrays receiving the density
 *   contrast and the potential of every force evaluation, n_force = n_steps (+1 with
 *   cfg.want_momenta); evaluation k is at t_k, the first at a_i. */
scola_status scola_tcola_workspace_size(const scola_plan* plan, size_t* bytes);
scola_status scola_tcola_forward(scola_plan* plan, const double* d_white_noise, void* d_pos,
                                 void* d_mom, void* d_density, void* d_record_delta,
                                 void* d_record_phi, void* d_workspace, hipStream_t stream);

/* The mass alarm of the workspace (FP32 plans; always zero for FP64 plans, whose 64-bit
 * node masses cannot wrap): *near_limit = node visits that found at least 1024 particles'
 * mass on a node since the last reset, *wrapped = the number of times a node's 32-bit mass
 * wrapped (a node above 2048 particles), from the exact mass identity of every box (see
 * scola_layout.dropped).  Valid after scola_evolve / scola_forward, and after operator-level
 * calls in which every deposit was followed by scola_op_poisson (otherwise SCOLA_ESTATE).
 * Synchronises `stream` (the counters are copied to the host after the work enqueued so
 * far).  Returns SCOLA_EOVERFLOW, with the counts written and a message, when *wrapped > 0:
 * the densities and forces of that run are invalid.  Either output pointer may be NULL. */
scola_status scola_mass_alarm(const scola_plan* plan, const void* d_workspace,
                              hipStream_t stream, int64_t* near_limit, int64_t* wrapped);

/* Diagnostics of the plan: number of tiles, total box particles, r and p (Sec. 3.2). */
scola_status scola_plan_info(const scola_plan* plan, int32_t* n_tiles, int64_t* n_particles,
                             double* oversimulation_r, double* parallel_p);

const char* scola_status_string(scola_status s);
const char* scola_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCOLA_H */
