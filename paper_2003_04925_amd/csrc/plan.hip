// C ABI of the tiled-sCOLA engine: plan construction (validation, host FP64 scalar tables,
// device tile table and block maps), workspace layout, and the orchestration of the set-up,
// the KDK step loop and the outputs.  See include/scola.h for the contract.
#include "scola.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "host_math.h"
#include "kernels.h"

using namespace scola;

namespace {

thread_local std::string g_last_error;

struct ScolaError : std::runtime_error {
  scola_status code;
  ScolaError(scola_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] void fail(scola_status c, const std::string& m) { throw ScolaError(c, m); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess)
    fail(SCOLA_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

template <typename F>
scola_status guarded(F f) {
  try {
    f();
    return SCOLA_OK;
  } catch (const ScolaError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return SCOLA_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return SCOLA_EINVAL;
  }
}

// Block maps of one kernel family over all tiles.  Tiles are laid out class by class
// (classes of equal box size M and final scale factor, in increasing M), so every class is
// one contiguous block range.
struct Maps {
  std::vector<int> tile, local;
  std::vector<int> first;    // per tile: first block of that tile
  std::vector<int> count;    // per tile: number of blocks
  std::vector<int> class_M, class_tc, class_first, class_count;
  int* d_tile = nullptr;
  int* d_local = nullptr;
};

}  // namespace

// KDK scalars of one final scale factor (Sec. 5.1: tiles need not share one final time).
struct TimeClass {
  double a_f = 0.0;
  std::vector<double> table;          // (n_steps + 1) x 8 scalar rows
  std::vector<double> D1, D2;         // growth at t_0 .. t_n
};

struct scola_plan {
  scola_config cfg{};
  scola_cosmology cosmo{};
  std::vector<scola_tile> tiles;
  std::vector<TileDesc> desc;
  Background bg;
  int device = 0;
  int max_M = 0;
  int64_t P = 0, G = 0, H = 0;
  std::vector<double> table;          // (n_steps + 1) x 8 scalar rows of cfg.a_f
  std::vector<double> D1, D2;         // growth at t_0 .. t_n of cfg.a_f
  std::vector<TimeClass> tclasses;    // [0]: cfg.a_f; then every other tile final time
  scola_layout lay{};
  TileDesc* d_tiles = nullptr;
  void* d_twiddles = nullptr;
  void* d_eigen = nullptr;
  void* d_sine = nullptr;      // FP32 plans: split sine matrices of the matrix-core DST
  Maps part, p1, p2, p3;
  // launch schedule per size class (index as part.class_M), chosen by scola_plan_tune
  std::vector<scola_class_schedule> sched;
  std::vector<std::vector<int>> class_tiles;   // tiles of each size class, in map order
  // concurrent box groups of the batched evolution: 1, 2 or 4 (the tiles of every class
  // split in equal shares, advanced on the caller's stream and on aux streams at once)
  int groups = 1;
  hipStream_t aux_stream[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
  uint64_t sched_version = 0;         // bumped whenever the schedule changes
  // the batched evolution over all tiles, captured once per workspace and schedule (from
  // the second call on) and replayed as one hipGraph launch
  bool use_graph = true;
  hipStream_t capture_stream = nullptr;
  hipGraph_t evolve_graph = nullptr;
  hipGraphExec_t evolve_exec = nullptr;
  const void* graph_ws = nullptr;
  uint64_t graph_version = 0;
  int graph_eager_calls = 0;
  bool is64 = false;
  int ng = 1;                         // ghost layers: finite differences of order 2 ng
  int N_lpt = 0;                      // LPT grid nodes per side (Np or a divisor of it)
  // one persistent cooperative launch per KDK step and class instead of four launches
  bool persistent = false;
  unsigned* d_barrier = nullptr;      // arrival counter + sticky failure flag
  int persistent_grid = 0;
  // call-order state, keyed by the workspace it refers to
  const void* setup_ws = nullptr;
  const void* forward_ws = nullptr;   // full forward with checkpoints done on this workspace
};

namespace {

void build_maps(Maps& m, const std::vector<TileDesc>& desc,
                const std::function<int(const TileDesc&)>& units) {
  m.tile.clear();
  m.local.clear();
  m.class_M.clear();
  m.class_tc.clear();
  m.class_first.clear();
  m.class_count.clear();
  m.first.assign(desc.size(), 0);
  m.count.assign(desc.size(), 0);
  std::vector<std::pair<int, int>> keys;   // (M, time class)
  for (auto& d : desc) keys.push_back({d.M, d.tclass});
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  for (const auto& key : keys) {
    const int M = key.first;
    m.class_M.push_back(M);
    m.class_tc.push_back(key.second);
    m.class_first.push_back((int)m.tile.size());
    for (size_t t = 0; t < desc.size(); ++t) {
      if (desc[t].M != M || desc[t].tclass != key.second) continue;
      const int n = units(desc[t]);
      m.first[t] = (int)m.tile.size();
      m.count[t] = n;
      for (int i = 0; i < n; ++i) {
        m.tile.push_back((int)t);
        m.local.push_back(i);
      }
    }
    m.class_count.push_back((int)m.tile.size() - m.class_first.back());
  }
}

void upload_maps(Maps& m) {
  const size_t n = std::max<size_t>(1, m.tile.size());
  hip_check(hipMalloc(&m.d_tile, n * sizeof(int)), "hipMalloc(block map)");
  hip_check(hipMalloc(&m.d_local, n * sizeof(int)), "hipMalloc(block map)");
  if (!m.tile.empty()) {
    hip_check(hipMemcpy(m.d_tile, m.tile.data(), m.tile.size() * sizeof(int),
                        hipMemcpyHostToDevice), "hipMemcpy(block map)");
    hip_check(hipMemcpy(m.d_local, m.local.data(), m.local.size() * sizeof(int),
                        hipMemcpyHostToDevice), "hipMemcpy(block map)");
  }
}

void free_maps(Maps& m) {
  if (m.d_tile) hipFree(m.d_tile);
  if (m.d_local) hipFree(m.d_local);
  m.d_tile = m.d_local = nullptr;
}

BlockMap full_map(const Maps& m) {
  BlockMap b;
  b.tile = m.d_tile;
  b.local = m.d_local;
  b.base = 0;
  b.count = (int)m.tile.size();
  return b;
}

BlockMap tile_map(const Maps& m, int t) {
  BlockMap b;
  b.tile = m.d_tile;
  b.local = m.d_local;
  b.base = m.first[t];
  b.count = m.count[t];
  return b;
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

void validate(const scola_config& c, const scola_cosmology& cs, const scola_tile* tiles,
              int n_tiles) {
  if (!(c.L > 0)) fail(SCOLA_EINVAL, "L must be > 0");
  if (!is_pow2(c.Np) || c.Np < 8 || c.Np > 1024)
    fail(SCOLA_EINVAL, "Np must be a power of two in [8, 1024]");
  if (c.N_out < 0 || c.N_out > 2048) fail(SCOLA_EINVAL, "N_out must be in [0, 2048]");
  if (c.n_steps < 1) fail(SCOLA_EINVAL, "n_steps must be >= 1");
  if (!(c.a_i > 0 && c.a_i < c.a_f)) fail(SCOLA_EINVAL, "need 0 < a_i < a_f");
  if (c.precision != SCOLA_FP32 && c.precision != SCOLA_FP64)
    fail(SCOLA_EINVAL, "precision must be SCOLA_FP32 or SCOLA_FP64");
  if (c.schedule != SCOLA_BATCHED && c.schedule != SCOLA_PER_TILE)
    fail(SCOLA_EINVAL, "schedule must be SCOLA_BATCHED or SCOLA_PER_TILE");
  if (c.checkpoint_every < 0) fail(SCOLA_EINVAL, "checkpoint_every must be >= 0");
  if (c.N_lpt != 0 && c.N_lpt != c.Np) {
    // a coarser LPT grid: a power-of-two divisor of Np (its FFTs are radix 2) of >= 8 nodes
    if (!(c.N_lpt >= 8 && c.N_lpt < c.Np && is_pow2(c.N_lpt) && c.Np % c.N_lpt == 0))
      fail(SCOLA_EINVAL, "N_lpt must be 0, Np or a power-of-two divisor of Np of at least 8");
  }
  if (c.fda_order != 0 && c.fda_order != 2 && c.fda_order != 4 && c.fda_order != 6)
    fail(SCOLA_EINVAL, "fda_order must be 0, 2, 4 or 6");
  if (!std::isfinite(c.n_lpt)) fail(SCOLA_EINVAL, "n_lpt must be finite");
  if (c.discretisation != SCOLA_MODIFIED && c.discretisation != SCOLA_STANDARD)
    fail(SCOLA_EINVAL, "discretisation must be SCOLA_MODIFIED or SCOLA_STANDARD");
  if (!(cs.Omega_m > 0 && cs.Omega_m <= 1 && cs.Omega_b >= 0 && cs.Omega_b < cs.Omega_m &&
        cs.h > 0 && cs.sigma8 > 0 && cs.T_cmb > 0))
    fail(SCOLA_EINVAL, "cosmology out of range");
  if (!tiles || n_tiles < 1) fail(SCOLA_EINVAL, "need at least one tile");
  const int Np = c.Np;
  std::vector<uint8_t> cover((size_t)Np * Np * Np, 0);
  for (int t = 0; t < n_tiles; ++t) {
    const scola_tile& s = tiles[t];
    const int M = s.core_n + 2 * s.buffer;
    if (s.core_n < 1 || s.buffer < 0) fail(SCOLA_EINVAL, "tile core_n >= 1, buffer >= 0");
    if (M % 16 != 0 || M < 16 || M > kMaxM)
      fail(SCOLA_EUNSUPPORTED, "tile " + std::to_string(t) + ": M = core_n + 2 buffer = " +
                                   std::to_string(M) + " must be one of 16, 32, 48, ..., 128");
    if (s.a_f != 0.0 && !(std::isfinite(s.a_f) && s.a_f > c.a_i))
      fail(SCOLA_EINVAL, "tile " + std::to_string(t) + ": a_f must be 0 (the run's a_f) or > a_i");
    for (int a = 0; a < 3; ++a) {
      if (s.mesh[a] < 0) fail(SCOLA_EINVAL, "tile " + std::to_string(t) + ": mesh must be >= 0");
      if (s.mesh[a] != 0 && s.mesh[a] != M)
        fail(SCOLA_EUNSUPPORTED, "tile " + std::to_string(t) + ": mesh[" + std::to_string(a) +
                                     "] = " + std::to_string(s.mesh[a]) +
                                     ": only a mesh of M = core_n + 2 buffer cells per side "
                                     "(node spacing = lattice spacing) is implemented");
    }
    if (s.core_n > Np || M > 4 * Np)
      fail(SCOLA_EINVAL, "tile " + std::to_string(t) + " larger than the lattice");
    for (int a = 0; a < 3; ++a)
      if (s.core_lo[a] < 0 || s.core_lo[a] >= Np)
        fail(SCOLA_EINVAL, "tile core_lo must be in [0, Np)");
    for (int i = 0; i < s.core_n; ++i)
      for (int j = 0; j < s.core_n; ++j)
        for (int k = 0; k < s.core_n; ++k) {
          const size_t x = (s.core_lo[0] + i) % Np, y = (s.core_lo[1] + j) % Np,
                       z = (s.core_lo[2] + k) % Np;
          uint8_t& o = cover[(x * Np + y) * Np + z];
          if (o) fail(SCOLA_EINVAL, "tiles overlap (tile " + std::to_string(t) + ")");
          o = 1;
        }
  }
  for (uint8_t o : cover)
    if (!o) fail(SCOLA_EINVAL, "tiles do not cover the lattice");
}

template <typename T>
void upload_tables(scola_plan* p) {
  // twiddles W_{2M}^m and the FDA eigenvalues of App. C.2 per distinct M (FP64 on the host,
  // stored in the plan's precision): with s(x) = sin^2(x) and theta = pi l / M,
  //   order 2: -4 s(theta/2); order 4: (s(theta) - 16 s(theta/2)) / 3;
  //   order 6: -(2 s(3 theta/2) - 27 s(theta) + 270 s(theta/2)) / 45
  std::map<int, std::pair<int, int>> offs;
  std::vector<T> tw, ev;
  for (auto& d : p->desc) {
    if (offs.count(d.M)) continue;
    const int tw_off = (int)(tw.size() / 2), ev_off = (int)ev.size();
    const int N = 2 * d.M;
    for (int m = 0; m < N; ++m) {
      tw.push_back((T)std::cos(2.0 * M_PI * m / N));
      tw.push_back((T)(-std::sin(2.0 * M_PI * m / N)));
    }
    for (int l = 1; l < d.M; ++l) {
      const double th = M_PI * l / d.M;
      auto s2 = [](double x) { return std::sin(x) * std::sin(x); };
      double v;
      if (p->ng == 1) {
        const double s = std::sin(M_PI * l / (2.0 * d.M));
        v = -4.0 * s * s;
      } else if (p->ng == 2) {
        v = (s2(th) - 16.0 * s2(0.5 * th)) / 3.0;
      } else {
        v = -(2.0 * s2(1.5 * th) - 27.0 * s2(th) + 270.0 * s2(0.5 * th)) / 45.0;
      }
      ev.push_back((T)v);
    }
    offs[d.M] = {tw_off, ev_off};
  }
  for (auto& d : p->desc) {
    d.tw_off = offs[d.M].first;
    d.ev_off = offs[d.M].second;
  }
  if (sizeof(T) == 4) {
    // FP32 plans: per M, the DST-I matrix S[j][k] = sin(pi (j+1)(k+1) / M) (App. C.2, eq.
    // DST_delta) for j, k < M - 1, zero-padded to M rows of K = 32 ceil(M / 32) columns, as
    // FP16 hi = fp16(S) and lo = fp16(S - hi) (hi table, then lo table); (j+1)(k+1) is taken
    // modulo 2M so that the sine is evaluated at an argument below 2 pi
    std::map<int, int> soff;
    std::vector<_Float16> sm;
    for (auto& d : p->desc) {
      if (!soff.count(d.M)) {
        const int M = d.M, K = 32 * ((M + 31) / 32);
        soff[M] = (int)sm.size();
        std::vector<_Float16> hi((size_t)M * K, (_Float16)0.0f), lo((size_t)M * K, (_Float16)0.0f);
        for (int j = 0; j < M - 1; ++j)
          for (int k = 0; k < M - 1; ++k) {
            const double v = std::sin(M_PI * (double)(((j + 1) * (k + 1)) % (2 * M)) / M);
            const _Float16 h = (_Float16)(float)v;
            hi[(size_t)j * K + k] = h;
            lo[(size_t)j * K + k] = (_Float16)(float)(v - (double)(float)h);
          }
        sm.insert(sm.end(), hi.begin(), hi.end());
        sm.insert(sm.end(), lo.begin(), lo.end());
      }
      d.dm_off = soff[d.M];
    }
    hip_check(hipMalloc(&p->d_sine, sm.size() * sizeof(_Float16)), "hipMalloc(sine)");
    hip_check(hipMemcpy(p->d_sine, sm.data(), sm.size() * sizeof(_Float16), hipMemcpyHostToDevice),
              "hipMemcpy(sine)");
  }
  hip_check(hipMalloc(&p->d_twiddles, tw.size() * sizeof(T)), "hipMalloc(twiddles)");
  hip_check(hipMemcpy(p->d_twiddles, tw.data(), tw.size() * sizeof(T), hipMemcpyHostToDevice),
            "hipMemcpy(twiddles)");
  hip_check(hipMalloc(&p->d_eigen, ev.size() * sizeof(T)), "hipMalloc(eigen)");
  hip_check(hipMemcpy(p->d_eigen, ev.data(), ev.size() * sizeof(T), hipMemcpyHostToDevice),
            "hipMemcpy(eigen)");
}

void compute_step_table(const scola_config& c, const Background& bg, std::vector<double>& table,
                        std::vector<double>& D1out, std::vector<double>& D2out);

void build_step_table(scola_plan* p) {
  compute_step_table(p->cfg, p->bg, p->table, p->D1, p->D2);
}

void compute_step_table(const scola_config& c, const Background& bg, std::vector<double>& table,
                        std::vector<double>& D1out, std::vector<double>& D2out) {
  const int n = c.n_steps;
  std::vector<double> t(n + 1), half(n);
  for (int k = 0; k <= n; ++k) t[k] = c.a_i + (c.a_f - c.a_i) * k / n;
  for (int k = 0; k < n; ++k) half[k] = 0.5 * (t[k] + t[k + 1]);
  std::vector<double> q(t);
  q.push_back(c.a_i);
  std::vector<double> D1, dD1, D2, dD2;
  bg.growth(q, D1, dD1, D2, dD2);
  const double n1 = D1[n + 1];                      // D1 normalised to 1 at a_i
  D1out.assign(n + 1, 0.0);
  D2out.assign(n + 1, 0.0);
  for (int k = 0; k <= n; ++k) {
    D1out[k] = D1[k] / n1;
    D2out[k] = D2[k] / (n1 * n1);
  }
  // App. B: modified time factors with u(a) = a^n_LPT (the paper's n_LPT = -2.5), or the
  // standard ones (integrals of the drift and kick prefactors over the sub-step)
  const double nlpt = c.n_lpt != 0.0 ? c.n_lpt : -2.5;
  const bool standard = c.discretisation == SCOLA_STANDARD;
  auto beta = [&](double ai, double af, double aD) {
    return standard ? bg.beta_standard(ai, af) : bg.beta_tilde(ai, af, aD, nlpt);
  };
  auto alpha = [&](double ai, double af, double aK) {
    return standard ? bg.alpha_standard(ai, af) : bg.alpha_tilde(ai, af, aK, nlpt);
  };
  table.assign((size_t)(n + 1) * 8, 0.0);
  for (int k = 0; k < n; ++k) {
    double* r = &table[(size_t)k * 8];
    const double aKi = k == 0 ? t[0] : half[k - 1];
    r[0] = t[k];
    r[1] = beta(aKi, half[k], t[k]);
    r[2] = alpha(t[k], t[k + 1], half[k]);
    r[3] = D1out[k];
    r[4] = D2out[k];
    r[5] = D1out[k + 1];
    r[6] = D2out[k + 1];
    r[7] = t[k + 1];
  }
  double* r = &table[(size_t)n * 8];
  const double af = t[n];
  const double inv_drift = af * af * af * bg.E(af);   // 1 / drift prefactor
  r[0] = af;
  r[1] = beta(half[n - 1], af, af);
  r[2] = D1out[n];
  r[3] = D2out[n];
  r[4] = -dD1[n] / n1 * inv_drift;                       // L+ : p_LPT coefficients
  r[5] = dD2[n] / (n1 * n1) * inv_drift;
}

// Bytes of the fixed-point mass mesh, rounded to 8 so it is cleared in 64-bit words.
size_t rho_bytes(const scola_plan* p) {
  const size_t b = (size_t)p->G * (p->is64 ? sizeof(MeshFixed<double>::rho_t)
                                           : sizeof(MeshFixed<float>::rho_t));
  return (b + 7) / 8 * 8;
}

void build_layout(scola_plan* p) {
  const size_t R = p->is64 ? 8 : 4;
  const int64_t N = p->cfg.Np;
  const int64_t No = p->cfg.N_out;
  scola_layout& l = p->lay;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  l.psi1 = take(3 * (size_t)p->P * R);
  l.psi2 = take(3 * (size_t)p->P * R);
  l.x_res = take(3 * (size_t)p->P * R);
  l.p_res = take(3 * (size_t)p->P * R);
  l.rho = take(rho_bytes(p));
  l.work = take((size_t)p->G * R);
  l.phi = take((size_t)p->H * R);
  l.bc0 = take((size_t)p->H * 8);
  // per tile dropped mass, the near-limit count, then per tile the mass the Poisson passes
  // found and the number of deposits (the mass identity of FP32 plans)
  l.dropped = take((3 * p->desc.size() + 1) * 8);
  l.cells = take((size_t)(p->P / kBlock) * 16);   // per brick: packed cell extent
  const size_t NL = (size_t)p->N_lpt;   // the set-up fields live on the LPT grid
  l.phi1 = take(NL * NL * NL * 8);
  l.phi2 = take(NL * NL * NL * 8);
  l.cbuf = take(NL * NL * NL * 16);
  l.outgrid = take((size_t)(No * No * No) * 8);
  const int c = p->cfg.checkpoint_every;
  if (c > 0) {
    const size_t n_ckpt = (size_t)((p->cfg.n_steps + c - 1) / c);
    l.ckpt = take(n_ckpt * 6 * (size_t)p->P * R);
    l.seg_x = take((size_t)(c + 1) * 3 * (size_t)p->P * R);
    l.seg_phi = take((size_t)(c + 1) * (size_t)p->H * R);
    l.lam_x = take(3 * (size_t)p->P * R);
    l.lam_p = take(3 * (size_t)p->P * R);
    l.lam_psi1 = take(3 * (size_t)p->P * R);
    l.lam_psi2 = take(3 * (size_t)p->P * R);
    l.lam_rho = take((size_t)p->G * R);
    l.lam_bc0 = take((size_t)p->H * 8);
    l.adj_grid = take(14 * (size_t)(N * N * N) * 8);
  }
  l.total = off;
  l.n_particles = p->P;
  l.n_nodes = p->G;
  l.n_padded = p->H;
  l.fixed_bits = p->is64 ? MeshFixed<double>::bits : MeshFixed<float>::bits;
}

Background background_of(const scola_cosmology& c) {
  Background bg;
  bg.Om = c.Omega_m;
  bg.Ob = c.Omega_b;
  bg.h = c.h;
  bg.ns = c.n_s;
  bg.sigma8 = c.sigma8;
  bg.Tcmb = c.T_cmb;
  bg.normalise();
  return bg;
}

char* ws_ptr(void* ws, size_t off) { return static_cast<char*>(ws) + off; }

void check_ws(const scola_plan* p, void* ws) {
  if (!p) fail(SCOLA_EINVAL, "plan is NULL");
  if (!ws) fail(SCOLA_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) fail(SCOLA_EINVAL, "workspace must be 256-byte aligned");
  int dev = -1;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev != p->device) fail(SCOLA_EINVAL, "current device differs from the plan's device");
}

std::vector<int> subset_list(const scola_plan* p, const int32_t* subset, int32_t n) {
  std::vector<int> out;
  if (!subset) {
    for (size_t t = 0; t < p->desc.size(); ++t) out.push_back((int)t);
    return out;
  }
  if (n < 1) fail(SCOLA_EINVAL, "n_subset must be >= 1");
  std::vector<uint8_t> seen(p->desc.size(), 0);
  for (int i = 0; i < n; ++i) {
    if (subset[i] < 0 || subset[i] >= (int)p->desc.size()) fail(SCOLA_EINVAL, "tile index out of range");
    if (seen[subset[i]]) fail(SCOLA_EINVAL, "duplicate tile in subset");
    seen[subset[i]] = 1;
    out.push_back(subset[i]);
  }
  return out;
}

// FP32 deposits leave each brick's dropped mass in word 3 of its hint for the Poisson pass
// that consumes them; a deposit that no pass follows (the operator-level calls) folds it
// into the per-tile counters here.
void fold_drops(scola_plan* p, void* ws, hipStream_t s) {
  hip_check(launch_fold_drops(p->d_tiles, (int)p->desc.size(),
                              reinterpret_cast<unsigned*>(ws_ptr(ws, p->lay.cells)),
                              reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped)),
                              s), "fold dropped mass");
}

template <typename T>
MeshArgs<T> mesh_args(scola_plan* p, void* ws, double D1_bc) {
  MeshArgs<T> a;
  a.tiles = p->d_tiles;
  a.rho = reinterpret_cast<typename MeshFixed<T>::rho_t*>(ws_ptr(ws, p->lay.rho));
  a.alarm = reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped)) + p->desc.size();
  a.kept = a.alarm + 1;
  a.dropped = a.alarm - p->desc.size();
  a.hints = reinterpret_cast<unsigned*>(ws_ptr(ws, p->lay.cells));
  a.work = reinterpret_cast<T*>(ws_ptr(ws, p->lay.work));
  a.phi = reinterpret_cast<T*>(ws_ptr(ws, p->lay.phi));
  a.bc0 = reinterpret_cast<const double*>(ws_ptr(ws, p->lay.bc0));
  a.twiddles = p->d_twiddles;
  a.eigen = reinterpret_cast<const T*>(p->d_eigen);
  a.sine = p->d_sine;
  a.D1_bc = D1_bc;
  a.ng = p->ng;
  return a;
}

template <typename T>
ParticleArgs<T> particle_args(scola_plan* p, void* ws, const StepScalars& sc) {
  ParticleArgs<T> a;
  a.tiles = p->d_tiles;
  a.psi1 = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.psi1));
  a.psi2 = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.psi2));
  a.xres = reinterpret_cast<T*>(ws_ptr(ws, p->lay.x_res));
  a.xout = a.xres;
  a.pres = reinterpret_cast<T*>(ws_ptr(ws, p->lay.p_res));
  a.phi = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.phi));
  a.rho = reinterpret_cast<typename MeshFixed<T>::rho_t*>(ws_ptr(ws, p->lay.rho));
  a.dropped = reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped));
  a.deposits = a.dropped + 2 * p->desc.size() + 1;
  a.cells = reinterpret_cast<uint4*>(ws_ptr(ws, p->lay.cells));
  a.use_hints = 1;
  a.P = p->P;
  a.sc = sc;
  a.ng = p->ng;
  return a;
}

const scola_class_schedule& sched_of(const scola_plan* p, int M) {
  for (size_t c = 0; c < p->part.class_M.size(); ++c)
    if (p->part.class_M[c] == M) return p->sched[c];
  return p->sched.front();
}

BlockMap class_map(const Maps& m, size_t c) {
  BlockMap b = full_map(m);
  b.base = m.class_first[c];
  b.count = m.class_count[c];
  return b;
}

// Tiles [i0, i1) of size class c's tile list for group g of G (halves when G = 2).
void group_range(const scola_plan* p, size_t c, int g, int G, size_t& i0, size_t& i1) {
  const size_t n = p->class_tiles[c].size();
  i0 = n * (size_t)g / (size_t)G;
  i1 = n * (size_t)(g + 1) / (size_t)G;
}

// Blocks of group g of G of size class c (the class's tiles are contiguous in every map).
BlockMap class_group_map(const scola_plan* p, const Maps& m, size_t c, int g, int G) {
  if (G == 1) return class_map(m, c);
  size_t i0, i1;
  group_range(p, c, g, G, i0, i1);
  BlockMap b = full_map(m);
  b.base = 0;
  b.count = 0;
  if (i0 < i1) {
    b.base = m.first[p->class_tiles[c][i0]];
    for (size_t i = i0; i < i1; ++i) b.count += m.count[p->class_tiles[c][i]];
  }
  return b;
}

// The tiles of group g of G over all classes.
std::vector<int> group_tiles(const scola_plan* p, int g, int G) {
  std::vector<int> out;
  for (size_t c = 0; c < p->class_tiles.size(); ++c) {
    size_t i0, i1;
    group_range(p, c, g, G, i0, i1);
    for (size_t i = i0; i < i1; ++i) out.push_back(p->class_tiles[c][i]);
  }
  std::sort(out.begin(), out.end());
  return out;
}

// The three Poisson passes over the boxes of size class c (group g of G), forward or
// adjoint solve.
template <typename T>
void poisson_class(const scola_plan* p, const MeshArgs<T>& a, size_t c, bool adjoint,
                   hipStream_t s, int g = 0, int G = 1) {
  BlockMap b1 = class_group_map(p, p->p1, c, g, G), b2 = class_group_map(p, p->p2, c, g, G),
           b3 = class_group_map(p, p->p3, c, g, G);
  if (b1.count == 0) return;
  b1.xcd_remap = b2.xcd_remap = b3.xcd_remap = p->sched[c].xcd_remap_mesh;
  hip_check(launch_poisson<T>(a, p->p1.class_M[c], b1, b2, b3, s, adjoint), "poisson kernels");
}

// Scalars of the evolution for time class tc: the growth at t_0 (kInit), the final half
// kick and L+ (kFinalKick), else row k of the class's step table.
StepScalars class_scalars(const scola_plan* p, int tc, int mode, int k) {
  const TimeClass& c = p->tclasses[tc];
  StepScalars sc{};
  if (mode == kInit || mode == kDepositOnly) {
    sc.D1 = c.D1[k];
    sc.D2 = c.D2[k];
    return sc;
  }
  const double* r = &c.table[(size_t)k * 8];
  if (mode == kFinalKick) {
    sc.beta = r[1];
    sc.D1 = r[2];
    sc.D2 = r[3];
    sc.c1 = r[4];
    sc.c2 = r[5];
    return sc;
  }
  sc.beta = r[1];
  sc.alpha = r[2];
  sc.D1 = r[3];
  sc.D2 = r[4];
  sc.D1n = r[5];
  sc.D2n = r[6];
  return sc;
}

// One call of each kernel family over a set of tiles: all in one launch (batched) or one
// launch per tile.
template <typename T>
struct Runner {
  scola_plan* p;
  void* ws;
  hipStream_t s;
  std::vector<int> tiles;
  bool batched;
  // optional redirections (segment recomputation of the reverse sweep): positions read from
  // x_in and written to x_out, potential written and read at phi
  T* x_in = nullptr;
  T* x_out = nullptr;
  T* phi = nullptr;
  int group = 0, ngroups = 1;   // batched: this group's share of every class
  // the evolution starts without writing the zeros of L- (no checkpoint reads them)
  bool fresh_start = false;

  std::vector<BlockMap> maps(const Maps& m) const {
    std::vector<BlockMap> out;
    if (batched) {
      out.push_back(full_map(m));
    } else {
      for (int t : tiles) out.push_back(tile_map(m, t));
    }
    return out;
  }
  void particles(int mode, const StepScalars& sc) {
    ParticleArgs<T> a = particle_args<T>(p, ws, sc);
    if (x_in) a.xres = x_in;
    a.xout = x_out ? x_out : a.xres;
    if (phi) a.phi = phi;
    const Maps& pm = p->part;
    if (batched) {
      for (size_t c = 0; c < pm.class_M.size(); ++c) {
        BlockMap b = class_group_map(p, pm, c, group, ngroups);
        if (b.count == 0) continue;
        b.xcd_remap = p->sched[c].xcd_remap_particles;
        hip_check(launch_particles<T>(a, mode, b, p->sched[c].waves_per_simd, s),
                  "particle kernel");
      }
    } else {
      for (int t : tiles) {
        const scola_class_schedule& cs = sched_of(p, p->desc[t].M);
        BlockMap b = tile_map(pm, t);
        b.xcd_remap = cs.xcd_remap_particles;
        hip_check(launch_particles<T>(a, mode, b, cs.waves_per_simd, s), "particle kernel");
      }
    }
  }
  // Step-indexed forms for the evolution: every class (or tile) takes the scalars of its
  // own time class.  mode kInit: the growth at t_0; kFinalKick: the final row; otherwise
  // row k of the step table.
  void particles_step(int mode, int k) {
    // L- and the first step of an evolution that starts fresh (see StepScalars::fresh)
    auto scalars = [&](int tc) {
      StepScalars sc = class_scalars(p, tc, mode, k);
      sc.fresh = fresh_start && k == 0 && mode != kFinalKick ? 1 : 0;
      return sc;
    };
    if (batched) {
      const Maps& pm = p->part;
      for (size_t c = 0; c < pm.class_M.size(); ++c) {
        BlockMap b = class_group_map(p, pm, c, group, ngroups);
        if (b.count == 0) continue;
        b.xcd_remap = p->sched[c].xcd_remap_particles;
        ParticleArgs<T> a = args_of(scalars(pm.class_tc[c]));
        hip_check(launch_particles<T>(a, mode, b, p->sched[c].waves_per_simd, s),
                  "particle kernel");
      }
    } else {
      for (int t : tiles) {
        const scola_class_schedule& cs = sched_of(p, p->desc[t].M);
        BlockMap b = tile_map(p->part, t);
        b.xcd_remap = cs.xcd_remap_particles;
        ParticleArgs<T> a = args_of(scalars(p->desc[t].tclass));
        hip_check(launch_particles<T>(a, mode, b, cs.waves_per_simd, s), "particle kernel");
      }
    }
  }
  ParticleArgs<T> args_of(const StepScalars& sc) {
    ParticleArgs<T> a = particle_args<T>(p, ws, sc);
    if (x_in) a.xres = x_in;
    a.xout = x_out ? x_out : a.xres;
    if (phi) a.phi = phi;
    return a;
  }
  // the Poisson solve of force evaluation k (at t_k of each class)
  void poisson_step(int k) {
    MeshArgs<T> a = mesh_args<T>(p, ws, 0.0);
    if (phi) a.phi = phi;
    // the boundary-source perimeter terms pass from each solve's P3 to the next one's P1
    // through the consumed work planes (the first solve of an evolution gathers them)
    if (!ov_delta && !ov_phi) a.bc_handoff = k == 0 ? 2 : 3;
    if (ov_delta || ov_phi) {
      const size_t N3 = (size_t)p->cfg.Np * p->cfg.Np * p->cfg.Np;
      a.ov_N = p->cfg.Np;
      if (ov_delta) a.ov_delta = ov_delta + (size_t)force * N3;
      if (ov_phi) a.ov_phi = ov_phi + (size_t)force * N3;
    }
    ++force;
    if (batched) {
      for (size_t c = 0; c < p->p1.class_M.size(); ++c) {
        a.D1_bc = p->tclasses[p->p1.class_tc[c]].D1[k];
        poisson_class(p, a, c, false, s, group, ngroups);
      }
    } else {
      for (int t : tiles) {
        a.D1_bc = p->tclasses[p->desc[t].tclass].D1[k];
        const int r = sched_of(p, p->desc[t].M).xcd_remap_mesh;
        BlockMap b1 = tile_map(p->p1, t), b2 = tile_map(p->p2, t), b3 = tile_map(p->p3, t);
        b1.xcd_remap = b2.xcd_remap = b3.xcd_remap = r;
        hip_check(launch_poisson<T>(a, p->desc[t].M, b1, b2, b3, s), "poisson kernels");
      }
    }
  }
  // consistency tests (Sec. 4.3): full-box fields [n_force][N^3] replacing the density
  // contrast and/or the boundary potential of force evaluation `force`
  const T* ov_delta = nullptr;
  const T* ov_phi = nullptr;
  int force = 0;
  void poisson(double D1_bc) {
    MeshArgs<T> a = mesh_args<T>(p, ws, D1_bc);
    if (phi) a.phi = phi;
    if (ov_delta || ov_phi) {
      const size_t N3 = (size_t)p->cfg.Np * p->cfg.Np * p->cfg.Np;
      a.ov_N = p->cfg.Np;
      if (ov_delta) a.ov_delta = ov_delta + (size_t)force * N3;
      if (ov_phi) a.ov_phi = ov_phi + (size_t)force * N3;
    }
    ++force;
    if (batched) {
      for (size_t c = 0; c < p->p1.class_M.size(); ++c)
        poisson_class(p, a, c, false, s, group, ngroups);
    } else {
      for (int t : tiles) {
        const int r = sched_of(p, p->desc[t].M).xcd_remap_mesh;
        BlockMap b1 = tile_map(p->p1, t), b2 = tile_map(p->p2, t), b3 = tile_map(p->p3, t);
        b1.xcd_remap = b2.xcd_remap = b3.xcd_remap = r;
        hip_check(launch_poisson<T>(a, p->desc[t].M, b1, b2, b3, s), "poisson kernels");
      }
    }
  }
};

SetupArgs setup_args(scola_plan* p, const double* w, void* ws) {
  SetupArgs a;
  a.white_noise = w;
  a.cbuf = reinterpret_cast<double2*>(ws_ptr(ws, p->lay.cbuf));
  a.phi1 = reinterpret_cast<double*>(ws_ptr(ws, p->lay.phi1));
  a.phi2 = reinterpret_cast<double*>(ws_ptr(ws, p->lay.phi2));
  a.N = p->N_lpt;
  a.L = p->cfg.L;
  a.amplitude = p->bg.amplitude;
  a.ns = p->bg.ns;
  a.Om = p->bg.Om;
  a.Ob = p->bg.Ob;
  a.h = p->bg.h;
  a.Tcmb = p->bg.Tcmb;
  // P_lin(k, a_i) = P_lin(k, 1) (D1(a_i) / D1(1))^2 with D1 normalised at a_i
  std::vector<double> q = {p->cfg.a_i, 1.0}, D1, dD1, D2, dD2;
  p->bg.growth(q, D1, dD1, D2, dD2);
  a.growth2 = (D1[0] / D1[1]) * (D1[0] / D1[1]);
  a.ng = p->ng;
  return a;
}

BoxSetupArgs box_setup_args(scola_plan* p, void* ws) {
  BoxSetupArgs b;
  b.tiles = p->d_tiles;
  b.n_tiles = (int)p->desc.size();
  b.blk_tile = p->part.d_tile;
  b.blk_first = p->part.d_local;
  b.n_blocks = (int)p->part.tile.size();
  b.phi1 = reinterpret_cast<double*>(ws_ptr(ws, p->lay.phi1));
  b.phi2 = reinterpret_cast<double*>(ws_ptr(ws, p->lay.phi2));
  b.psi1 = ws_ptr(ws, p->lay.psi1);
  b.psi2 = ws_ptr(ws, p->lay.psi2);
  b.bc0 = reinterpret_cast<double*>(ws_ptr(ws, p->lay.bc0));
  b.N = p->N_lpt;
  b.P = p->P;
  b.ng = p->ng;
  b.Np = p->cfg.Np;
  return b;
}

template <typename T>
void do_setup(scola_plan* p, const double* w, void* ws, hipStream_t s) {
  SetupArgs a = setup_args(p, w, ws);
  hip_check(launch_setup_potentials(a, s), "set-up potentials");
  BoxSetupArgs b = box_setup_args(p, ws);
  hip_check(launch_setup_boxes<T>(b, reinterpret_cast<T*>(ws_ptr(ws, p->lay.x_res)),
                                  reinterpret_cast<T*>(ws_ptr(ws, p->lay.p_res)), s),
            "set-up boxes");
  hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.rho)),
                            (int64_t)(rho_bytes(p) / 8), s), "zero rho");
  // zero words decode to an extent wider than any window: the first force pass reduces
  // its own
  hip_check(launch_zero_u32(reinterpret_cast<unsigned*>(ws_ptr(ws, p->lay.cells)),
                            (p->P / kBlock) * 4, s), "zero cell hints");
}

StepScalars row_scalars(const scola_plan* p, int k) {
  const double* r = &p->table[(size_t)k * 8];
  StepScalars sc{};
  sc.beta = r[1];
  sc.alpha = r[2];
  sc.D1 = r[3];
  sc.D2 = r[4];
  sc.D1n = r[5];
  sc.D2n = r[6];
  return sc;
}

// (x_res, p_res) of the given tiles -> checkpoint slot (to_ckpt) or back; tiles whose
// particle ranges are adjacent are copied together.
template <typename T>
void copy_checkpoint(scola_plan* p, const std::vector<int>& tiles, int slot, bool to_ckpt,
                     void* ws, hipStream_t s) {
  const size_t R = sizeof(T);
  char* ck = ws_ptr(ws, p->lay.ckpt) + (size_t)slot * 6 * p->P * R;
  char* st[2] = {ws_ptr(ws, p->lay.x_res), ws_ptr(ws, p->lay.p_res)};
  std::vector<int> sorted = tiles;
  std::sort(sorted.begin(), sorted.end());
  std::vector<std::pair<int64_t, int64_t>> runs;   // [first particle, count)
  for (int t : sorted) {
    const int64_t M = p->desc[t].M, off = p->desc[t].p_off, cnt = M * M * M;
    if (!runs.empty() && runs.back().first + runs.back().second == off)
      runs.back().second += cnt;
    else
      runs.push_back({off, cnt});
  }
  for (int a = 0; a < 2; ++a) {
    char* c = ck + (size_t)a * 3 * p->P * R;
    for (int comp = 0; comp < 3; ++comp)
      for (const auto& r : runs) {
        const size_t o = ((size_t)comp * p->P + (size_t)r.first) * R;
        const size_t nb = (size_t)r.second * R;
        hip_check(hipMemcpyAsync(to_ckpt ? c + o : st[a] + o, to_ckpt ? st[a] + o : c + o, nb,
                                 hipMemcpyDeviceToDevice, s), "checkpoint copy");
      }
  }
}

// Fork G - 1 plan-owned streams from s (after everything enqueued on s so far) and join
// them back into s.
void fork_streams(scola_plan* p, int G, hipStream_t s) {
  if (!p->ev_fork) hip_check(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming), "event");
  hip_check(hipEventRecord(p->ev_fork, s), "hipEventRecord");
  for (int g = 1; g < G; ++g) {
    if (!p->aux_stream[g - 1])
      hip_check(hipStreamCreateWithFlags(&p->aux_stream[g - 1], hipStreamNonBlocking),
                "hipStreamCreateWithFlags");
    if (!p->ev_join[g - 1])
      hip_check(hipEventCreateWithFlags(&p->ev_join[g - 1], hipEventDisableTiming), "event");
    hip_check(hipStreamWaitEvent(p->aux_stream[g - 1], p->ev_fork, 0), "hipStreamWaitEvent");
  }
}

void join_streams(scola_plan* p, int G, hipStream_t s) {
  for (int g = 1; g < G; ++g) {
    hip_check(hipEventRecord(p->ev_join[g - 1], p->aux_stream[g - 1]), "hipEventRecord");
    hip_check(hipStreamWaitEvent(s, p->ev_join[g - 1], 0), "hipStreamWaitEvent");
  }
}

// Runs of adjacent tiles: [first, count) in particle (or node) units.
std::vector<std::pair<int64_t, int64_t>> tile_runs(const scola_plan* p, const std::vector<int>& tiles,
                                                   bool nodes) {
  std::vector<int> sorted = tiles;
  std::sort(sorted.begin(), sorted.end());
  std::vector<std::pair<int64_t, int64_t>> runs;
  for (int t : sorted) {
    const int64_t M = p->desc[t].M;
    const int64_t off = nodes ? p->desc[t].g_off : p->desc[t].p_off;
    const int64_t cnt = nodes ? (M - 1) * (M - 1) * (M - 1) : M * M * M;
    if (!runs.empty() && runs.back().first + runs.back().second == off)
      runs.back().second += cnt;
    else
      runs.push_back({off, cnt});
  }
  return runs;
}

// dst[3][P] <- src[3][P] for the particles of the given tiles.
template <typename T>
void copy_particle_ranges(const scola_plan* p, const std::vector<int>& tiles, T* dst,
                          const T* src, hipStream_t s) {
  for (const auto& r : tile_runs(p, tiles, false))
    for (int comp = 0; comp < 3; ++comp) {
      const size_t o = (size_t)comp * p->P + (size_t)r.first;
      hip_check(hipMemcpyAsync(dst + o, src + o, (size_t)r.second * sizeof(T),
                               hipMemcpyDeviceToDevice, s), "checkpoint restore");
    }
}

// Clear the interior-node array entries [G] of the given tiles.
template <typename T>
void zero_node_ranges(const scola_plan* p, const std::vector<int>& tiles, T* arr, hipStream_t s) {
  for (const auto& r : tile_runs(p, tiles, true))
    hip_check(launch_zero_u32(reinterpret_cast<unsigned*>(arr + r.first),
                              r.second * (int64_t)(sizeof(T) / 4), s), "zero");
}

// One KDK step k of every class as one persistent launch per class (FP32 batched plans):
// the particle step and the Poisson passes of force k + 1.
template <typename T>
void persistent_step(scola_plan* p, void* ws, int k, bool fresh, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    for (size_t c = 0; c < p->part.class_M.size(); ++c) {
      const int tc = p->part.class_tc[c];
      StepScalars sc = class_scalars(p, tc, kStep, k);
      sc.fresh = fresh ? 1 : 0;
      ParticleArgs<T> pa = particle_args<T>(p, ws, sc);
      MeshArgs<T> ma = mesh_args<T>(p, ws, p->tclasses[tc].D1[k + 1]);
      ma.bc_handoff = 3;   // solve k + 1 of an evolution (see Runner::poisson_step)
      BlockMap mp = class_map(p->part, c), m1 = class_map(p->p1, c), m2 = class_map(p->p2, c),
               m3 = class_map(p->p3, c);
      mp.xcd_remap = p->sched[c].xcd_remap_particles;
      m1.xcd_remap = m2.xcd_remap = m3.xcd_remap = p->sched[c].xcd_remap_mesh;
      hip_check(launch_step_persistent<T>(pa, ma, p->part.class_M[c], mp, m1, m2, m3,
                                          p->d_barrier, s, &p->persistent_grid),
                "persistent step kernel");
    }
  } else {
    fail(SCOLA_EUNSUPPORTED, "the persistent step is built for FP32 plans");
  }
}

// allow_groups = false keeps the whole evolution on `s` (no plan-owned streams or events
// are created or used).
template <typename T>
void do_evolve(scola_plan* p, const std::vector<int>& tiles, void* ws, hipStream_t s,
               bool allow_groups = true, const T* ov_delta = nullptr,
               const T* ov_phi = nullptr) {
  const bool batched = p->cfg.schedule == SCOLA_BATCHED && tiles.size() == p->desc.size();
  hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped)),
                            3 * (int64_t)p->desc.size() + 1, s), "zero dropped");
  if (p->persistent) hip_check(launch_zero_u32(p->d_barrier, 2, s), "zero barrier");
  const int n = p->cfg.n_steps;
  auto run = [&](const std::vector<int>& set, bool b, hipStream_t s, int g, int G) {
    Runner<T> r{p, ws, s, set, b};
    r.group = g;
    r.ngroups = G;
    r.ov_delta = ov_delta;
    r.ov_phi = ov_phi;
    const int ck = p->cfg.checkpoint_every;
    // without checkpoints nothing reads x_res, p_res before the first step writes them, so
    // L- leaves them unwritten and the first step takes them as zero (48 bytes a particle
    // less per evolution); a checkpoint of step 0 needs the stored zeros
    r.fresh_start = ck <= 0;
    r.particles_step(kInit, 0);             // L-: x_res = p_res = 0, deposit x_LPT(t_0)
    r.poisson_step(0);
    const bool fused = p->persistent && b && G == 1 && !ov_delta && !ov_phi;
    for (int k = 0; k < n; ++k) {
      if (ck > 0 && k % ck == 0) copy_checkpoint<T>(p, set, k / ck, true, ws, s);
      const bool need_force = k < n - 1 || p->cfg.want_momenta;
      if (need_force && fused) {
        persistent_step<T>(p, ws, k, r.fresh_start && k == 0, s);
        r.force++;
        continue;
      }
      r.particles_step(need_force ? kStep : kStepNoDeposit, k);
      if (need_force) r.poisson_step(k + 1);
    }
    if (p->cfg.want_momenta) r.particles_step(kFinalKick, n);
  };
  // the persistent step runs every class on the caller's stream (one group)
  const int G = batched && allow_groups && !p->persistent
                    ? std::min<int>(p->groups, (int)tiles.size()) : 1;
  if (batched && G > 1) {
    // G shares of every size class advance concurrently on G streams, so one share's
    // Poisson passes overlap another share's particle kernel
    fork_streams(p, G, s);
    for (int g = 0; g < G; ++g)
      run(group_tiles(p, g, G), true, g ? p->aux_stream[g - 1] : s, g, G);
    join_streams(p, G, s);
  } else if (batched) {
    run(tiles, true, s, 0, 1);
  } else {
    for (int t : tiles) run(std::vector<int>{t}, false, s, 0, 1);   // plain per-tile schedule
  }
}

template <typename T>
void do_output(scola_plan* p, void* pos, void* mom, void* dens, const std::vector<int>& tiles,
               void* ws, hipStream_t s) {
  OutputArgs<T> a;
  a.tiles = p->d_tiles;
  a.psi1 = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.psi1));
  a.psi2 = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.psi2));
  a.xres = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.x_res));
  a.pres = reinterpret_cast<const T*>(ws_ptr(ws, p->lay.p_res));
  a.pos = reinterpret_cast<T*>(pos);
  a.mom = reinterpret_cast<T*>(mom);
  a.grid = reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.outgrid));
  a.P = p->P;
  a.Np = p->cfg.Np;
  a.N_out = p->cfg.N_out;
  a.D1 = p->D1[p->cfg.n_steps];
  a.D2 = p->D2[p->cfg.n_steps];
  a.cell = p->cfg.L / p->cfg.Np;
  a.L = p->cfg.L;
  const bool all = tiles.size() == p->desc.size();
  if (all) {
    hip_check(launch_output<T>(a, full_map(p->part), dens != nullptr,
                               reinterpret_cast<T*>(dens), s), "output kernel");
  } else {
    for (int t : tiles)
      hip_check(launch_output<T>(a, tile_map(p->part, t), false, nullptr, s), "output kernel");
  }
}

void zero_bytes(void* ptr, size_t bytes, hipStream_t s) {
  // every region zeroed here is 8-byte aligned and a multiple of 4 bytes long
  if (bytes % 8 == 0) {
    hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ptr), (int64_t)(bytes / 8), s),
              "zero");
  } else {
    hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ptr), (int64_t)(bytes / 8), s),
              "zero");
    hip_check(hipMemsetAsync(static_cast<char*>(ptr) + bytes - 4, 0, 4, s), "zero tail");
  }
}

// Positions x_res and potentials of the steps of one segment, kept in a ring of c + 1 slots
// indexed by step mod (c + 1): the segment [k0, k1] needs k1 - k0 + 1 <= c + 1 of them, and
// the slot of step k1 still holds what the recomputation of the later segment left there.
template <typename T>
struct SegmentRing {
  T* x;
  T* phi;
  int slots;
  int64_t P, H;
  T* xs(int k) const { return x + (size_t)(k % slots) * 3 * P; }
  T* ph(int k) const { return phi + (size_t)(k % slots) * H; }
};

template <typename T>
void do_backward(scola_plan* p, const T* lam_dens, double* grad_w, void* ws, hipStream_t s) {
  const scola_layout& l = p->lay;
  const int n = p->cfg.n_steps, c = p->cfg.checkpoint_every, N = p->cfg.Np;
  const int nseg = (n + c - 1) / c;
  const size_t R = sizeof(T);
  const int64_t N3 = (int64_t)N * N * N;
  AdjointArgs<T> a{};
  a.tiles = p->d_tiles;
  a.psi1 = reinterpret_cast<const T*>(ws_ptr(ws, l.psi1));
  a.psi2 = reinterpret_cast<const T*>(ws_ptr(ws, l.psi2));
  a.lam_x = reinterpret_cast<T*>(ws_ptr(ws, l.lam_x));
  a.lam_p = reinterpret_cast<T*>(ws_ptr(ws, l.lam_p));
  a.lam_psi1 = reinterpret_cast<T*>(ws_ptr(ws, l.lam_psi1));
  a.lam_psi2 = reinterpret_cast<T*>(ws_ptr(ws, l.lam_psi2));
  a.lam_rho = reinterpret_cast<const T*>(ws_ptr(ws, l.lam_rho));
  a.work = reinterpret_cast<T*>(ws_ptr(ws, l.work));
  a.lam_bc0 = reinterpret_cast<double*>(ws_ptr(ws, l.lam_bc0));
  a.P = p->P;
  a.H = p->H;
  zero_bytes(a.lam_bc0, (size_t)p->H * 8, s);
  // transpose of the output density at the final positions
  a.xg = reinterpret_cast<const T*>(ws_ptr(ws, l.x_res));
  a.D1g = p->D1[n];
  a.D2g = p->D2[n];
  hip_check(launch_adj_output<T>(a, full_map(p->part), lam_dens, N, p->cfg.N_out, s),
            "adjoint output");
  std::vector<int> all = subset_list(p, nullptr, 0);
  const SegmentRing<T> ring{reinterpret_cast<T*>(ws_ptr(ws, l.seg_x)),
                            reinterpret_cast<T*>(ws_ptr(ws, l.seg_phi)), c + 1, p->P, p->H};
  MeshArgs<T> m = mesh_args<T>(p, ws, 0.0);
  m.lam_rho = const_cast<T*>(a.lam_rho);
  m.lam_bc0 = a.lam_bc0;
  // The boxes are independent until the set-up adjoint: G groups of them (the tuned
  // concurrency) run their whole reverse sweep on G streams.
  auto reverse = [&](int grp, int G, hipStream_t st) {
    AdjointArgs<T> ga = a;
    MeshArgs<T> gm = m;
    const std::vector<int> mine = G == 1 ? all : group_tiles(p, grp, G);
    auto particle_maps = [&]() {
      std::vector<BlockMap> out;
      for (size_t cl = 0; cl < p->part.class_M.size(); ++cl) {
        BlockMap b = class_group_map(p, p->part, cl, grp, G);
        if (b.count > 0) out.push_back(b);
      }
      return out;
    };
    const std::vector<BlockMap> pmaps = particle_maps();
    auto set_gather = [&](int gs) {       // force of step gs
      const StepScalars sg = row_scalars(p, gs);
      ga.xg = ring.xs(gs);
      ga.phi = ring.ph(gs);
      ga.beta_g = sg.beta;
      ga.D1g = sg.D1;
      ga.D2g = sg.D2;
    };
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int k0 = seg * c, k1 = std::min(k0 + c, n);
      // recompute the segment from its checkpoint: x_res and the potential of steps
      // k0 .. k1-1 into the ring (step k1's entries are there from the later segment)
      const T* ck = reinterpret_cast<const T*>(ws_ptr(ws, l.ckpt) + (size_t)seg * 6 * p->P * R);
      copy_particle_ranges<T>(p, mine, ring.xs(k0), ck, st);
      copy_particle_ranges<T>(p, mine, reinterpret_cast<T*>(ws_ptr(ws, l.p_res)), ck + 3 * p->P,
                              st);
      Runner<T> r{p, ws, st, mine, true};
      r.group = grp;
      r.ngroups = G;
      r.x_in = ring.xs(k0);
      r.phi = ring.ph(k0);
      StepScalars d0{};
      d0.D1 = p->D1[k0];
      d0.D2 = p->D2[k0];
      r.particles(kDepositOnly, d0);
      r.poisson(p->D1[k0]);
      for (int k = k0; k + 1 < k1; ++k) {
        r.x_in = ring.xs(k);
        r.x_out = ring.xs(k + 1);
        r.phi = ring.ph(k);
        r.particles(kStep, row_scalars(p, k));
        r.phi = ring.ph(k + 1);
        r.poisson(p->D1[k + 1]);
      }
      zero_node_ranges<T>(p, mine, ga.work, st);   // left over from the recomputation
      // reverse the segment: gather of step k+1 fused with the scatter of step k
      for (int k = k1 - 1; k >= k0; --k) {
        const bool gather = k + 1 < n;
        if (gather) set_gather(k + 1);
        const StepScalars sc = row_scalars(p, k);
        ga.xs = ring.xs(k);
        ga.alpha = sc.alpha;
        ga.beta = sc.beta;
        ga.D1 = sc.D1;
        ga.D2 = sc.D2;
        for (const BlockMap& b : pmaps)
          hip_check(launch_adj_step<T>(ga, b, gather, true, st), "adjoint particles");
        gm.D1_bc = sc.D1;
        for (size_t cl = 0; cl < p->p1.class_M.size(); ++cl)
          poisson_class(p, gm, cl, true, st, grp, G);
      }
    }
    set_gather(0);
    for (const BlockMap& b : pmaps)
      hip_check(launch_adj_step<T>(ga, b, true, false, st), "adjoint particles");
  };
  const int G = std::min<int>(p->groups, (int)p->desc.size());
  if (G > 1) {
    fork_streams(p, G, s);
    for (int grp = 0; grp < G; ++grp) reverse(grp, G, grp ? p->aux_stream[grp - 1] : s);
    join_streams(p, G, s);
  } else {
    reverse(0, 1, s);
  }
  // FP64 set-up adjoint: Psi1, Psi2, Phi_BC^0 -> phi1, phi2 -> white noise
  double* g = reinterpret_cast<double*>(ws_ptr(ws, l.adj_grid));
  double* lam_psig = g;               // 6 N^3
  double* lam_phi1 = g + 6 * N3;      // N^3
  double* lam_s = g + 7 * N3;         // N^3
  double* f6 = g + 8 * N3;            // 6 N^3
  double2* cbuf = reinterpret_cast<double2*>(ws_ptr(ws, l.cbuf));
  zero_bytes(g, 7 * (size_t)N3 * 8, s);
  BoxSetupArgs b = box_setup_args(p, ws);
  hip_check(launch_adj_setup_scatter<T>(b, a.lam_psi1, a.lam_psi2, lam_psig, a.lam_bc0, lam_phi1, s),
            "adjoint set-up scatter");
  hip_check(launch_adj_phi_from_psi(lam_psig, lam_phi1, cbuf, N, s), "adjoint D^T");
  hip_check(fft3d_forward(cbuf, N, s), "fft");
  hip_check(launch_inverse_laplacian(cbuf, N, p->ng, s), "adjoint Poisson (2LPT)");
  hip_check(fft3d_inverse(cbuf, N, s), "fft");
  hip_check(launch_take_real(cbuf, lam_s, 1.0 / (double)N3, N3, s), "take real");
  hip_check(launch_adj_source(reinterpret_cast<const double*>(ws_ptr(ws, l.phi1)), lam_s, f6,
                              lam_phi1, N, s), "adjoint second-order source");
  hip_check(launch_real_to_complex(lam_phi1, cbuf, N3, s), "real to complex");
  hip_check(fft3d_forward(cbuf, N, s), "fft");
  SetupArgs sa = setup_args(p, nullptr, ws);
  hip_check(launch_ic_filter(sa, s), "adjoint IC filter");
  hip_check(fft3d_inverse(cbuf, N, s), "fft");
  hip_check(launch_take_real(cbuf, grad_w, 1.0 / (double)N3, N3, s), "take real");
}

void drop_graph(scola_plan* p) {
  if (p->evolve_exec) hipGraphExecDestroy(p->evolve_exec);
  if (p->evolve_graph) hipGraphDestroy(p->evolve_graph);
  p->evolve_exec = nullptr;
  p->evolve_graph = nullptr;
  p->graph_ws = nullptr;
  p->graph_eager_calls = 0;
}

// Record the batched evolution (every kernel, checkpoint copy and counter reset of
// do_evolve; no memset nodes) on the plan's capture stream and instantiate it.
template <typename T>
void capture_evolve(scola_plan* p, const std::vector<int>& tiles, void* ws) {
  if (!p->capture_stream)
    hip_check(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking),
              "hipStreamCreateWithFlags");
  hip_check(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal),
            "hipStreamBeginCapture");
  try {
    do_evolve<T>(p, tiles, ws, p->capture_stream);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(p->capture_stream, &g);
    if (g) hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  hip_check(hipStreamEndCapture(p->capture_stream, &g), "hipStreamEndCapture");
  hipGraphExec_t e = nullptr;
  const hipError_t err = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    hipGraphDestroy(g);
    hip_check(err, "hipGraphInstantiate");
  }
  p->evolve_graph = g;
  p->evolve_exec = e;
}

// Launch-schedule autotuner.  For every size class it times, on the workspace's own
// particles at the positions of the last step (x_res as left by the set-up, i.e. on the
// 2LPT trajectory) with zero kick and drift so the particle state is unchanged: the fused
// step kernel with and without the XCD-aware block numbering, then the three Poisson passes
// with and without it; the fastest of each is kept.  Then whole evolutions choose, together,
// the particle kernel's occupancy (6 or 8 waves per SIMD, all classes), whether the Poisson
// numbering chosen alone is kept or flipped (all classes), and the number of concurrent box
// groups.  The deposits and potentials it leaves are cleared or overwritten by the next
// scola_evolve (which starts from L-).
template <typename T>
void do_tune(scola_plan* p, void* ws, hipStream_t s, int reps) {
  const int n = p->cfg.n_steps;
  StepScalars sc = row_scalars(p, n - 1);
  sc.beta = 0.0;
  sc.alpha = 0.0;
  ParticleArgs<T> a = particle_args<T>(p, ws, sc);
  MeshArgs<T> ma = mesh_args<T>(p, ws, p->D1[n - 1]);
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "hipEventCreate");
  hip_check(hipEventCreate(&e1), "hipEventCreate");
  auto timed = [&](const std::function<void()>& f) {
    f();                                               // warm-up
    hip_check(hipEventRecord(e0, s), "hipEventRecord");
    for (int r = 0; r < reps; ++r) f();
    hip_check(hipEventRecord(e1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
    return ms;
  };
  const Maps& pm = p->part;
  for (size_t c = 0; c < pm.class_M.size(); ++c) {
    scola_class_schedule& cs = p->sched[c];
    float best = 1e30f;
    for (int remap : {1, 0}) {
      BlockMap b = class_map(pm, c);
      b.xcd_remap = remap;
      const float ms = timed([&] {
        hip_check(launch_particles<T>(a, kStep, b, 6, s), "tuning launch");
      });
      if (ms < best) {
        best = ms;
        cs.xcd_remap_particles = remap;
      }
    }
    // the Poisson passes on a cleared mass mesh (the tuning launches above left their
    // deposits in it), the two numberings timed in turn, twice each
    hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.rho)),
                              (int64_t)(rho_bytes(p) / 8), s), "zero rho");
    float total[2] = {0.0f, 0.0f};
    for (int round = 0; round < 2; ++round)
      for (int remap : {1, 0}) {
        cs.xcd_remap_mesh = remap;
        total[remap] += timed([&] { poisson_class(p, ma, c, false, s); });
      }
    cs.xcd_remap_mesh = total[1] <= total[0] ? 1 : 0;
  }
  // the particle kernel's occupancy, the Poisson passes' block numbering (as chosen above,
  // or flipped in every class) and the number of concurrent box groups, chosen together
  // from whole evolutions (eager): a choice that wins for one kernel alone can lose once
  // its launches share the GPU with other groups' kernels
  const std::vector<int> all = subset_list(p, nullptr, 0);
  const bool grouped = p->desc.size() >= 2 && p->cfg.schedule == SCOLA_BATCHED;
  const std::vector<int> group_choices = grouped ? std::vector<int>{1, 2, 4}
                                                 : std::vector<int>{p->groups};
  std::vector<int> mesh_alone(p->sched.size());
  for (size_t c = 0; c < p->sched.size(); ++c) mesh_alone[c] = p->sched[c].xcd_remap_mesh;
  float best = 1e30f;
  int occ_choice = 6, flip_choice = 0, group_choice = p->groups;
  for (int occ : {6, 8})
    for (int flip : {0, 1}) {
      for (size_t c = 0; c < p->sched.size(); ++c) {
        p->sched[c].waves_per_simd = occ;
        p->sched[c].xcd_remap_mesh = mesh_alone[c] ^ flip;
      }
      for (int G : group_choices) {
        p->groups = G;
        const float ms = timed([&] { do_evolve<T>(p, all, ws, s); });
        if (ms < best) {
          best = ms;
          occ_choice = occ;
          flip_choice = flip;
          group_choice = G;
        }
      }
    }
  for (size_t c = 0; c < p->sched.size(); ++c) {
    p->sched[c].waves_per_simd = occ_choice;
    p->sched[c].xcd_remap_mesh = mesh_alone[c] ^ flip_choice;
  }
  p->groups = group_choice;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.rho)),
                            (int64_t)(rho_bytes(p) / 8), s), "zero rho");
  hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped)),
                            3 * (int64_t)p->desc.size() + 1, s), "zero dropped");
  // the tuning launches leave extents and unfolded dropped mass in the hints
  hip_check(launch_zero_u32(reinterpret_cast<unsigned*>(ws_ptr(ws, p->lay.cells)),
                            (p->P / kBlock) * 4, s), "zero cell hints");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // namespace

namespace {

// Workspace of the monolithic periodic tCOLA run (byte offsets, 256-byte aligned).
struct TcolaLayout {
  size_t psi1, psi2, x_res, p_res, rho, phi, cbuf, phi1, phi2, outgrid, total;
};

TcolaLayout tcola_layout(const scola_plan* p) {
  const size_t R = p->is64 ? 8 : 4;
  const size_t N3 = (size_t)p->cfg.Np * p->cfg.Np * p->cfg.Np;
  const size_t No3 = (size_t)p->cfg.N_out * p->cfg.N_out * p->cfg.N_out;
  TcolaLayout l{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  l.psi1 = take(3 * N3 * R);
  l.psi2 = take(3 * N3 * R);
  l.x_res = take(3 * N3 * R);
  l.p_res = take(3 * N3 * R);
  l.rho = take(N3 * 8);
  l.phi = take(N3 * R);
  l.cbuf = take(N3 * 16);
  l.phi1 = take(N3 * 8);
  l.phi2 = take(N3 * 8);
  l.outgrid = take(No3 * 8);
  l.total = off;
  return l;
}

// Sec. 2.2: the full periodic box evolved by the same KDK schedule as the boxes.
template <typename T>
void do_tcola(scola_plan* p, const double* w, void* pos, void* mom, void* dens, void* rec_d,
              void* rec_p, void* ws, hipStream_t s) {
  const TcolaLayout l = tcola_layout(p);
  const int N = p->cfg.Np, n = p->cfg.n_steps;
  const int64_t N3 = (int64_t)N * N * N;
  SetupArgs sa = setup_args(p, w, ws);
  sa.cbuf = reinterpret_cast<double2*>(ws_ptr(ws, l.cbuf));
  sa.phi1 = reinterpret_cast<double*>(ws_ptr(ws, l.phi1));
  sa.phi2 = reinterpret_cast<double*>(ws_ptr(ws, l.phi2));
  hip_check(launch_setup_potentials(sa, s), "set-up potentials");
  TcolaArgs<T> a{};
  a.psi1 = reinterpret_cast<const T*>(ws_ptr(ws, l.psi1));
  a.psi2 = reinterpret_cast<const T*>(ws_ptr(ws, l.psi2));
  a.xres = reinterpret_cast<T*>(ws_ptr(ws, l.x_res));
  a.pres = reinterpret_cast<T*>(ws_ptr(ws, l.p_res));
  a.rho = reinterpret_cast<unsigned long long*>(ws_ptr(ws, l.rho));
  a.phi = reinterpret_cast<const T*>(ws_ptr(ws, l.phi));
  a.N = N;
  a.ng = p->ng;
  T* phi = reinterpret_cast<T*>(ws_ptr(ws, l.phi));
  hip_check(launch_tcola_setup<T>(a, sa.phi1, sa.phi2, s), "tCOLA set-up");
  hip_check(launch_zero_u64(a.rho, N3, s), "zero rho");
  int force = 0;
  auto poisson = [&]() {
    T* rd = rec_d ? reinterpret_cast<T*>(rec_d) + (size_t)force * N3 : nullptr;
    T* rp = rec_p ? reinterpret_cast<T*>(rec_p) + (size_t)force * N3 : nullptr;
    hip_check(launch_tcola_poisson<T>(a, sa.cbuf, phi, rd, rp, s), "tCOLA Poisson");
    ++force;
  };
  a.sc = StepScalars{};
  a.sc.D1 = p->D1[0];
  a.sc.D2 = p->D2[0];
  hip_check(launch_tcola_particles<T>(a, kInit, s), "tCOLA particles");
  poisson();
  for (int k = 0; k < n; ++k) {
    const bool need_force = k < n - 1 || p->cfg.want_momenta;
    a.sc = row_scalars(p, k);
    hip_check(launch_tcola_particles<T>(a, need_force ? kStep : kStepNoDeposit, s),
              "tCOLA particles");
    if (need_force) poisson();
  }
  if (p->cfg.want_momenta) {
    const double* f = &p->table[(size_t)n * 8];
    a.sc = StepScalars{};
    a.sc.beta = f[1];
    a.sc.D1 = f[2];
    a.sc.D2 = f[3];
    a.sc.c1 = f[4];
    a.sc.c2 = f[5];
    hip_check(launch_tcola_particles<T>(a, kFinalKick, s), "tCOLA final kick");
  }
  a.sc = StepScalars{};
  a.sc.D1 = p->D1[n];
  a.sc.D2 = p->D2[n];
  hip_check(launch_tcola_output<T>(a, reinterpret_cast<T*>(pos), reinterpret_cast<T*>(mom),
                                   reinterpret_cast<unsigned long long*>(ws_ptr(ws, l.outgrid)),
                                   reinterpret_cast<T*>(dens), p->cfg.N_out,
                                   p->cfg.L / p->cfg.Np, p->cfg.L, s),
            "tCOLA output");
}

}  // namespace

// Static device workspace of scola_forward_noalloc: one copy per GPU, held until the process
// ends.  In host code `scratch` is only a host-side handle of the symbol: its device address
// on a GPU is obtained once per device with hipGetSymbolAddress (with that device current)
// and only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[SCOLA_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call per device).
void* static_workspace(int device) {
  if (device < 0 || device >= kMaxDevices) fail(SCOLA_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256)
      fail(SCOLA_EDEVICE, "static workspace address is not 256-byte aligned");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

const char* scola_status_string(scola_status s) {
  switch (s) {
    case SCOLA_OK: return "SCOLA_OK";
    case SCOLA_EINVAL: return "SCOLA_EINVAL";
    case SCOLA_ENOMEM: return "SCOLA_ENOMEM";
    case SCOLA_EDEVICE: return "SCOLA_EDEVICE";
    case SCOLA_ESTATE: return "SCOLA_ESTATE";
    case SCOLA_EUNSUPPORTED: return "SCOLA_EUNSUPPORTED";
    case SCOLA_EOVERFLOW: return "SCOLA_EOVERFLOW";
  }
  return "unknown scola_status";
}

const char* scola_last_error(void) { return g_last_error.c_str(); }

scola_status scola_uniform_tiling(int32_t Np, int32_t tps, int32_t buffer, scola_tile* out,
                                  int32_t capacity) {
  return guarded([&] {
    if (Np < 1 || tps < 1 || Np % tps) fail(SCOLA_EINVAL, "Np must be a multiple of tiles_per_side");
    if (buffer < 0) fail(SCOLA_EINVAL, "buffer must be >= 0");
    if (!out || capacity < tps * tps * tps) fail(SCOLA_EINVAL, "output capacity too small");
    const int n = Np / tps;
    int i = 0;
    for (int x = 0; x < tps; ++x)
      for (int y = 0; y < tps; ++y)
        for (int z = 0; z < tps; ++z) {
          scola_tile& t = out[i++];
          t.core_lo[0] = x * n;
          t.core_lo[1] = y * n;
          t.core_lo[2] = z * n;
          t.core_n = n;
          t.buffer = buffer;
          t.mesh[0] = t.mesh[1] = t.mesh[2] = 0;
          t.a_f = 0.0;
        }
  });
}

scola_status scola_plan_create(const scola_config* cfg, const scola_cosmology* cosmo,
                               const scola_tile* tiles, int32_t n_tiles, scola_plan** out) {
  if (out) *out = nullptr;
  scola_plan* p = nullptr;
  scola_status st = guarded([&] {
    if (!cfg || !cosmo || !out) fail(SCOLA_EINVAL, "NULL argument");
    validate(*cfg, *cosmo, tiles, n_tiles);
    p = new scola_plan();
    p->cfg = *cfg;
    if (p->cfg.N_out == 0) p->cfg.N_out = cfg->Np;
    p->cosmo = *cosmo;
    p->is64 = cfg->precision == SCOLA_FP64;
    p->ng = p->cfg.fda_order > 0 ? p->cfg.fda_order / 2 : 1;
    p->N_lpt = p->cfg.N_lpt > 0 ? p->cfg.N_lpt : p->cfg.Np;
    p->tiles.assign(tiles, tiles + n_tiles);
    hip_check(hipGetDevice(&p->device), "hipGetDevice");
    p->bg = background_of(*cosmo);
    int64_t P = 0, G = 0, H = 0;
    for (int t = 0; t < n_tiles; ++t) {
      const scola_tile& s = tiles[t];
      TileDesc d{};
      d.M = s.core_n + 2 * s.buffer;
      for (int a = 0; a < 3; ++a) {
        d.origin[a] = s.core_lo[a] - s.buffer;
        d.core_lo[a] = s.buffer;
      }
      d.core_n = s.core_n;
      d.p_off = P;
      d.g_off = G;
      d.h_off = H;
      P += (int64_t)d.M * d.M * d.M;
      G += (int64_t)(d.M - 1) * (d.M - 1) * (d.M - 1);
      const int64_t Mp = d.M + 1 + 2 * p->ng;
      H += Mp * Mp * Mp;
      p->max_M = std::max(p->max_M, d.M);
      p->desc.push_back(d);
    }
    p->P = P;
    p->G = G;
    p->H = H;
    build_step_table(p);
    // time classes: cfg.a_f first, then every other final scale factor of a tile
    p->tclasses.clear();
    TimeClass tc0;
    tc0.a_f = cfg->a_f;
    tc0.table = p->table;
    tc0.D1 = p->D1;
    tc0.D2 = p->D2;
    p->tclasses.push_back(tc0);
    for (int t = 0; t < n_tiles; ++t) {
      const double af = tiles[t].a_f != 0.0 ? tiles[t].a_f : cfg->a_f;
      int c = -1;
      for (size_t i = 0; i < p->tclasses.size(); ++i)
        if (p->tclasses[i].a_f == af) c = (int)i;
      if (c < 0) {
        TimeClass tc;
        tc.a_f = af;
        scola_config ct = p->cfg;
        ct.a_f = af;
        compute_step_table(ct, p->bg, tc.table, tc.D1, tc.D2);
        c = (int)p->tclasses.size();
        p->tclasses.push_back(tc);
      }
      TileDesc& d = p->desc[t];
      d.tclass = c;
      d.D1f = p->tclasses[c].D1[cfg->n_steps];
      d.D2f = p->tclasses[c].D2[cfg->n_steps];
    }
    build_layout(p);
    if (p->is64)
      upload_tables<double>(p);
    else
      upload_tables<float>(p);
    build_maps(p->part, p->desc, [](const TileDesc& d) { return d.M * d.M * d.M / kBlock; });
    p->sched.clear();
    for (int M : p->part.class_M) p->sched.push_back(scola_class_schedule{M, 6, 1, 1});
    p->class_tiles.assign(p->part.class_M.size(), {});
    for (size_t c = 0; c < p->part.class_M.size(); ++c)
      for (size_t t = 0; t < p->desc.size(); ++t)
        if (p->desc[t].M == p->part.class_M[c] && p->desc[t].tclass == p->part.class_tc[c])
          p->class_tiles[c].push_back((int)t);
    build_maps(p->p1, p->desc, [](const TileDesc& d) { return d.M - 1; });
    // the pencil pass: chunks of consecutive pencils of the box's (M - 1)^2
    const int chunk = p->is64 ? pencil_chunk<double>() : pencil_chunk<float>();
    build_maps(p->p2, p->desc, [chunk](const TileDesc& d) {
      return ((d.M - 1) * (d.M - 1) + chunk - 1) / chunk;
    });
    // the interior x planes, then the 2 (ng + 1) shell planes
    const int ng = p->ng;
    build_maps(p->p3, p->desc, [ng](const TileDesc& d) { return d.M - 1 + 2 * (ng + 1); });
    upload_maps(p->part);
    upload_maps(p->p1);
    upload_maps(p->p2);
    upload_maps(p->p3);
    hip_check(hipMalloc(&p->d_barrier, 2 * sizeof(unsigned)), "hipMalloc(barrier)");
    hip_check(hipMalloc(&p->d_tiles, p->desc.size() * sizeof(TileDesc)), "hipMalloc(tiles)");
    hip_check(hipMemcpy(p->d_tiles, p->desc.data(), p->desc.size() * sizeof(TileDesc),
                        hipMemcpyHostToDevice), "hipMemcpy(tiles)");
    *out = p;
  });
  if (st != SCOLA_OK && p) scola_plan_destroy(p);
  return st;
}

scola_status scola_plan_destroy(scola_plan* p) {
  if (!p) return SCOLA_OK;
  free_maps(p->part);
  free_maps(p->p1);
  free_maps(p->p2);
  free_maps(p->p3);
  drop_graph(p);
  if (p->capture_stream) hipStreamDestroy(p->capture_stream);
  for (int i = 0; i < 3; ++i) {
    if (p->aux_stream[i]) hipStreamDestroy(p->aux_stream[i]);
    if (p->ev_join[i]) hipEventDestroy(p->ev_join[i]);
  }
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  if (p->d_tiles) hipFree(p->d_tiles);
  if (p->d_barrier) hipFree(p->d_barrier);
  if (p->d_twiddles) hipFree(p->d_twiddles);
  if (p->d_eigen) hipFree(p->d_eigen);
  if (p->d_sine) hipFree(p->d_sine);
  delete p;
  return SCOLA_OK;
}

scola_status scola_workspace_size(const scola_plan* p, size_t* bytes) {
  return guarded([&] {
    if (!p || !bytes) fail(SCOLA_EINVAL, "NULL argument");
    *bytes = p->lay.total;
  });
}

scola_status scola_workspace_layout(const scola_plan* p, scola_layout* out) {
  return guarded([&] {
    if (!p || !out) fail(SCOLA_EINVAL, "NULL argument");
    *out = p->lay;
  });
}

scola_status scola_setup(scola_plan* p, const double* w, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    if (!w) fail(SCOLA_EINVAL, "white noise is NULL");
    if (p->is64)
      do_setup<double>(p, w, ws, s);
    else
      do_setup<float>(p, w, ws, s);
    p->setup_ws = ws;
    p->forward_ws = nullptr;
  });
}

scola_status scola_evolve(scola_plan* p, const int32_t* subset, int32_t n_subset, void* ws,
                          hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    if (p->setup_ws != ws) fail(SCOLA_ESTATE, "scola_setup has not run on this workspace");
    const std::vector<int> tiles = subset_list(p, subset, n_subset);
    p->forward_ws = (p->cfg.checkpoint_every > 0 && tiles.size() == p->desc.size()) ? ws : nullptr;
    const bool graphable = p->use_graph && !p->persistent &&
                           p->cfg.schedule == SCOLA_BATCHED && tiles.size() == p->desc.size();
    if (graphable) {
      if (p->graph_ws != ws || p->graph_version != p->sched_version) {
        drop_graph(p);
        p->graph_ws = ws;
        p->graph_version = p->sched_version;
      }
      if (!p->evolve_exec && p->graph_eager_calls >= 1) {
        if (p->is64)
          capture_evolve<double>(p, tiles, ws);
        else
          capture_evolve<float>(p, tiles, ws);
      }
      if (p->evolve_exec) {
        hip_check(hipGraphLaunch(p->evolve_exec, s), "hipGraphLaunch");
        return;
      }
      ++p->graph_eager_calls;   // the first call runs eagerly (it also sets kernel attributes)
    }
    if (p->is64)
      do_evolve<double>(p, tiles, ws, s);
    else
      do_evolve<float>(p, tiles, ws, s);
  });
}

scola_status scola_evolve_overrides(scola_plan* p, const void* d_delta, const void* d_phi,
                                    void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    if (p->setup_ws != ws) fail(SCOLA_ESTATE, "scola_setup has not run on this workspace");
    const std::vector<int> tiles = subset_list(p, nullptr, 0);
    p->forward_ws = nullptr;
    if (p->is64)
      do_evolve<double>(p, tiles, ws, s, false, reinterpret_cast<const double*>(d_delta),
                        reinterpret_cast<const double*>(d_phi));
    else
      do_evolve<float>(p, tiles, ws, s, false, reinterpret_cast<const float*>(d_delta),
                       reinterpret_cast<const float*>(d_phi));
  });
}

scola_status scola_plan_tune(scola_plan* p, void* ws, hipStream_t s, int32_t reps) {
  return guarded([&] {
    check_ws(p, ws);
    if (p->setup_ws != ws) fail(SCOLA_ESTATE, "scola_setup has not run on this workspace");
    if (reps < 1 || reps > 1000) fail(SCOLA_EINVAL, "reps must be in [1, 1000]");
    p->forward_ws = nullptr;
    if (p->is64)
      do_tune<double>(p, ws, s, reps);
    else
      do_tune<float>(p, ws, s, reps);
    ++p->sched_version;
  });
}

scola_status scola_plan_set_graph(scola_plan* p, int32_t enable) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "null plan");
    p->use_graph = enable != 0;
    if (!p->use_graph) drop_graph(p);
  });
}

scola_status scola_plan_set_persistent(scola_plan* p, int32_t enable) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "null plan");
    if (enable && p->is64) fail(SCOLA_EUNSUPPORTED, "the persistent step is built for FP32 plans");
    if (enable && p->cfg.schedule != SCOLA_BATCHED)
      fail(SCOLA_EINVAL, "the persistent step needs the batched schedule");
    if (enable && p->ng != 1)
      fail(SCOLA_EUNSUPPORTED, "the persistent step is built for finite differences of order 2");
    p->persistent = enable != 0;
    drop_graph(p);
    ++p->sched_version;
  });
}

scola_status scola_plan_persistent(const scola_plan* p, hipStream_t s, int32_t* enabled,
                                   int32_t* grid, int32_t* barrier_failures) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "null plan");
    unsigned w[2] = {0, 0};
    hip_check(hipMemcpyAsync(w, p->d_barrier, sizeof(w), hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (enabled) *enabled = p->persistent ? 1 : 0;
    if (grid) *grid = p->persistent_grid;
    if (barrier_failures) *barrier_failures = (int32_t)w[1];
  });
}

scola_status scola_plan_concurrency(const scola_plan* p, int32_t* groups) {
  return guarded([&] {
    if (!p || !groups) fail(SCOLA_EINVAL, "null argument");
    *groups = p->groups;
  });
}

scola_status scola_plan_set_concurrency(scola_plan* p, int32_t groups) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "null plan");
    if (groups != 1 && groups != 2 && groups != 4) fail(SCOLA_EINVAL, "groups must be 1, 2 or 4");
    p->groups = groups;
    ++p->sched_version;
  });
}

scola_status scola_plan_schedule(const scola_plan* p, scola_class_schedule* out,
                                 int32_t capacity, int32_t* n_classes) {
  return guarded([&] {
    if (!p || !n_classes) fail(SCOLA_EINVAL, "null argument");
    const int nc = (int)p->sched.size();
    *n_classes = nc;
    if (!out) return;
    if (capacity < nc) fail(SCOLA_EINVAL, "capacity too small");
    for (int c = 0; c < nc; ++c) out[c] = p->sched[c];
  });
}

scola_status scola_plan_set_schedule(scola_plan* p, const scola_class_schedule* in,
                                     int32_t n_classes) {
  return guarded([&] {
    if (!p || !in) fail(SCOLA_EINVAL, "null argument");
    if (n_classes != (int)p->sched.size())
      fail(SCOLA_EINVAL, "n_classes must equal the number of box sizes of the plan");
    for (int c = 0; c < n_classes; ++c) {
      if (in[c].M != p->sched[c].M) fail(SCOLA_EINVAL, "class order or M does not match");
      if (in[c].waves_per_simd != 6 && in[c].waves_per_simd != 8)
        fail(SCOLA_EINVAL, "waves_per_simd must be 6 or 8");
      if ((in[c].xcd_remap_particles | in[c].xcd_remap_mesh) & ~1)
        fail(SCOLA_EINVAL, "xcd_remap flags must be 0 or 1");
    }
    for (int c = 0; c < n_classes; ++c) p->sched[c] = in[c];
    ++p->sched_version;
  });
}

scola_status scola_output(scola_plan* p, void* pos, void* mom, void* dens,
                          const int32_t* subset, int32_t n_subset, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    const std::vector<int> tiles = subset_list(p, subset, n_subset);
    if (dens && tiles.size() != p->desc.size())
      fail(SCOLA_EINVAL, "the density needs every tile (pass d_density = NULL with a subset)");
    if (mom && !p->cfg.want_momenta) fail(SCOLA_EINVAL, "d_mom needs cfg.want_momenta");
    if (p->is64)
      do_output<double>(p, pos, mom, dens, tiles, ws, s);
    else
      do_output<float>(p, pos, mom, dens, tiles, ws, s);
  });
}

scola_status scola_forward(scola_plan* p, const double* w, void* pos, void* mom, void* dens,
                           const int32_t* subset, int32_t n_subset, void* ws, hipStream_t s) {
  scola_status st = scola_setup(p, w, ws, s);
  if (st != SCOLA_OK) return st;
  st = scola_evolve(p, subset, n_subset, ws, s);
  if (st != SCOLA_OK) return st;
  return scola_output(p, pos, mom, dens, subset, n_subset, ws, s);
}

scola_status scola_forward_noalloc(scola_plan* p, const double* w, void* pos, void* mom,
                                   void* dens, hipStream_t s) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "plan is NULL");
    if (!w) fail(SCOLA_EINVAL, "white noise is NULL");
    if (p->lay.total > (size_t)SCOLA_STATIC_WORKSPACE_BYTES)
      fail(SCOLA_EINVAL, "the plan needs a workspace of " + std::to_string(p->lay.total) +
                             " bytes, more than the static workspace of " +
                             std::to_string((size_t)SCOLA_STATIC_WORKSPACE_BYTES) + " bytes");
    if (mom && !p->cfg.want_momenta) fail(SCOLA_EINVAL, "d_mom needs cfg.want_momenta");
    int dev = -1;
    hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (dev != p->device) fail(SCOLA_EINVAL, "current device differs from the plan's device");
    void* ws = static_workspace(dev);
    const std::vector<int> tiles = subset_list(p, nullptr, 0);
    if (p->is64) {
      do_setup<double>(p, w, ws, s);
      do_evolve<double>(p, tiles, ws, s, false);
      do_output<double>(p, pos, mom, dens, tiles, ws, s);
    } else {
      do_setup<float>(p, w, ws, s);
      do_evolve<float>(p, tiles, ws, s, false);
      do_output<float>(p, pos, mom, dens, tiles, ws, s);
    }
    // no caller workspace was touched, so their call-order state stands
  });
}

scola_status scola_backward(scola_plan* p, const void* grad_density, double* grad_w, void* ws,
                            hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    if (!grad_density || !grad_w) fail(SCOLA_EINVAL, "NULL gradient buffer");
    if (p->cfg.checkpoint_every <= 0)
      fail(SCOLA_ESTATE, "the plan was created with checkpoint_every = 0 (no reverse mode)");
    if (p->forward_ws != ws)
      fail(SCOLA_ESTATE, "scola_backward needs a full scola_forward on this workspace first");
    if (p->tclasses.size() > 1)
      fail(SCOLA_EUNSUPPORTED, "the reverse mode needs one final scale factor for all tiles");
    if (p->ng != 1)
      fail(SCOLA_EUNSUPPORTED, "the reverse mode is built for finite differences of order 2");
    if (p->N_lpt != p->cfg.Np)
      fail(SCOLA_EUNSUPPORTED, "the reverse mode is built for an LPT grid of Np nodes per side");
    if (p->is64)
      do_backward<double>(p, reinterpret_cast<const double*>(grad_density), grad_w, ws, s);
    else
      do_backward<float>(p, reinterpret_cast<const float*>(grad_density), grad_w, ws, s);
    p->forward_ws = nullptr;   // the particle state now belongs to the first segment
  });
}

scola_status scola_op_deposit(scola_plan* p, double D1, double D2, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    p->forward_ws = nullptr;
    hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.rho)),
                              (int64_t)(rho_bytes(p) / 8), s), "zero rho");
    hip_check(launch_zero_u64(reinterpret_cast<unsigned long long*>(ws_ptr(ws, p->lay.dropped)),
                              3 * (int64_t)p->desc.size() + 1, s), "zero dropped");
    StepScalars sc{};
    sc.D1 = D1;
    sc.D2 = D2;
    if (p->is64) {
      Runner<double> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(kDepositOnly, sc);
    } else {
      Runner<float> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(kDepositOnly, sc);
      fold_drops(p, ws, s);
    }
  });
}

scola_status scola_op_poisson(scola_plan* p, double D1_bc, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    p->forward_ws = nullptr;
    if (p->is64) {
      Runner<double> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.poisson(D1_bc);
    } else {
      Runner<float> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.poisson(D1_bc);
    }
  });
}

scola_status scola_op_step(scola_plan* p, double beta, double alpha, double D1, double D2,
                           double D1n, double D2n, int32_t deposit, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    p->forward_ws = nullptr;
    StepScalars sc{};
    sc.beta = beta;
    sc.alpha = alpha;
    sc.D1 = D1;
    sc.D2 = D2;
    sc.D1n = D1n;
    sc.D2n = D2n;
    const int mode = deposit ? kStep : kStepNoDeposit;
    if (p->is64) {
      Runner<double> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(mode, sc);
    } else {
      Runner<float> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(mode, sc);
      if (deposit) fold_drops(p, ws, s);
    }
  });
}

scola_status scola_op_final_kick(scola_plan* p, double beta, double D1, double D2, double c1,
                                 double c2, void* ws, hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    p->forward_ws = nullptr;
    StepScalars sc{};
    sc.beta = beta;
    sc.D1 = D1;
    sc.D2 = D2;
    sc.c1 = c1;
    sc.c2 = c2;
    if (p->is64) {
      Runner<double> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(kFinalKick, sc);
    } else {
      Runner<float> r{p, ws, s, subset_list(p, nullptr, 0), true};
      r.particles(kFinalKick, sc);
    }
  });
}

scola_status scola_step_table(const scola_plan* p, double* rows, int32_t cap) {
  return guarded([&] {
    if (!p || !rows) fail(SCOLA_EINVAL, "NULL argument");
    if (cap < p->cfg.n_steps + 1) fail(SCOLA_EINVAL, "rows_capacity < n_steps + 1");
    std::memcpy(rows, p->table.data(), p->table.size() * sizeof(double));
  });
}

scola_status scola_power_spectrum(const scola_plan* p, const double* k, double* out, int32_t n) {
  return guarded([&] {
    if (!p || (n > 0 && (!k || !out))) fail(SCOLA_EINVAL, "NULL argument");
    for (int i = 0; i < n; ++i) out[i] = p->bg.power(k[i]);
  });
}

scola_status scola_schedule_table(const scola_config* cfg, const scola_cosmology* cosmo,
                                  double* rows, int32_t cap) {
  return guarded([&] {
    if (!cfg || !cosmo || !rows) fail(SCOLA_EINVAL, "NULL argument");
    if (cfg->n_steps < 1 || !(cfg->a_i > 0 && cfg->a_i < cfg->a_f))
      fail(SCOLA_EINVAL, "need n_steps >= 1 and 0 < a_i < a_f");
    if (cap < cfg->n_steps + 1) fail(SCOLA_EINVAL, "rows_capacity < n_steps + 1");
    Background bg = background_of(*cosmo);
    std::vector<double> table, D1, D2;
    compute_step_table(*cfg, bg, table, D1, D2);
    std::memcpy(rows, table.data(), table.size() * sizeof(double));
  });
}

scola_status scola_linear_power(const scola_cosmology* cosmo, const double* k, double* out,
                                int32_t n) {
  return guarded([&] {
    if (!cosmo || (n > 0 && (!k || !out))) fail(SCOLA_EINVAL, "NULL argument");
    Background bg = background_of(*cosmo);
    for (int i = 0; i < n; ++i) out[i] = bg.power(k[i]);
  });
}

scola_status scola_tcola_workspace_size(const scola_plan* p, size_t* bytes) {
  return guarded([&] {
    if (!p || !bytes) fail(SCOLA_EINVAL, "NULL argument");
    *bytes = tcola_layout(p).total;
  });
}

scola_status scola_tcola_forward(scola_plan* p, const double* w, void* pos, void* mom,
                                 void* dens, void* rec_delta, void* rec_phi, void* ws,
                                 hipStream_t s) {
  return guarded([&] {
    check_ws(p, ws);
    if (!w) fail(SCOLA_EINVAL, "white noise is NULL");
    if (mom && !p->cfg.want_momenta) fail(SCOLA_EINVAL, "d_mom needs cfg.want_momenta");
    if (p->N_lpt != p->cfg.Np)
      fail(SCOLA_EUNSUPPORTED, "tCOLA is built for an LPT grid of Np nodes per side");
    if (p->is64)
      do_tcola<double>(p, w, pos, mom, dens, rec_delta, rec_phi, ws, s);
    else
      do_tcola<float>(p, w, pos, mom, dens, rec_delta, rec_phi, ws, s);
  });
}

scola_status scola_mass_alarm(const scola_plan* p, const void* ws, hipStream_t s,
                              int64_t* near_limit, int64_t* wrapped) {
  return guarded([&] {
    check_ws(p, const_cast<void*>(ws));
    const size_t nt = p->desc.size();
    int64_t near = 0, wraps = 0;
    if (!p->is64) {
      // [dropped per tile][near-limit][found per tile][deposits per tile]
      std::vector<uint64_t> c(3 * nt + 1);
      hip_check(hipMemcpyAsync(c.data(), static_cast<const char*>(ws) + p->lay.dropped,
                               c.size() * 8, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      near = (int64_t)c[nt];
      const int bits = MeshFixed<float>::bits;
      for (size_t t = 0; t < nt; ++t) {
        const uint64_t M = (uint64_t)p->desc[t].M;
        const uint64_t expect = c[2 * nt + 1 + t] * (M * M * M) << bits;
        const uint64_t seen = c[t] + c[nt + 1 + t];
        // every deposit has been read by a Poisson pass: the deficit is whole 2^32 units
        if (seen > expect || ((expect - seen) & 0xffffffffull))
          fail(SCOLA_ESTATE, "the mass counters are inconsistent: a deposit has not been "
                             "followed by its Poisson pass (or the workspace is not the one "
                             "the last evolution ran on)");
        wraps += (int64_t)((expect - seen) >> 32);
      }
    }
    if (near_limit) *near_limit = near;
    if (wrapped) *wrapped = wraps;
    if (wraps > 0)
      fail(SCOLA_EOVERFLOW, std::to_string(wraps) + " node mass(es) wrapped the 32-bit "
                            "fixed-point range (more than 2048 particles on one node): the "
                            "densities and forces of this run are invalid; use an FP64 plan");
  });
}

scola_status scola_plan_info(const scola_plan* p, int32_t* n_tiles, int64_t* n_particles,
                             double* r, double* pp) {
  return guarded([&] {
    if (!p) fail(SCOLA_EINVAL, "NULL plan");
    const double np3 = (double)p->cfg.Np * p->cfg.Np * p->cfg.Np;
    if (n_tiles) *n_tiles = (int32_t)p->desc.size();
    if (n_particles) *n_particles = p->P;
    if (r) *r = (double)p->P / np3;
    if (pp) *pp = np3 * p->desc.size() / (double)p->P;
  });
}

}  // extern "C"
