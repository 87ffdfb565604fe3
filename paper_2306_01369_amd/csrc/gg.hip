// Host side of libgg: the C ABI declared in include/gg.h, argument checks,
// device buffers, kinematic body poses, and the per-step launch sequence.
#include "gg.h"
#include "kernels.hip.h"
#include "adjoint.hip.h"
#include "observe.hip.h"
#include "fused.hip.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>
#include <mutex>

// Workspace of gg_goal_reward_noalloc: one copy per GPU, held until the process
// ends; every call on a GPU shares it.
constexpr size_t kNoAllocScratchBytes = (size_t)2 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

thread_local std::string g_detail;

gg_status fail(gg_status s, const std::string& msg) {
  g_detail = msg;
  return s;
}

struct HostBody {
  int32_t env, shape;
  float params[4];
  double R[9], t[3], nu[3], om[3];
  int32_t grid = -1;  // GG_GRID: index of the registered grid
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool finite3(const float* a) { return std::isfinite(a[0]) && std::isfinite(a[1]) && std::isfinite(a[2]); }

// Upper bound on how many spheres of radius >= r_min can touch one sphere of
// radius r_max: caps of half-angle asin(r_min / (r_max + r_min)) cannot
// overlap on the unit sphere, so N <= 2 / (1 - cos theta); 25% margin for
// overlapping (compressed) neighbours.
int contact_bound(double r_min, double r_max) {
  double s = r_min / (r_max + r_min);
  double c = std::sqrt(std::max(0.0, 1.0 - s * s));
  double N = 2.0 / (1.0 - c);
  return (int)std::ceil(1.25 * N);
}

// Mean particles per occupied cell (cells of edge 1/inv_c; environments
// overlapping in space count together, which only matters for this estimate).
double particles_per_cell(const std::vector<float>& x, int64_t n, float inv_c) {
  if (n == 0) return 1.0;
  size_t cap = 1;
  while (cap < (size_t)n * 2) cap <<= 1;
  std::vector<uint64_t> table(cap, ~0ull);
  int64_t occupied = 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t key = 0;
    for (int a = 0; a < 3; ++a)
      key = key * 2097143ull + (uint64_t)(int64_t)std::nearbyint(x[3 * i + a] * inv_c) + (1ull << 40);
    uint64_t h = key * 0x9E3779B97F4A7C15ull;
    size_t slot = (size_t)(h >> 20) & (cap - 1);
    while (table[slot] != ~0ull && table[slot] != key) slot = (slot + 1) & (cap - 1);
    if (table[slot] == ~0ull) {
      table[slot] = key;
      ++occupied;
    }
  }
  return (double)n / (double)std::max<int64_t>(1, occupied);
}

// Detection launch shape from the particle count and the particles per cell:
// the workgroup size (256 threads for large beds, 128 otherwise, so small
// beds still spread over several workgroups), the largest Z-order node whose
// particles fit one workgroup, and an LDS budget for the node's box
// plus a one-cell halo and one cell of drift.  Only locality and work
// decomposition depend on it, never results.
void default_tile(int64_t n, double ppc, gg_params& p) {
  if (p.tile_threads == 0) p.tile_threads = n >= (1 << 18) ? 256 : 128;
  // lanes per particle shorten the sweeps' dependent-load chains where they,
  // not bandwidth, bound a sweep: four up to 2^17 particles (-26..31% per step
  // at 4k..64k), two up to 2^19; bandwidth-bound large beds keep one lane
  if (p.pja_lanes == 0) p.pja_lanes = n < (1 << 17) ? 4 : (n < (1 << 19) ? 2 : 1);
  if (p.tile_node_shift == 0) {
    int shift = 1;
    while (shift < 12 && ppc * (double)(1 << (shift + 1)) <= (double)p.tile_threads) ++shift;
    p.tile_node_shift = shift;
  }
  const int sh = p.tile_node_shift;
  const int dx = 1 << ((sh + 2) / 3), dy = 1 << ((sh + 1) / 3), dz = 1 << (sh / 3);
  const int cells = (dx + 3) * (dy + 3) * (dz + 3);
  if (p.tile_max_cells == 0) p.tile_max_cells = std::min(cells, 4096);
  if (p.tile_max_stage == 0)
    p.tile_max_stage = std::min(2048, (int)std::ceil(p.tile_max_cells * (ppc + 0.6) * 1.1));
}

// Exp(dt [om]x) R by Rodrigues' formula, t += dt nu (double precision).
void advance_pose(HostBody& B, double dt) {
  for (int a = 0; a < 3; ++a) B.t[a] += dt * B.nu[a];
  double w[3] = {B.om[0] * dt, B.om[1] * dt, B.om[2] * dt};
  double th = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
  if (th == 0.0) return;
  double k[3] = {w[0] / th, w[1] / th, w[2] / th};
  double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  double s = std::sin(th), c1 = 1.0 - std::cos(th);
  double E[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double kk = 0;
      for (int m = 0; m < 3; ++m) kk += K[3 * r + m] * K[3 * m + c];
      E[3 * r + c] = (r == c ? 1.0 : 0.0) + s * K[3 * r + c] + c1 * kk;
    }
  double Rn[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double acc = 0;
      for (int m = 0; m < 3; ++m) acc += E[3 * r + m] * B.R[3 * m + c];
      Rn[3 * r + c] = acc;
    }
  std::memcpy(B.R, Rn, sizeof(Rn));
}

// grid: the registered grid of a GG_GRID body (else nullptr); values: the
// device copy of all grids' values.
ggk::DevBody to_dev(const HostBody& B, const gg_grid* grid, const float* values, float r_max) {
  ggk::DevBody d{};
  d.shape = B.shape;
  d.env = B.env;
  for (int q = 0; q < 4; ++q) d.params[q] = B.params[q];
  for (int q = 0; q < 9; ++q) {
    d.R[q] = (float)B.R[q];
    d.Rd[q] = B.R[q];
  }
  for (int q = 0; q < 3; ++q) {
    d.t[q] = (float)B.t[q];
    d.nu[q] = (float)B.nu[q];
    d.om[q] = (float)B.om[q];
    d.td[q] = B.t[q];
    d.nud[q] = B.nu[q];
    d.omd[q] = B.om[q];
  }
  // world box of the body's points, for the detection cull (planes are unbounded)
  double blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
  bool bounded = true;
  if (B.shape == GG_BOX) {
    for (int r = 0; r < 3; ++r) {
      double e = 0;
      for (int c = 0; c < 3; ++c) e += std::fabs(B.R[3 * r + c]) * (double)B.params[c];
      blo[r] = B.t[r] - e;
      bhi[r] = B.t[r] + e;
    }
  } else if (B.shape == GG_CAPSULE) {
    for (int r = 0; r < 3; ++r) {
      const double e = std::fabs(B.R[3 * r + 2]) * (double)B.params[1] + (double)B.params[0];
      blo[r] = B.t[r] - e;
      bhi[r] = B.t[r] + e;
    }
  } else if (B.shape == GG_GRID && grid) {
    const double ext[3] = {(grid->nx - 1) / (double)grid->inv_spacing, (grid->ny - 1) / (double)grid->inv_spacing,
                           (grid->nz - 1) / (double)grid->inv_spacing};
    for (int r = 0; r < 3; ++r) {
      double c0 = B.t[r], e = 0;
      for (int c = 0; c < 3; ++c) {
        const double mid = (double)grid->origin[c] + 0.5 * ext[c];
        c0 += B.R[3 * r + c] * mid;
        e += std::fabs(B.R[3 * r + c]) * 0.5 * ext[c];
      }
      blo[r] = c0 - e;
      bhi[r] = c0 + e;
    }
  } else {
    bounded = false;
  }
  if (bounded) {
    d.cull = 1;
    for (int r = 0; r < 3; ++r) {
      // r_max plus a margin far above the rounding of the binary32 decision
      const double m = (double)r_max + 1e-4 + 1e-5 * std::max(std::fabs(blo[r]), std::fabs(bhi[r]));
      d.lo[r] = (float)(blo[r] - m);
      d.hi[r] = (float)(bhi[r] + m);
    }
  }
  if (grid) {
    d.gv = values + grid->offset;
    d.gn[0] = grid->nx;
    d.gn[1] = grid->ny;
    d.gn[2] = grid->nz;
    for (int q = 0; q < 3; ++q) d.go[q] = grid->origin[q];
    d.gih = grid->inv_spacing;
  }
  return d;
}

template <typename T>
hipError_t dev_alloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

hipError_t dev_alloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  return hipMalloc(p, bytes == 0 ? 16 : bytes);
}

}  // namespace

struct gg_sim {
  gg_params p{};
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool failed = false;

  int64_t n = 0;
  int32_t n_envs = 1;
  std::vector<int64_t> env_off;
  std::vector<int32_t> env_nh, env_boff;    // Eq. (6) table per env (the reported cell index)
  std::vector<int32_t> env_tblk, env_toff;  // internal bucket table per env (blocks of 64 buckets)
  int64_t n_buckets = 0;                    // internal buckets in all
  float cell = 0, inv_c = 0, r_max = 0, r_min = 0;
  int K = 0, K_pp = 0;
  int64_t n_pad = 0;

  std::vector<HostBody> bodies;
  std::vector<int32_t> body_lo, body_hi;
  std::vector<gg_grid> grids;       // registered SDF grids (gg_set_grids)
  float* d_grid_values = nullptr;   // their values, device copy

  // device buffers.  Real-valued state is V4<R> / R of the build's precision
  // (fp64: double), so those buffers are untyped here.
  bool fp64 = false;
  size_t es = 4, es4 = 16;                             // bytes of R and of V4<R>
  void *x = nullptr, *v = nullptr, *wa = nullptr, *wb = nullptr, *dv = nullptr;
  void *x2 = nullptr, *v2 = nullptr;                   // permutation targets
  int32_t *orig = nullptr, *orig2 = nullptr;            // caller index of each internal slot
  unsigned long long *mk[2] = {nullptr, nullptr};      // Z-order keys (radix ping-pong)
  int32_t *mv[2] = {nullptr, nullptr};                 // permutation values
  int32_t *rs_hist = nullptr, *rs_bsum = nullptr;      // radix histograms and their scan
  int rs_nb = 0, rs_passes = 0;
  int det_grid = 2048;  // detection workgroups: what the device holds at once (occupancy API)
  int fused_grid = 0;   // GG_FLAG_FUSED: workgroups of the cooperative step kernel (all resident)
  bool small_table = false;  // bucket table built by one workgroup (k_bucket_small)
  // detection items taken from per-XCD work queues rather than in fixed
  // contiguous shares (the fused step kernel keeps fixed shares)
  bool det_queue = false;
  void* xs = nullptr;                                  // bucket-ordered positions
  int32_t* os = nullptr;                               // bucket-ordered original indices
  int32_t *it_f = nullptr, *it_e = nullptr, *it_first = nullptr, *it_g = nullptr, *it_h = nullptr;
  int32_t *item_start = nullptr, *it_bsum = nullptr;
  int64_t steps_global = 0;
  int32_t *h = nullptr, *rank = nullptr, *counts = nullptr, *bstart = nullptr, *bsum = nullptr;
  int32_t *sidx = nullptr, *ncon = nullptr, *partner = nullptr;
  int K_floor = 0;   // automatic capacity: the largest a step has needed
  bool imp_rows = false;   // the last step's impulses lie in jagged rows (one lane per particle)
  void* imass = nullptr;  // 1/m_i in the internal order (written by detection, R)
  void *Px = nullptr, *Py = nullptr, *Pz = nullptr, *Psi = nullptr;
  int32_t* h6 = nullptr;  // Eq. (6) cell index of each particle at the last detection
  int32_t *d_env_tblk = nullptr, *d_env_toff = nullptr;
  int32_t *env_of = nullptr, *d_env_nh = nullptr, *d_env_boff = nullptr, *d_body_lo = nullptr,
          *d_body_hi = nullptr;
  ggk::DevBody* d_bodies = nullptr;
  int64_t d_bodies_cap = 0;
  ggk::DevBody* h_bodies = nullptr;  // pinned staging
  int64_t h_bodies_cap = 0;
  ggk::Ctl* ctl = nullptr;
  ggk::Ctl* h_ctl = nullptr;  // pinned
  ggk::DetPart* det_part = nullptr;  // per-workgroup detection counts (max of both detection grids)
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  std::vector<hipEvent_t> events;

  gg_stats stats{};
  bool contacts_valid = false;
  std::vector<HostBody> pose_hist;  // scratch for gg_step
  // record of the last differentiable call (GG_FLAG_TAPE)
  bool tape_ok = false;
  int tape_steps = 0;
  std::vector<HostBody> tape_poses;   // (steps + 1) x bodies, double precision
  std::vector<float> tape_twists;     // steps x bodies x 6
  void* ck = nullptr;                 // checkpoints: per segment x then v (V4<R>)
  size_t ck_cap = 0;
  unsigned long long* d_counts = nullptr;  // per step (pairs, body contacts) of a differentiable call
  size_t d_counts_cap = 0;
  std::vector<unsigned long long> tape_counts;
  // captured launch sequences of gg_step (GG_FLAG_GRAPH)
  struct Graph {
    hipGraphExec_t exec = nullptr;
    int n_steps = 0, nb = 0;
    int64_t phase = 0;
    uint64_t epoch = 0;
    void *x0 = nullptr, *x1 = nullptr, *v1 = nullptr;
    int32_t* o1 = nullptr;
    uint64_t used = 0;
  };
  std::vector<Graph> graphs;
  uint64_t epoch = 1;  // bumped whenever a buffer a captured launch names is reallocated
  uint64_t graph_clock = 0;
  hipStream_t cap_stream = nullptr;
  // observations (gg_render_depth, gg_goal_reward); sized on first use
  ggk::DevCamera* d_cams = nullptr;
  int64_t d_cams_cap = 0;
  ggk::DevPlane* d_planes = nullptr;
  int64_t d_planes_cap = 0;
  float* obs_img = nullptr;           // depth staging for host destinations
  int64_t obs_img_cap = 0;
  int32_t *d_chunks = nullptr, *d_env_chunk = nullptr, *d_env_count = nullptr, *d_part_n = nullptr;
  double* d_part_d = nullptr;
  float* d_boxes = nullptr;
  double* d_reward = nullptr;
  int64_t* d_inside = nullptr;
  int32_t n_chunks = 0;
};

namespace {

// Device memory in use (whole device) into the peak statistic.
void sample_memory(gg_sim* s) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) == hipSuccess)
    s->stats.device_bytes_peak = std::max<int64_t>(s->stats.device_bytes_peak, (int64_t)(tot - fr));
}

gg_status hip_fail(gg_sim* s, hipError_t e, const char* what) {
  if (s) s->failed = true;
  return fail(GG_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(sim, expr)                              \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return hip_fail(sim, _e, #expr); \
  } while (0)

gg_status check_params(const gg_params* p) {
  if (!p) return fail(GG_ERR_INVALID, "params is NULL");
  if (!(p->dt > 0.0f) || !std::isfinite(p->dt)) return fail(GG_ERR_INVALID, "dt must be finite and > 0");
  if (!(p->alpha >= 0.0f) || !std::isfinite(p->alpha)) return fail(GG_ERR_INVALID, "alpha must be finite and >= 0");
  if (!(p->mu >= 0.0f) || !std::isfinite(p->mu)) return fail(GG_ERR_INVALID, "mu must be finite and >= 0");
  if (!finite3(p->gravity)) return fail(GG_ERR_INVALID, "gravity must be finite");
  if (p->n_iters < 1 || p->n_iters > 100000) return fail(GG_ERR_INVALID, "n_iters must be in [1, 100000]");
  if (!(p->cell_size >= 0.0f) || !std::isfinite(p->cell_size)) return fail(GG_ERR_INVALID, "cell_size must be finite and >= 0");
  if (p->hash_size < 0 || p->hash_size > (int64_t)1 << 30) return fail(GG_ERR_INVALID, "hash_size must be in [0, 2^30]");
  if (!(p->relax >= 0.0f && p->relax <= 2.0f)) return fail(GG_ERR_INVALID, "relax must be in [0, 2] (0 = default 1)");
  if (p->mass_split != 0 && p->mass_split != 1) return fail(GG_ERR_INVALID, "mass_split must be 0 or 1");
  if (p->checkpoint_every < 0) return fail(GG_ERR_INVALID, "checkpoint_every must be >= 0");
  if (p->max_contacts_per_particle < 0 || p->max_contacts_per_particle > 256)
    return fail(GG_ERR_INVALID, "max_contacts_per_particle must be in [0, 256]");
  if (p->precision != 0 && p->precision != 1) return fail(GG_ERR_INVALID, "precision must be 0 or 1");
  if (!(p->density >= 0.0f) || !std::isfinite(p->density)) return fail(GG_ERR_INVALID, "density must be finite and >= 0");
  if (p->flags & ~(GG_FLAG_PROFILE | GG_FLAG_DIAGNOSTICS | GG_FLAG_TAPE | GG_FLAG_GRAPH | GG_FLAG_FUSED))
    return fail(GG_ERR_INVALID, "unknown flag bits");
  if ((p->flags & GG_FLAG_FUSED) && (p->flags & GG_FLAG_TAPE))
    return fail(GG_ERR_INVALID, "GG_FLAG_FUSED does not record the sweeps for GG_FLAG_TAPE");
  if (p->tile_max_cells < 0 || p->tile_max_cells > 4096) return fail(GG_ERR_INVALID, "tile_max_cells must be in [0, 4096]");
  if (p->tile_max_stage < 0 || p->tile_max_stage > 2048) return fail(GG_ERR_INVALID, "tile_max_stage must be in [0, 2048]");
  if (p->tile_node_shift < 0 || p->tile_node_shift > 15) return fail(GG_ERR_INVALID, "tile_node_shift must be in [0, 15]");
  if (p->pja_lanes != 0 && p->pja_lanes != 1 && p->pja_lanes != 2 && p->pja_lanes != 4)
    return fail(GG_ERR_INVALID, "pja_lanes must be 0, 1, 2 or 4");
  if (!std::isfinite(p->cyclic_z[0]) || !std::isfinite(p->cyclic_z[1]))
    return fail(GG_ERR_INVALID, "cyclic_z must be finite");
  if (p->tile_threads != 0 && p->tile_threads != 64 && p->tile_threads != 128 && p->tile_threads != 256)
    return fail(GG_ERR_INVALID, "tile_threads must be 0, 64, 128 or 256");
  if (p->device < 0) return fail(GG_ERR_INVALID, "device must be >= 0");
  return GG_OK;
}

gg_status ensure_tmp(gg_sim* s, size_t bytes) {
  if (bytes <= s->tmp_bytes) return GG_OK;
  if (s->tmp) HIPCHK(s, hipFree(s->tmp));
  s->tmp = nullptr;
  s->tmp_bytes = 0;
  hipError_t e = hipMalloc(&s->tmp, bytes);
  if (e != hipSuccess) return fail(GG_ERR_OOM, "readout buffer allocation failed");
  s->tmp_bytes = bytes;
  return GG_OK;
}

// Contact-table slots are indexed in 32-bit arithmetic on the device
// (ell_slot): n_pad * K must stay below 2^31.
constexpr int64_t kMaxSlots = ((int64_t)1 << 31) - 1;

bool slots_fit(int64_t n_pad, int K) { return n_pad * (int64_t)K <= kMaxSlots; }

gg_status slots_error(int64_t n_pad, int K) {
  return fail(GG_ERR_INVALID, "contact table of " + std::to_string(n_pad) + " x " + std::to_string(K) +
                                  " slots exceeds 2^31 - 1 (fewer particles or a smaller contact capacity)");
}

// (Re)allocate the contact table for capacity K per particle.
gg_status ensure_ell(gg_sim* s, int K) {
  if (K == s->K && s->partner) return GG_OK;
  if (!slots_fit(s->n_pad, K)) return slots_error(s->n_pad, K);
  (void)hipFree(s->partner); (void)hipFree(s->Px); (void)hipFree(s->Py); (void)hipFree(s->Pz);
  (void)hipFree(s->Psi);
  s->partner = nullptr; s->Px = s->Py = s->Pz = s->Psi = nullptr;
  size_t slots = (size_t)s->n_pad * (size_t)K;
  if (dev_alloc(&s->partner, slots) != hipSuccess || dev_alloc_bytes(&s->Px, slots * s->es) != hipSuccess ||
      dev_alloc_bytes(&s->Py, slots * s->es) != hipSuccess || dev_alloc_bytes(&s->Pz, slots * s->es) != hipSuccess ||
      dev_alloc_bytes(&s->Psi, slots * s->es) != hipSuccess)
    return fail(GG_ERR_OOM, "contact table allocation failed");
  s->K = K;
  s->stats.capacity = K;
  s->contacts_valid = false;
  ++s->epoch;
  sample_memory(s);
  return GG_OK;
}

// Contact capacity per particle: the explicit one, else the packing bound of
// the radius ratio plus the largest number of bodies of one environment.
int capacity_for(const gg_params& p, int K_pp, int nb_env) {
  if (p.max_contacts_per_particle > 0) return p.max_contacts_per_particle;
  int K = K_pp + nb_env;
  K = (K + 1) & ~1;
  return std::min(K, 256);
}

// The capacity limit: the explicit capacity, else the packing bound.
int bound_K(const gg_sim* s) {
  int nb_env = 0;
  for (int e = 0; e < s->n_envs; ++e) nb_env = std::max(nb_env, s->body_hi[e] - s->body_lo[e]);
  return capacity_for(s->p, s->K_pp, nb_env);
}

// Particles of a bed seldom come near the packing bound (a polydisperse bed
// of radii 1-4 mm: 22 contacts at most against a bound of 132), so the
// automatic capacity starts here, plus the bodies, and grows when a step
// needs more (gg_step); it never shrinks below what a step has needed.
constexpr int kAutoCapacity = 24;

// The capacity to allocate: the explicit one, else the automatic one.
int compute_K(const gg_sim* s) {
  const int bound = bound_K(s);
  if (s->p.max_contacts_per_particle > 0) return bound;
  int nb_env = 0;
  for (int e = 0; e < s->n_envs; ++e) nb_env = std::max(nb_env, s->body_hi[e] - s->body_lo[e]);
  const int start = (kAutoCapacity + nb_env + 1) & ~1;
  return std::min(bound, std::max(start, s->K_floor));
}

ggk::EnvTables env_tables(const gg_sim* s) {
  ggk::EnvTables t;
  t.env_of = s->env_of;
  t.nh = s->d_env_nh;
  t.boff = s->d_env_boff;
  t.tblk = s->d_env_tblk;
  t.toff = s->d_env_toff;
  t.body_lo = s->d_body_lo;
  t.body_hi = s->d_body_hi;
  return t;
}

void free_all(gg_sim* s) {
  void* bufs[] = {s->x, s->v, s->wa, s->wb, s->dv, s->x2, s->v2, s->orig, s->orig2, s->mk[0], s->mk[1],
                  s->mv[0], s->mv[1], s->rs_hist, s->rs_bsum, s->xs, s->os, s->it_f, s->it_e, s->it_first,
                  s->it_g, s->it_h, s->item_start, s->it_bsum, s->ck, s->d_counts, s->h, s->rank, s->counts, s->bstart, s->bsum,
                  s->sidx, s->ncon, s->imass, s->partner, s->Px, s->Py, s->Pz, s->Psi, s->env_of, s->d_env_nh,
                  s->d_env_boff, s->d_body_lo, s->d_body_hi, s->d_bodies, s->ctl, s->det_part, s->tmp, s->h6,
                  s->d_env_tblk, s->d_env_toff, s->d_grid_values, s->d_cams, s->d_planes, s->obs_img,
                  s->d_chunks, s->d_env_chunk, s->d_env_count, s->d_part_n, s->d_part_d, s->d_boxes,
                  s->d_reward, s->d_inside};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  if (s->h_bodies) (void)hipHostFree(s->h_bodies);
  if (s->h_ctl) (void)hipHostFree(s->h_ctl);
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  s->events.clear();
  for (auto& G : s->graphs) (void)hipGraphExecDestroy(G.exec);
  s->graphs.clear();
  if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

gg_status copy_in(const void* src, size_t bytes, gg_mem where, void* host_dst) {
  if (bytes == 0) return GG_OK;
  if (where == GG_MEM_HOST) {
    std::memcpy(host_dst, src, bytes);
    return GG_OK;
  }
  hipError_t e = hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(GG_ERR_HIP, std::string("copy of device input: ") + hipGetErrorString(e));
  return GG_OK;
}

// Goal-reward chunk tables, fixed for a simulation: chunks of at most
// kRewardChunk particles, none spanning two environments (env, begin, end),
// each environment's first chunk, and its particle count.
gg_status build_reward_tables(gg_sim* s) {
  const int ne = s->n_envs;
  std::vector<int32_t> ch, ec(ne + 1, 0), cnt(ne);
  for (int e = 0; e < ne; ++e) {
    ec[e] = (int32_t)(ch.size() / 3);
    cnt[e] = (int32_t)(s->env_off[e + 1] - s->env_off[e]);
    for (int64_t b = s->env_off[e]; b < s->env_off[e + 1]; b += ggk::kRewardChunk) {
      ch.push_back(e);
      ch.push_back((int32_t)b);
      ch.push_back((int32_t)std::min<int64_t>(b + ggk::kRewardChunk, s->env_off[e + 1]));
    }
  }
  ec[ne] = (int32_t)(ch.size() / 3);
  const int nc = ec[ne];
  bool ok = dev_alloc(&s->d_chunks, (size_t)std::max(1, nc) * 3) == hipSuccess &&
            dev_alloc(&s->d_env_chunk, (size_t)ne + 1) == hipSuccess &&
            dev_alloc(&s->d_env_count, (size_t)std::max(1, ne)) == hipSuccess;
  if (!ok) return fail(GG_ERR_OOM, "reward table allocation failed");
  if (nc > 0) HIPCHK(s, hipMemcpy(s->d_chunks, ch.data(), ch.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(s, hipMemcpy(s->d_env_chunk, ec.data(), ec.size() * 4, hipMemcpyHostToDevice));
  if (ne > 0) HIPCHK(s, hipMemcpy(s->d_env_count, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice));
  s->n_chunks = nc;
  return GG_OK;
}

gg_status upload_env_bodies(gg_sim* s) {
  std::vector<int32_t> lo(s->n_envs, 0), hi(s->n_envs, 0);
  for (int e = 0; e < s->n_envs; ++e) lo[e] = hi[e] = 0;
  int nb = (int)s->bodies.size();
  for (int e = 0, b = 0; e < s->n_envs; ++e) {
    while (b < nb && s->bodies[b].env < e) ++b;
    lo[e] = b;
    while (b < nb && s->bodies[b].env == e) ++b;
    hi[e] = b;
  }
  s->body_lo = lo;
  s->body_hi = hi;
  if (s->env_of) {
    HIPCHK(s, hipMemcpy(s->d_body_lo, lo.data(), lo.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(s, hipMemcpy(s->d_body_hi, hi.data(), hi.size() * 4, hipMemcpyHostToDevice));
  }
  return GG_OK;
}

// Buffers one step reads and writes.  w[l] (l = 0..I-1) receives the Jacobi
// iterate after sweep l (w[0] from detection); P*[l] (l = 1..I) the impulses of
// sweep l.  The plain step alternates two iterate buffers and updates one
// impulse array in place; the recorded step (for the adjoint) keeps all.
template <typename R>
struct StepIO {
  ggk::V4<R>* x;
  ggk::V4<R>* v;
  int32_t* ncon;
  R* imass;
  int32_t* partner;
  R* Psi;
  std::vector<ggk::V4<R>*> w;
  std::vector<R*> Px, Py, Pz;
  ggk::V4<R>* dv;
  int32_t* pofs = nullptr;  // compact impulse offsets (recorded steps), else ELL slots
};

template <typename R>
StepIO<R> plain_io(gg_sim* s) {
  StepIO<R> io;
  io.x = (ggk::V4<R>*)s->x;
  io.v = (ggk::V4<R>*)s->v;
  io.ncon = s->ncon;
  io.imass = (R*)s->imass;
  io.partner = s->partner;
  io.Psi = (R*)s->Psi;
  const int I = s->p.n_iters;
  io.w.resize(I + 1);
  io.Px.assign(I + 1, (R*)s->Px);
  io.Py.assign(I + 1, (R*)s->Py);
  io.Pz.assign(I + 1, (R*)s->Pz);
  for (int l = 0; l <= I; ++l) io.w[l] = (ggk::V4<R>*)((l & 1) ? s->wb : s->wa);
  io.dv = (ggk::V4<R>*)s->dv;
  return io;
}

// Z-order re-sort of the internal particle order and rebuild of the detection
// work items (memory locality only; results do not depend on it).
template <typename R>
void launch_reorder(gg_sim* s) {
  using V = ggk::V4<R>;
  const int n = (int)s->n;
  const int grid = (n + ggk::kBlock - 1) / ggk::kBlock;
  const int rs_m = 256 * s->rs_nb;
  const int rs_nbs = (rs_m + ggk::kScanTile - 1) / ggk::kScanTile;
  hipStream_t S = s->stream;
  ggk::k_morton_keys<R><<<grid, ggk::kBlock, 0, S>>>(n, (const V*)s->x, s->inv_c, s->env_of, s->ncon,
                                                     s->p.tile_node_shift, s->mk[0]);
  for (int pass = 0; pass < s->rs_passes; ++pass) {
    const int src = pass & 1, dst = src ^ 1;
    ggk::k_rs_hist<<<s->rs_nb, ggk::kBlock, 0, S>>>(n, s->mk[src], pass * ggk::kRsBits, s->rs_nb, s->rs_hist);
    ggk::k_scan_a<<<rs_nbs, ggk::kBlock, 0, S>>>(rs_m, s->rs_hist, s->rs_hist, s->rs_bsum, 0);
    ggk::k_scan_b<<<1, 1024, 0, S>>>(rs_nbs, s->rs_bsum, rs_m, s->rs_hist);
    ggk::k_scan_c<<<rs_nbs, ggk::kBlock, 0, S>>>(rs_m, s->rs_bsum, s->rs_hist);
    ggk::k_rs_scatter<<<s->rs_nb, ggk::kBlock, 0, S>>>(n, s->mk[src], pass == 0 ? nullptr : s->mv[src], s->mk[dst],
                                                         s->mv[dst], pass * ggk::kRsBits, s->rs_nb, s->rs_hist);
  }
  ggk::k_permute<R><<<grid, ggk::kBlock, 0, S>>>(n, s->mv[s->rs_passes & 1], (const V*)s->x, (const V*)s->v,
                                                 s->orig, (V*)s->x2, (V*)s->v2, s->orig2);
  std::swap(s->x, s->x2);
  std::swap(s->v, s->v2);
  std::swap(s->orig, s->orig2);
  const unsigned long long* keys = s->mk[s->rs_passes & 1];
  const int it_nbs = (n + ggk::kScanTile - 1) / ggk::kScanTile;
  ggk::k_node_flags<<<grid, ggk::kBlock, 0, S>>>(n, keys, s->p.tile_node_shift + ggk::kCountBits, s->it_f);
  ggk::k_scan_a<<<it_nbs, ggk::kBlock, 0, S>>>(n, s->it_f, s->it_e, s->it_bsum, 0);
  ggk::k_scan_b<<<1, 1024, 0, S>>>(it_nbs, s->it_bsum, n, s->it_e);
  ggk::k_scan_c<<<it_nbs, ggk::kBlock, 0, S>>>(n, s->it_bsum, s->it_e);
  ggk::k_node_first<<<grid, ggk::kBlock, 0, S>>>(n, s->it_f, s->it_e, s->it_first);
  ggk::k_item_flags<<<grid, ggk::kBlock, 0, S>>>(n, s->it_f, s->it_e, s->it_first, s->p.tile_threads, s->it_g);
  ggk::k_scan_a<<<it_nbs, ggk::kBlock, 0, S>>>(n, s->it_g, s->it_h, s->it_bsum, 0);
  ggk::k_scan_b<<<1, 1024, 0, S>>>(it_nbs, s->it_bsum, n, s->it_h);
  ggk::k_scan_c<<<it_nbs, ggk::kBlock, 0, S>>>(n, s->it_bsum, s->it_h);
  ggk::k_item_starts<<<grid, ggk::kBlock, 0, S>>>(n, s->it_g, s->it_h, s->item_start);
  ggk::k_copy_i32<<<1, 64, 0, S>>>(s->it_h + n, &s->ctl->items);
}

// Bytes of dynamic LDS of a detection tile.
size_t detect_lds_bytes(const gg_sim* s) {
  const size_t max_cells = (size_t)s->p.tile_max_cells, max_stage = (size_t)s->p.tile_max_stage;
  return (((2 * max_cells + 1) * 4 + 31) & ~(size_t)31) + max_stage * (s->es4 + 4 + 4);
}

// The detection kernel for a workgroup size of TB threads.
template <typename R, int TB>
void detect_kernel(gg_sim* s, const StepIO<R>& io, int st, const ggk::DevBody* bod, int dgrid, size_t dlds,
                   int blk1, const ggk::EnvTables& et) {
  using V = ggk::V4<R>;
  ggk::k_detect<R, TB><<<dgrid, TB, dlds, s->stream>>>(
      (int)s->n, s->K, io.x, io.v, s->orig, s->inv_c, blk1, et, s->bstart, s->sidx, (const V*)s->xs, s->os,
      s->item_start, &s->ctl->items, bod, (int)s->bodies.size(), (R)s->p.gravity[0], (R)s->p.gravity[1],
      (R)s->p.gravity[2], (R)s->p.dt, s->p.mass_split, s->p.tile_max_cells, s->p.tile_max_stage, io.ncon,
      io.partner, io.Psi, io.w[0], io.imass, s->ctl, s->det_part, st, s->det_queue,
      (s->p.flags & GG_FLAG_TAPE) ? 1 : 0);
}

// Detection workgroups of a split step (their counts are summed by k_integrate).
int detect_grid(const gg_sim* s) {
  return std::max(1, std::min((int)((s->n + 31) / 32), s->det_grid));
}

// Bucket table and contact detection of one step.
template <typename R>
void launch_detect(gg_sim* s, const StepIO<R>& io, int st, const ggk::DevBody* bod, bool with_detect = true) {
  using V = ggk::V4<R>;
  const int n = (int)s->n;
  const int grid = (n + ggk::kBlock - 1) / ggk::kBlock;
  const int m = (int)s->n_buckets;
  const int nbs = (m + ggk::kScanTile - 1) / ggk::kScanTile;
  const int dgrid = detect_grid(s);
  const size_t dlds = detect_lds_bytes(s);
  const ggk::EnvTables et = env_tables(s);
  const int nh1 = s->env_nh[0];
  const int blk1 = s->env_tblk[0];
  hipStream_t S = s->stream;
  if (s->small_table) {
    // small bed: keys, scan and scatter in one workgroup (counters in LDS)
    ggk::k_bucket_small<R><<<1, ggk::kSmallBlock, (size_t)(m + 1) * 4, S>>>(
        n, m, io.x, s->inv_c, nh1, blk1, et, s->h, s->h6, s->rank, s->bstart, s->orig, s->sidx, (V*)s->xs, s->os,
        s->ctl, st);
  } else {
    ggk::k_key<R><<<grid, ggk::kBlock, 0, S>>>(n, io.x, s->inv_c, nh1, blk1, et, s->h, s->h6, s->rank, s->counts,
                                               s->ctl, st);
    ggk::k_scan_a<<<nbs, ggk::kBlock, 0, S>>>(m, s->counts, s->bstart, s->bsum, 1);
    ggk::k_scan_b<<<1, 1024, 0, S>>>(nbs, s->bsum, m, s->bstart);
    ggk::k_scan_c<<<nbs, ggk::kBlock, 0, S>>>(m, s->bsum, s->bstart);
    ggk::k_scatter<R><<<grid, ggk::kBlock, 0, S>>>(n, s->h, s->rank, s->bstart, io.x, s->orig, s->sidx, (V*)s->xs,
                                                   s->os);
  }
  if (!with_detect) return;
  switch (s->p.tile_threads) {
    case 64: detect_kernel<R, 64>(s, io, st, bod, dgrid, dlds, blk1, et); break;
    case 256: detect_kernel<R, 256>(s, io, st, bod, dgrid, dlds, blk1, et); break;
    default: detect_kernel<R, 128>(s, io, st, bod, dgrid, dlds, blk1, et); break;
  }
}

// The projected-Jacobi sweeps of one step (the last one writes the velocity).
template <typename R>
void launch_sweeps(gg_sim* s, const StepIO<R>& io, const ggk::DevBody* bod) {
  const int n = (int)s->n;
  const int grid = (n + ggk::kBlock - 1) / ggk::kBlock;
  const int I = s->p.n_iters;
  const R alpha_dt = (R)s->p.alpha / (R)s->p.dt;
  const int L = s->p.pja_lanes;
  const int lgrid = (int)(((int64_t)n * L + ggk::kBlock - 1) / ggk::kBlock);
  for (int it = 0; it < I; ++it) {
    const int l = it + 1;
    const int mode = (it == 0 ? 1 : 0) | (it == I - 1 ? 2 : 0);
    if (L == 1)
      ggk::k_pja<R><<<grid, ggk::kBlock, 0, s->stream>>>(
          n, s->K, io.x, io.v, io.w[l - 1], io.w[l], io.ncon, io.partner, io.Psi, io.Px[l - 1], io.Py[l - 1],
          io.Pz[l - 1], io.Px[l], io.Py[l], io.Pz[l], bod, (R)s->p.gravity[0], (R)s->p.gravity[1],
          (R)s->p.gravity[2], (R)s->p.dt, alpha_dt, (R)s->p.mu, (R)s->p.relax, mode, io.dv, io.pofs, io.imass,
          s->ctl);
    else if (L == 2)
      ggk::k_pja_lanes<R, 2><<<lgrid, ggk::kBlock, 0, s->stream>>>(
          n, s->K, io.x, io.v, io.w[l - 1], io.w[l], io.ncon, io.partner, io.Psi, io.Px[l - 1], io.Py[l - 1],
          io.Pz[l - 1], io.Px[l], io.Py[l], io.Pz[l], bod, (R)s->p.gravity[0], (R)s->p.gravity[1],
          (R)s->p.gravity[2], (R)s->p.dt, alpha_dt, (R)s->p.mu, (R)s->p.relax, mode, io.dv, io.pofs, io.imass,
          s->ctl);
    else
      ggk::k_pja_lanes<R, 4><<<lgrid, ggk::kBlock, 0, s->stream>>>(
          n, s->K, io.x, io.v, io.w[l - 1], io.w[l], io.ncon, io.partner, io.Psi, io.Px[l - 1], io.Py[l - 1],
          io.Pz[l - 1], io.Px[l], io.Py[l], io.Pz[l], bod, (R)s->p.gravity[0], (R)s->p.gravity[1],
          (R)s->p.gravity[2], (R)s->p.dt, alpha_dt, (R)s->p.mu, (R)s->p.relax, mode, io.dv, io.pofs, io.imass,
          s->ctl);
  }
}

// The cyclic vertical boundary in the build's precision (span 0: off).
template <typename R>
R cyc_lo(const gg_sim* s);
template <typename R>
R cyc_span(const gg_sim* s);

// Detection, sweeps and position update of one step as one cooperative launch
// (GG_FLAG_FUSED); the bucket table is built by the preceding launches.
template <typename R, int TB>
hipError_t fused_kernel(gg_sim* s, ggk::FusedArgs<R>& a) {
  void* args[] = {&a};
  return hipLaunchCooperativeKernel((const void*)ggk::k_step_fused<R, TB>, dim3(s->fused_grid), dim3(TB), args,
                                    (unsigned)detect_lds_bytes(s), s->stream);
}

template <typename R>
gg_status launch_fused(gg_sim* s, const StepIO<R>& io, int st, const ggk::DevBody* bod) {
  ggk::FusedArgs<R> a;
  a.n = (int)s->n;
  a.K = s->K;
  a.x = io.x;
  a.v = io.v;
  a.orig = s->orig;
  a.inv_c = s->inv_c;
  a.n_blk = s->env_tblk[0];
  a.env = env_tables(s);
  a.start = s->bstart;
  a.sidx = s->sidx;
  a.xs = (const ggk::V4<R>*)s->xs;
  a.os = s->os;
  a.item_start = s->item_start;
  a.n_items = &s->ctl->items;
  a.bodies = bod;
  a.n_bodies = (int)s->bodies.size();
  a.mass_split = s->p.mass_split;
  a.max_cells = s->p.tile_max_cells;
  a.max_stage = s->p.tile_max_stage;
  a.iters = s->p.n_iters;
  a.gx = (R)s->p.gravity[0];
  a.gy = (R)s->p.gravity[1];
  a.gz = (R)s->p.gravity[2];
  a.dt = (R)s->p.dt;
  a.alpha_dt = (R)s->p.alpha / (R)s->p.dt;
  a.mu = (R)s->p.mu;
  a.relax = (R)s->p.relax;
  a.zlo = cyc_lo<R>(s);
  a.zspan = cyc_span<R>(s);
  a.ncon = io.ncon;
  a.partner = io.partner;
  a.Psi = io.Psi;
  a.wa = io.w[0];
  a.wb = io.w[1];
  a.Px = io.Px[0];
  a.Py = io.Py[0];
  a.Pz = io.Pz[0];
  a.dv = io.dv;
  a.imass = io.imass;
  a.ctl = s->ctl;
  a.part = s->det_part;
  a.step = st;
  a.pair_gaps = (s->p.flags & GG_FLAG_TAPE) ? 1 : 0;
  hipError_t e;
  switch (s->p.tile_threads) {
    case 64: e = fused_kernel<R, 64>(s, a); break;
    case 256: e = fused_kernel<R, 256>(s, a); break;
    default: e = fused_kernel<R, 128>(s, a); break;
  }
  HIPCHK(s, e);
  ggk::k_detect_stats<<<1, ggk::kBlock, 0, s->stream>>>(s->fused_grid, s->det_part, s->ctl, nullptr);
  return GG_OK;
}

template <typename R>
R cyc_lo(const gg_sim* s) {
  return (R)s->p.cyclic_z[0];
}
template <typename R>
R cyc_span(const gg_sim* s) {
  return s->p.cyclic_z[1] > s->p.cyclic_z[0] ? (R)s->p.cyclic_z[1] - (R)s->p.cyclic_z[0] : R(0);
}

// Enqueue the launches of n_steps steps on s->stream (eager or under capture).
template <typename R>
gg_status enqueue_steps_t(gg_sim* s, int n_steps, int nb, bool taped, bool prof) {
  using V = ggk::V4<R>;
  const int n = (int)s->n;
  const int grid = (n + ggk::kBlock - 1) / ggk::kBlock;
  const R dt = (R)s->p.dt;
  hipStream_t S = s->stream;
  ggk::k_begin<<<1, 64, 0, S>>>(s->ctl);
  for (int st = 0; st < n_steps && n > 0; ++st) {
    const ggk::DevBody* bod = s->d_bodies + (size_t)st * nb;
    if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st], S));
    const int64_t g = s->steps_global + st;
    // a differentiable call keeps one internal order throughout (re-sorted only at its start)
    if (s->p.reorder_every > 0 && (taped ? st == 0 : g % s->p.reorder_every == 0)) launch_reorder<R>(s);
    if (taped && st % s->p.checkpoint_every == 0) {
      V* ckx = (V*)s->ck + (size_t)(st / s->p.checkpoint_every) * 2 * n;
      HIPCHK(s, hipMemcpyAsync(ckx, s->x, (size_t)n * sizeof(V), hipMemcpyDeviceToDevice, S));
      HIPCHK(s, hipMemcpyAsync(ckx + n, s->v, (size_t)n * sizeof(V), hipMemcpyDeviceToDevice, S));
    }
    const StepIO<R> io = plain_io<R>(s);
    if (s->p.flags & GG_FLAG_FUSED) {  // (never taped: rejected at creation)
      launch_detect<R>(s, io, st, bod, false);
      if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 1], S));
      gg_status fs = launch_fused<R>(s, io, st, bod);
      if (fs != GG_OK) return fs;
      if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 2], S));
      if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 3], S));
      continue;
    }
    launch_detect<R>(s, io, st, bod);
    if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 1], S));
    launch_sweeps<R>(s, io, bod);
    if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 2], S));
    ggk::k_integrate<R><<<grid, ggk::kBlock, 0, S>>>(n, (V*)s->x, (const V*)s->v, dt, cyc_lo<R>(s), cyc_span<R>(s),
                                                     s->ctl, s->det_part, detect_grid(s),
                                                     taped ? s->d_counts + 2 * (size_t)st : nullptr);
    if (prof) HIPCHK(s, hipEventRecord(s->events[4 * st + 3], S));
  }
  return GG_OK;
}

gg_status enqueue_steps(gg_sim* s, int n_steps, int nb, bool taped, bool prof) {
  return s->fp64 ? enqueue_steps_t<double>(s, n_steps, nb, taped, prof)
                 : enqueue_steps_t<float>(s, n_steps, nb, taped, prof);
}

// Replay (capturing first if needed) the launch sequence of n_steps steps.  A
// capture is keyed by everything its launches name that can change between
// calls: the step count, the re-sort phase, which of the two state buffers is
// current, the body count and the allocation epoch.
gg_status launch_graphed(gg_sim* s, int n_steps, int nb) {
  const int64_t R = s->p.reorder_every;
  const int64_t phase = R > 0 ? s->steps_global % R : 0;
  gg_sim::Graph* hit = nullptr;
  for (auto& G : s->graphs)
    if (G.n_steps == n_steps && G.phase == phase && G.x0 == s->x && G.nb == nb && G.epoch == s->epoch) hit = &G;
  if (!hit) {
    if (!s->cap_stream) HIPCHK(s, hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    gg_sim::Graph G;
    G.n_steps = n_steps;
    G.phase = phase;
    G.x0 = s->x;
    G.nb = nb;
    G.epoch = s->epoch;
    void *x0 = s->x, *v0 = s->v;
    int32_t* o0 = s->orig;
    hipStream_t user = s->stream;
    s->stream = s->cap_stream;
    hipError_t e = hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal);
    gg_status st = GG_OK;
    if (e == hipSuccess) st = enqueue_steps(s, n_steps, nb, false, false);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &graph);
    s->stream = user;
    G.x1 = s->x;
    G.v1 = s->v;
    G.o1 = s->orig;
    // nothing ran: restore the pointer state the capture walked through
    s->x = x0;
    s->v = v0;
    s->orig = o0;
    if (s->x != G.x1) {
      s->x2 = G.x1;
      s->v2 = G.v1;
      s->orig2 = G.o1;
    }
    if (e != hipSuccess) return hip_fail(s, e, "hipStreamBeginCapture");
    if (st != GG_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    if (e2 != hipSuccess) return hip_fail(s, e2, "hipStreamEndCapture");
    e = hipGraphInstantiateWithFlags(&G.exec, graph, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(s, e, "hipGraphInstantiate");
    if (s->graphs.size() >= 64) {   // (every re-sort phase and buffer parity of one-step calls)
      size_t old = 0;
      for (size_t k = 1; k < s->graphs.size(); ++k)
        if (s->graphs[k].used < s->graphs[old].used) old = k;
      (void)hipGraphExecDestroy(s->graphs[old].exec);
      s->graphs.erase(s->graphs.begin() + (long)old);
    }
    s->graphs.push_back(G);
    hit = &s->graphs.back();
  }
  hit->used = ++s->graph_clock;
  HIPCHK(s, hipGraphLaunch(hit->exec, s->stream));
  if (hit->x1 != s->x) {
    std::swap(s->x, s->x2);
    std::swap(s->v, s->v2);
    std::swap(s->orig, s->orig2);
  }
  return GG_OK;
}

template <typename R>
gg_status backward_t(gg_sim* s, const float* dL_dx, const float* dL_dv, float* dL_dx0, float* dL_dv0,
                     float* dL_dtwists, gg_mem where);

}  // namespace

extern "C" {

const char* gg_status_string(gg_status st) {
  switch (st) {
    case GG_OK: return "ok";
    case GG_ERR_INVALID: return "invalid argument";
    case GG_ERR_OOM: return "out of memory";
    case GG_ERR_HIP: return "HIP runtime error";
    case GG_ERR_CAPACITY: return "contact capacity exceeded";
    case GG_ERR_NONFINITE: return "non-finite or out-of-range state";
    case GG_ERR_NO_TAPE: return "no recorded forward pass";
    case GG_ERR_UNSUPPORTED: return "unsupported in this build";
  }
  return "unknown status";
}

const char* gg_error_detail(void) { return g_detail.c_str(); }

gg_status gg_create(const gg_params* params, int32_t n_envs, const int64_t* env_offsets, int64_t n,
                    const float* x, const float* v, const float* radius, gg_mem where, gg_sim** out) {
  g_detail.clear();
  if (!out) return fail(GG_ERR_INVALID, "out is NULL");
  *out = nullptr;
  gg_status st = check_params(params);
  if (st != GG_OK) return st;
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  if (n < 0 || n > ((int64_t)1 << 30)) return fail(GG_ERR_INVALID, "n must be in [0, 2^30]");
  if (n_envs < 1) return fail(GG_ERR_INVALID, "n_envs must be >= 1");
  std::vector<int64_t> off(n_envs + 1);
  if (env_offsets) {
    for (int e = 0; e <= n_envs; ++e) off[e] = env_offsets[e];
    if (off[0] != 0 || off[n_envs] != n) return fail(GG_ERR_INVALID, "env_offsets must start at 0 and end at n");
    for (int e = 0; e < n_envs; ++e)
      if (off[e + 1] < off[e]) return fail(GG_ERR_INVALID, "env_offsets must be non-decreasing");
  } else {
    if (n_envs != 1) return fail(GG_ERR_INVALID, "env_offsets is required when n_envs > 1");
    off[0] = 0;
    off[1] = n;
  }
  if (n > 0 && (!x || !v || !radius)) return fail(GG_ERR_INVALID, "x, v and radius are required when n > 0");

  // ---- inputs to the host, then checks
  std::vector<float> hx(3 * n), hv(3 * n), hr(n);
  if (where == GG_MEM_DEVICE) {
    DeviceGuard g(params->device);
    if (!g.ok) return fail(GG_ERR_HIP, "hipSetDevice failed");
    if ((st = copy_in(x, 12 * n, where, hx.data())) != GG_OK) return st;
    if ((st = copy_in(v, 12 * n, where, hv.data())) != GG_OK) return st;
    if ((st = copy_in(radius, 4 * n, where, hr.data())) != GG_OK) return st;
  } else {
    copy_in(x, 12 * n, where, hx.data());
    copy_in(v, 12 * n, where, hv.data());
    copy_in(radius, 4 * n, where, hr.data());
  }
  float rmax = 0.0f, rmin = INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    if (!(hr[i] > 0.0f) || !std::isfinite(hr[i])) return fail(GG_ERR_INVALID, "radius must be finite and > 0");
    rmax = std::max(rmax, hr[i]);
    rmin = std::min(rmin, hr[i]);
    if (!finite3(&hx[3 * i]) || !finite3(&hv[3 * i])) return fail(GG_ERR_NONFINITE, "non-finite position or velocity");
  }
  if (n == 0) rmin = rmax = 1.0f;
  float cell = params->cell_size;
  if (cell == 0.0f) cell = (float)(2.0 * (double)rmax * (1.0 + 1.0 / 1024.0));
  if (n > 0 && !((double)cell >= 2.0 * (double)rmax))
    return fail(GG_ERR_INVALID, "cell_size must be at least twice the largest radius");
  const float inv_c = 1.0f / cell;
  for (int64_t q = 0; q < 3 * n; ++q) {
    float s = hx[q] * inv_c;
    if (!(std::fabs(std::nearbyint(s)) < 1073741824.0f))
      return fail(GG_ERR_INVALID, "position too far from the origin for the cell size (|x/c| >= 2^30)");
  }
  std::vector<int32_t> env_nh(n_envs), env_boff(n_envs), env_tblk(n_envs), env_toff(n_envs);
  int64_t total = 0, total_tab = 0;
  for (int e = 0; e < n_envs; ++e) {
    int64_t ne = off[e + 1] - off[e];
    int64_t nh = params->hash_size > 0 ? params->hash_size : std::max<int64_t>(1, 2 * ne);
    env_nh[e] = (int32_t)nh;
    env_boff[e] = (int32_t)total;
    total += nh;
    // The internal table (the counting sort's buckets) follows n_h, but a
    // large single bed gets at least four buckets per particle: Z-order nodes
    // that share a block of buckets stage each other's particles, and at two
    // per particle about a third of the nodes share one (1M-grain settled
    // bed: 9-12 items per step exceed the detection tile and take the
    // per-particle path; none at four).  Eq. (6)'s index still uses n_h.
    int64_t tab = nh;
    if (n_envs == 1 && ne >= ((int64_t)1 << 18)) tab = std::max<int64_t>(tab, 4 * ne);
    const int64_t blk = (tab + 63) / 64;
    env_tblk[e] = (int32_t)blk;
    env_toff[e] = (int32_t)total_tab;
    total_tab += 64 * blk;
    if (total_tab > ((int64_t)1 << 31) - 2) return fail(GG_ERR_INVALID, "total hash buckets exceed 2^31 - 2");
  }

  {
    const int64_t n_pad = (n + 63) / 64 * 64;
    int K0 = capacity_for(*params, contact_bound(rmin, rmax), 0);
    if (params->max_contacts_per_particle == 0) K0 = std::min(K0, kAutoCapacity);
    if (!slots_fit(n_pad, K0)) return slots_error(n_pad, K0);
  }

  gg_sim* s = new (std::nothrow) gg_sim();
  if (!s) return fail(GG_ERR_OOM, "host allocation failed");
  s->p = *params;
  if (s->p.relax == 0.0f) s->p.relax = 1.0f;
  if (s->p.density == 0.0f) s->p.density = 2500.0f;
  if (s->p.checkpoint_every == 0) s->p.checkpoint_every = 10;
  // a re-sort costs ~30 launches; below 2^19 particles the order decays slowly
  // relative to it (measured: 32 steps 3-9% faster per step than 8), above
  // every 16 steps; large beds of spread radii every 4 steps, where contact
  // counts vary most and the count order within nodes pays (4M polydisperse
  // bed: 27.3 ms per step against 28.7 at 16)
  if (s->p.reorder_every == 0)
    s->p.reorder_every = n < (1 << 19) ? 32 : ((double)rmax > 1.25 * (double)rmin ? 4 : 16);
  default_tile(n, particles_per_cell(hx, n, inv_c), s->p);
  {
    // (keys are 64 bits: beyond 2^26 environments the environment's high bits
    // fall off, which only costs locality)
    int bits = 30 + ggk::kCountBits;
    while (bits < 64 && (int64_t{1} << (bits - 30 - ggk::kCountBits)) < (int64_t)n_envs) ++bits;
    s->rs_passes = (bits + ggk::kRsBits - 1) / ggk::kRsBits;
    s->rs_nb = (int)((n + ggk::kRsItems - 1) / ggk::kRsItems);
  }
  s->fp64 = s->p.precision == 1;
  s->es = s->fp64 ? 8 : 4;
  s->es4 = 4 * s->es;
  s->dev = params->device;
  s->n = n;
  s->n_envs = n_envs;
  s->env_off = off;
  s->env_nh = env_nh;
  s->env_boff = env_boff;
  s->env_tblk = env_tblk;
  s->env_toff = env_toff;
  s->n_buckets = total_tab;
  s->cell = cell;
  s->inv_c = inv_c;
  s->r_max = rmax;
  s->r_min = rmin;
  s->K_pp = contact_bound(rmin, rmax);
  // measured with keys and sort: the queues take 16% off detection in a
  // polydisperse 4M bed, 17% in a settled uniform 1M bed and 11% in a
  // uniform lattice, against fixed contiguous shares (the fused step kernel
  // keeps those)
  s->det_queue = (s->p.flags & GG_FLAG_FUSED) == 0;
  s->n_pad = (n + 63) / 64 * 64;
  s->body_lo.assign(n_envs, 0);
  s->body_hi.assign(n_envs, 0);
  s->stats.n = n;
  s->stats.n_buckets = total_tab;

  DeviceGuard g(s->dev);
  auto bail = [&](gg_status code) {
    free_all(s);
    delete s;
    return code;
  };
  if (!g.ok) return bail(fail(GG_ERR_HIP, "hipSetDevice failed"));
  if (params->stream) {
    s->stream = (hipStream_t)params->stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(nullptr, e, "hipStreamCreateWithFlags"));
    s->own_stream = true;
  }
  const size_t N = (size_t)std::max<int64_t>(n, 1);
  const size_t N4 = N * s->es4;
  bool ok = dev_alloc_bytes(&s->x, N4) == hipSuccess && dev_alloc_bytes(&s->v, N4) == hipSuccess &&
            dev_alloc_bytes(&s->wa, N4) == hipSuccess && dev_alloc_bytes(&s->wb, N4) == hipSuccess &&
            dev_alloc(&s->h, N) == hipSuccess && dev_alloc(&s->rank, N) == hipSuccess &&
            dev_alloc(&s->h6, N) == hipSuccess &&
            dev_alloc(&s->counts, (size_t)total_tab) == hipSuccess &&
            dev_alloc(&s->bstart, (size_t)total_tab + 1) == hipSuccess &&
            dev_alloc(&s->bsum, (size_t)(total_tab + ggk::kScanTile - 1) / ggk::kScanTile + 1) == hipSuccess &&
            dev_alloc(&s->sidx, N) == hipSuccess && dev_alloc(&s->ncon, N) == hipSuccess &&
            dev_alloc_bytes(&s->imass, N * s->es) == hipSuccess &&
            dev_alloc(&s->ctl, 1) == hipSuccess && dev_alloc_bytes(&s->x2, N4) == hipSuccess &&
            dev_alloc_bytes(&s->v2, N4) == hipSuccess && dev_alloc(&s->orig, N) == hipSuccess &&
            dev_alloc(&s->orig2, N) == hipSuccess && dev_alloc(&s->mk[0], N) == hipSuccess &&
            dev_alloc(&s->mk[1], N) == hipSuccess && dev_alloc(&s->mv[0], N) == hipSuccess &&
            dev_alloc(&s->mv[1], N) == hipSuccess &&
            dev_alloc(&s->rs_hist, (size_t)256 * std::max(1, s->rs_nb) + 1) == hipSuccess &&
            dev_alloc(&s->rs_bsum, (size_t)(256 * std::max(1, s->rs_nb) + ggk::kScanTile - 1) / ggk::kScanTile + 1) == hipSuccess &&
            dev_alloc_bytes(&s->xs, N4) == hipSuccess && dev_alloc(&s->os, N) == hipSuccess &&
            dev_alloc(&s->it_f, N + 1) == hipSuccess && dev_alloc(&s->it_e, N + 1) == hipSuccess &&
            dev_alloc(&s->it_first, N + 1) == hipSuccess && dev_alloc(&s->it_g, N + 1) == hipSuccess &&
            dev_alloc(&s->it_h, N + 1) == hipSuccess && dev_alloc(&s->item_start, N + 2) == hipSuccess &&
            dev_alloc(&s->it_bsum, (N + 1 + ggk::kScanTile - 1) / ggk::kScanTile + 1) == hipSuccess;
  if (ok && (s->p.flags & GG_FLAG_DIAGNOSTICS)) ok = dev_alloc_bytes(&s->dv, N4) == hipSuccess;
  if (ok && n_envs > 1) {
    ok = dev_alloc(&s->env_of, N) == hipSuccess && dev_alloc(&s->d_env_nh, (size_t)n_envs) == hipSuccess &&
         dev_alloc(&s->d_env_boff, (size_t)n_envs) == hipSuccess &&
         dev_alloc(&s->d_env_tblk, (size_t)n_envs) == hipSuccess &&
         dev_alloc(&s->d_env_toff, (size_t)n_envs) == hipSuccess &&
         dev_alloc(&s->d_body_lo, (size_t)n_envs) == hipSuccess &&
         dev_alloc(&s->d_body_hi, (size_t)n_envs) == hipSuccess;
  }
  if (!ok) return bail(fail(GG_ERR_OOM, "device allocation failed"));
  if (hipHostMalloc((void**)&s->h_ctl, sizeof(ggk::Ctl), hipHostMallocDefault) != hipSuccess)
    return bail(fail(GG_ERR_OOM, "pinned allocation failed"));

  // ---- upload state: x = (x, r), v = (v, 1/m)
  std::vector<float4> hx4(s->fp64 ? 0 : N), hv4(s->fp64 ? 0 : N);
  std::vector<double4> hx8(s->fp64 ? N : 0), hv8(s->fp64 ? N : 0);
  const double rho = (double)s->p.density;
  for (int64_t i = 0; i < n; ++i) {
    double r = hr[i];
    double m = rho * (4.0 / 3.0) * M_PI * r * r * r;
    if (s->fp64) {
      hx8[i] = make_double4(hx[3 * i], hx[3 * i + 1], hx[3 * i + 2], hr[i]);
      hv8[i] = make_double4(hv[3 * i], hv[3 * i + 1], hv[3 * i + 2], 1.0 / m);
    } else {
      hx4[i] = make_float4(hx[3 * i], hx[3 * i + 1], hx[3 * i + 2], hr[i]);
      hv4[i] = make_float4(hv[3 * i], hv[3 * i + 1], hv[3 * i + 2], (float)(1.0 / m));
    }
  }
  hipError_t e = hipSuccess;
  if (n > 0) {
    const void* px = s->fp64 ? (const void*)hx8.data() : (const void*)hx4.data();
    const void* pv = s->fp64 ? (const void*)hv8.data() : (const void*)hv4.data();
    if (e == hipSuccess) e = hipMemcpy(s->x, px, n * s->es4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->v, pv, n * s->es4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipMemset(s->counts, 0, (size_t)total_tab * 4);
  if (e == hipSuccess) e = hipMemset(s->ctl, 0, sizeof(ggk::Ctl));
  if (e == hipSuccess) e = hipMemset(s->ncon, 0, N * 4);   // (the first re-sort's contact counts)
  if (e == hipSuccess && n > 0) {
    ggk::k_iota<<<(int)((n + 255) / 256), 256>>>((int)n, s->orig);
    ggk::k_item_fixed<<<(int)((n + 255) / 256), 256>>>((int)n, s->p.tile_threads, s->item_start, &s->ctl->items);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
  }
  if (e == hipSuccess && n_envs > 1) {
    std::vector<int32_t> eo(N, 0);
    for (int q = 0; q < n_envs; ++q)
      for (int64_t i = off[q]; i < off[q + 1]; ++i) eo[i] = q;
    e = hipMemcpy(s->env_of, eo.data(), N * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_env_nh, env_nh.data(), n_envs * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_env_boff, env_boff.data(), n_envs * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_env_tblk, env_tblk.data(), n_envs * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_env_toff, env_toff.data(), n_envs * 4, hipMemcpyHostToDevice);
    std::vector<int32_t> zeros(n_envs, 0);
    if (e == hipSuccess) e = hipMemcpy(s->d_body_lo, zeros.data(), n_envs * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->d_body_hi, zeros.data(), n_envs * 4, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return bail(hip_fail(nullptr, e, "upload"));
  {
    // detection workgroups: every resident slot once (each takes a contiguous
    // run of work items), so no second partial wave of workgroups trails
    int per_cu = 0, n_cu = 0;
    const size_t dlds = detect_lds_bytes(s);
    const int tb = s->p.tile_threads;
    hipError_t oe;
    if (s->fp64) {
      oe = tb == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<double, 64>, tb, dlds)
           : tb == 256 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<double, 256>, tb, dlds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<double, 128>, tb, dlds);
    } else {
      oe = tb == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<float, 64>, tb, dlds)
           : tb == 256 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<float, 256>, tb, dlds)
                       : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ggk::k_detect<float, 128>, tb, dlds);
    }
    if (oe == hipSuccess) oe = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->dev);
    if (oe != hipSuccess) return bail(hip_fail(nullptr, oe, "occupancy query"));
    s->det_grid = std::max(1, per_cu * n_cu);
    // small tables: counters of every bucket in one workgroup's LDS
    int max_lds = 0;
    oe = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->dev);
    if (oe != hipSuccess) return bail(hip_fail(nullptr, oe, "LDS size query"));
    const int64_t need_lds = (s->n_buckets + 1) * 4 + 256;
    s->small_table = s->n_buckets <= ggk::kSmallBuckets && need_lds <= max_lds;
    if (s->p.flags & GG_FLAG_FUSED) {
      int coop = 0;
      oe = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, s->dev);
      if (oe != hipSuccess) return bail(hip_fail(nullptr, oe, "cooperative launch query"));
      if (!coop) return bail(fail(GG_ERR_UNSUPPORTED, "GG_FLAG_FUSED needs cooperative launches"));
      int fpc = 0;
      if (s->fp64)
        oe = tb == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<double, 64>, tb, dlds)
             : tb == 256 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<double, 256>, tb, dlds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<double, 128>, tb, dlds);
      else
        oe = tb == 64    ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<float, 64>, tb, dlds)
             : tb == 256 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<float, 256>, tb, dlds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&fpc, ggk::k_step_fused<float, 128>, tb, dlds);
      if (oe != hipSuccess) return bail(hip_fail(nullptr, oe, "occupancy query"));
      if (fpc < 1) return bail(fail(GG_ERR_UNSUPPORTED, "the fused step kernel does not fit a compute unit"));
      // resident at once, and no more workgroups than particles call for
      s->fused_grid = std::max(1, std::min(fpc * n_cu, (int)((s->n + tb - 1) / tb)));
    }
    const size_t parts = (size_t)std::max(s->det_grid, s->fused_grid);
    oe = dev_alloc(&s->det_part, parts);
    if (oe == hipSuccess) oe = hipMemset(s->det_part, 0, parts * sizeof(ggk::DetPart));
    if (oe != hipSuccess) return bail(fail(GG_ERR_OOM, "device allocation failed"));
  }
  s->stats.tile_threads = s->p.tile_threads;
  s->stats.tile_node_shift = s->p.tile_node_shift;
  s->stats.tile_max_cells = s->p.tile_max_cells;
  s->stats.tile_max_stage = s->p.tile_max_stage;
  s->stats.detect_workgroups = s->det_grid;
  s->stats.reorder_every = s->p.reorder_every;
  s->stats.pja_lanes = s->p.pja_lanes;
  s->stats.detect_queues = s->det_queue ? 1 : 0;
  st = ensure_ell(s, compute_K(s));
  if (st != GG_OK) return bail(st);
  st = build_reward_tables(s);
  if (st != GG_OK) return bail(st);
  sample_memory(s);
  *out = s;
  return GG_OK;
}

gg_status gg_set_bodies(gg_sim* s, int32_t n_bodies, const gg_body* bodies, gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (n_bodies < 0 || n_bodies > 65536) return fail(GG_ERR_INVALID, "n_bodies must be in [0, 65536]");
  if (n_bodies > 0 && !bodies) return fail(GG_ERR_INVALID, "bodies is NULL");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  std::vector<gg_body> hb(n_bodies);
  if (where == GG_MEM_DEVICE) {
    DeviceGuard g(s->dev);
    gg_status st = copy_in(bodies, sizeof(gg_body) * n_bodies, where, hb.data());
    if (st != GG_OK) return st;
  } else {
    copy_in(bodies, sizeof(gg_body) * n_bodies, where, hb.data());
  }
  std::vector<HostBody> nb(n_bodies);
  int prev_env = 0;
  for (int b = 0; b < n_bodies; ++b) {
    const gg_body& B = hb[b];
    if (B.env < 0 || B.env >= s->n_envs) return fail(GG_ERR_INVALID, "body env out of range");
    if (B.env < prev_env) return fail(GG_ERR_INVALID, "bodies must be grouped by env in non-decreasing order");
    prev_env = B.env;
    if (B.shape < GG_PLANE || B.shape > GG_GRID) return fail(GG_ERR_INVALID, "unknown body shape");
    if (B.shape == GG_GRID &&
        !(B.params[0] >= 0.0f && B.params[0] < (float)s->grids.size() && B.params[0] == std::floor(B.params[0])))
      return fail(GG_ERR_INVALID, "grid body: params[0] must index a grid registered with gg_set_grids");
    for (int q = 0; q < 4; ++q)
      if (!std::isfinite(B.params[q])) return fail(GG_ERR_INVALID, "non-finite body parameter");
    if (B.shape == GG_BOX && !(B.params[0] > 0 && B.params[1] > 0 && B.params[2] > 0))
      return fail(GG_ERR_INVALID, "box half extents must be > 0");
    if (B.shape == GG_CAPSULE && !(B.params[0] > 0 && B.params[1] >= 0))
      return fail(GG_ERR_INVALID, "capsule radius must be > 0 and half length >= 0");
    for (int q = 0; q < 12; ++q)
      if (!std::isfinite(B.pose[q])) return fail(GG_ERR_INVALID, "non-finite body pose");
    for (int q = 0; q < 6; ++q)
      if (!std::isfinite(B.twist[q])) return fail(GG_ERR_INVALID, "non-finite body twist");
    HostBody& H = nb[b];
    H.env = B.env;
    H.shape = B.shape;
    H.grid = B.shape == GG_GRID ? (int32_t)B.params[0] : -1;
    for (int q = 0; q < 4; ++q) H.params[q] = B.params[q];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) H.R[3 * r + c] = B.pose[4 * r + c];
      H.t[r] = B.pose[4 * r + 3];
    }
    for (int q = 0; q < 3; ++q) {
      H.nu[q] = B.twist[q];
      H.om[q] = B.twist[3 + q];
    }
  }
  {
    int nb_env = 0;
    for (int b = 0; b < n_bodies;) {
      int e = nb[b].env, c = 0;
      while (b < n_bodies && nb[b].env == e) ++b, ++c;
      nb_env = std::max(nb_env, c);
    }
    int K1 = capacity_for(s->p, s->K_pp, nb_env);
    if (s->p.max_contacts_per_particle == 0) K1 = std::min(K1, std::max((kAutoCapacity + nb_env + 1) & ~1, s->K_floor));
    if (!slots_fit(s->n_pad, K1)) return slots_error(s->n_pad, K1);
  }
  DeviceGuard g(s->dev);
  // the recorded forward names the old bodies (count, poses, grid values)
  s->tape_ok = false;
  s->bodies = nb;
  gg_status st = upload_env_bodies(s);
  if (st != GG_OK) return st;
  return ensure_ell(s, compute_K(s));
}

gg_status gg_set_grids(gg_sim* s, int32_t n_grids, const gg_grid* grids, int64_t n_values, const float* values,
                       gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  if (n_grids < 0 || n_grids > 4096) return fail(GG_ERR_INVALID, "n_grids must be in [0, 4096]");
  if (n_values < 0) return fail(GG_ERR_INVALID, "n_values must be >= 0");
  if (n_grids > 0 && !grids) return fail(GG_ERR_INVALID, "grids is NULL");
  if (n_values > 0 && !values) return fail(GG_ERR_INVALID, "values is NULL");
  std::vector<gg_grid> G(grids, grids + n_grids);
  for (const gg_grid& g : G) {
    if (g.nx < 2 || g.ny < 2 || g.nz < 2) return fail(GG_ERR_INVALID, "a grid needs at least 2 knots per axis");
    if (!(g.inv_spacing > 0.0f) || !std::isfinite(g.inv_spacing) || !finite3(g.origin))
      return fail(GG_ERR_INVALID, "grid origin and inv_spacing must be finite, inv_spacing > 0");
    const int64_t m = (int64_t)g.nx * g.ny * g.nz;
    if (g.offset < 0 || g.offset > n_values - m) return fail(GG_ERR_INVALID, "a grid lies outside the values array");
  }
  std::vector<float> hv((size_t)n_values);
  DeviceGuard dg(s->dev);
  if (!dg.ok) return fail(GG_ERR_HIP, "hipSetDevice failed");
  gg_status st = copy_in(values, (size_t)n_values * 4, where, hv.data());
  if (st != GG_OK) return st;
  for (float f : hv)
    if (!std::isfinite(f)) return fail(GG_ERR_INVALID, "non-finite grid value");
  float* d = nullptr;
  if (n_values > 0) {
    if (dev_alloc(&d, (size_t)n_values) != hipSuccess) return fail(GG_ERR_OOM, "grid allocation failed");
    hipError_t e = hipMemcpy(d, hv.data(), (size_t)n_values * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return hip_fail(s, e, "grid upload");
    }
  }
  if (s->stream) HIPCHK(s, hipStreamSynchronize(s->stream));  // no step still reads the old values
  // the recorded forward's body records point into the old values
  s->tape_ok = false;
  if (s->d_grid_values) HIPCHK(s, hipFree(s->d_grid_values));
  s->d_grid_values = d;
  s->grids = G;
  return GG_OK;
}

// One attempt at n_steps steps with the current contact capacity (gg_step's
// work; tw: n_steps x bodies x 6 twists, or empty to keep the bodies' own).
gg_status run_steps(gg_sim* s, int32_t n_steps, const std::vector<float>& tw) {
  const int nb = (int)s->bodies.size();
  s->stats.steps_done = 0;
  s->stats.last_status = GG_OK;
  if (n_steps == 0) return GG_OK;

  // ---- body poses for every step (double precision), staged for upload
  const int64_t need = (int64_t)n_steps * std::max(nb, 1);
  if (need > s->d_bodies_cap) {
    if (s->d_bodies) HIPCHK(s, hipFree(s->d_bodies));
    if (s->h_bodies) HIPCHK(s, hipHostFree(s->h_bodies));
    s->d_bodies = nullptr;
    s->h_bodies = nullptr;
    s->d_bodies_cap = 0;
    if (dev_alloc(&s->d_bodies, (size_t)need) != hipSuccess ||
        hipHostMalloc((void**)&s->h_bodies, (size_t)need * sizeof(ggk::DevBody), hipHostMallocDefault) != hipSuccess)
      return fail(GG_ERR_OOM, "body staging allocation failed");
    s->d_bodies_cap = need;
    ++s->epoch;   // captured launches name the old staging buffer
  }
  s->pose_hist.resize((size_t)(n_steps + 1) * nb);
  std::vector<HostBody> cur = s->bodies;
  for (int st = 0; st < n_steps; ++st) {
    for (int b = 0; b < nb; ++b) {
      if (!tw.empty()) {
        const float* t6 = &tw[((size_t)st * nb + b) * 6];
        for (int q = 0; q < 3; ++q) {
          cur[b].nu[q] = t6[q];
          cur[b].om[q] = t6[3 + q];
        }
      }
      const gg_grid* gr = cur[b].shape == GG_GRID ? &s->grids[cur[b].grid] : nullptr;
      s->h_bodies[(size_t)st * nb + b] = to_dev(cur[b], gr, s->d_grid_values, s->r_max);
      s->pose_hist[(size_t)st * nb + b] = cur[b];
      advance_pose(cur[b], (double)s->p.dt);
    }
  }
  for (int b = 0; b < nb; ++b) s->pose_hist[(size_t)n_steps * nb + b] = cur[b];
  if (nb > 0)
    HIPCHK(s, hipMemcpyAsync(s->d_bodies, s->h_bodies, (size_t)n_steps * nb * sizeof(ggk::DevBody),
                             hipMemcpyHostToDevice, s->stream));

  const bool prof = (s->p.flags & GG_FLAG_PROFILE) != 0;
  if (prof) {
    size_t ne = (size_t)n_steps * 4;
    while (s->events.size() < ne) {
      hipEvent_t ev;
      HIPCHK(s, hipEventCreate(&ev));
      s->events.push_back(ev);
    }
  }

  const int n = (int)s->n;
  const int K = s->K;
  hipStream_t S = s->stream;

  const bool taped = (s->p.flags & GG_FLAG_TAPE) != 0;
  s->tape_ok = false;
  if (taped && n > 0) {
    const int C = s->p.checkpoint_every;
    const int nseg = (n_steps + C - 1) / C;
    const size_t need_ck = (size_t)nseg * 2 * (size_t)n;
    if (need_ck > s->ck_cap) {
      if (s->ck) HIPCHK(s, hipFree(s->ck));
      s->ck = nullptr;
      s->ck_cap = 0;
      if (dev_alloc_bytes(&s->ck, need_ck * s->es4) != hipSuccess)
        return fail(GG_ERR_OOM, "checkpoint allocation failed");
      s->ck_cap = need_ck;
    }
    if ((size_t)n_steps * 2 > s->d_counts_cap) {
      if (s->d_counts) HIPCHK(s, hipFree(s->d_counts));
      s->d_counts = nullptr;
      s->d_counts_cap = 0;
      if (dev_alloc(&s->d_counts, (size_t)n_steps * 2) != hipSuccess) return fail(GG_ERR_OOM, "count allocation failed");
      s->d_counts_cap = (size_t)n_steps * 2;
    }
  }
  s->imp_rows = (s->p.flags & GG_FLAG_FUSED) || s->p.pja_lanes == 1;   // (launch_sweeps, the fused step)
  const bool graphed = (s->p.flags & GG_FLAG_GRAPH) && !(s->p.flags & GG_FLAG_FUSED) && !prof && !taped && n > 0;
  if (graphed) {
    gg_status gs = launch_graphed(s, n_steps, nb);
    if (gs != GG_OK) return gs;
  } else {
    gg_status es = enqueue_steps(s, n_steps, nb, taped, prof);
    if (es != GG_OK) return es;
  }
  HIPCHK(s, hipGetLastError());
  HIPCHK(s, hipMemcpyAsync(s->h_ctl, s->ctl, sizeof(ggk::Ctl), hipMemcpyDeviceToHost, S));
  HIPCHK(s, hipStreamSynchronize(S));

  const ggk::Ctl c = *s->h_ctl;
  int done = n > 0 ? c.steps_done : n_steps;
  if (done < 0) done = 0;
  if (done > n_steps) done = n_steps;
  for (int b = 0; b < nb; ++b) s->bodies[b] = s->pose_hist[(size_t)done * nb + b];
  if (!tw.empty() && done > 0)
    for (int b = 0; b < nb; ++b) {
      const float* t6 = &tw[((size_t)(done - 1) * nb + b) * 6];
      for (int q = 0; q < 3; ++q) {
        s->bodies[b].nu[q] = t6[q];
        s->bodies[b].om[q] = t6[3 + q];
      }
    }
  s->stats.steps_done = done;
  s->stats.steps_total += done;
  sample_memory(s);
  s->steps_global += n_steps;
  if (n > 0) {
    s->stats.n_pp = (int64_t)c.n_pp;
    s->stats.n_pb = (int64_t)c.n_pb;
    s->stats.candidates = (int64_t)c.cand;
    s->stats.max_contacts = c.max_cnt;
    s->stats.contacts_summed = (int64_t)c.summed;
    s->stats.detect_fallback = c.fallback;
    s->stats.detect_items = c.items;
  }
  s->stats.capacity = K;
  if (prof && n > 0) {
    double td = 0, tp = 0, ti = 0;
    for (int st = 0; st < n_steps; ++st) {
      float a = 0, b2 = 0, c3 = 0;
      HIPCHK(s, hipEventElapsedTime(&a, s->events[4 * st], s->events[4 * st + 1]));
      HIPCHK(s, hipEventElapsedTime(&b2, s->events[4 * st + 1], s->events[4 * st + 2]));
      HIPCHK(s, hipEventElapsedTime(&c3, s->events[4 * st + 2], s->events[4 * st + 3]));
      td += a;
      tp += b2;
      ti += c3;
    }
    s->stats.ms_detect = td;
    s->stats.ms_pja = tp;
    s->stats.ms_integrate = ti;
    s->stats.pja_launches = (int64_t)n_steps * s->p.n_iters;
  }
  if (c.err != 0) {
    s->stats.last_status = c.err;
    s->contacts_valid = false;
    if (c.err == GG_ERR_CAPACITY)
      return fail(GG_ERR_CAPACITY, "a particle exceeded the contact capacity of " + std::to_string(K) +
                                       " at step " + std::to_string(c.fail_step) + " of the call");
    return fail((gg_status)c.err, "non-finite or out-of-range position at step " + std::to_string(c.fail_step));
  }
  s->contacts_valid = n > 0;
  if (taped && n > 0) {
    s->tape_ok = true;
    s->tape_steps = n_steps;
    s->tape_twists.assign((size_t)n_steps * nb * 6, 0.0f);
    for (int st = 0; st < n_steps; ++st)
      for (int b = 0; b < nb; ++b) {
        const HostBody& H = s->pose_hist[(size_t)st * nb + b];
        for (int q = 0; q < 3; ++q) {
          s->tape_twists[((size_t)st * nb + b) * 6 + q] = (float)H.nu[q];
          s->tape_twists[((size_t)st * nb + b) * 6 + 3 + q] = (float)H.om[q];
        }
      }
    s->tape_poses = s->pose_hist;
    s->tape_counts.assign((size_t)n_steps * 2, 0);
    HIPCHK(s, hipMemcpy(s->tape_counts.data(), s->d_counts, (size_t)n_steps * 2 * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost));
  }
  return GG_OK;
}


gg_status gg_step(gg_sim* s, int32_t n_steps, const float* twists, gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (n_steps < 0) return fail(GG_ERR_INVALID, "n_steps must be >= 0");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  const int nb = (int)s->bodies.size();
  DeviceGuard g(s->dev);
  if (!g.ok) return fail(GG_ERR_HIP, "hipSetDevice failed");
  std::vector<float> tw;
  if (twists && nb > 0 && n_steps > 0) {
    tw.resize((size_t)n_steps * nb * 6);
    gg_status st = copy_in(twists, tw.size() * 4, where, tw.data());
    if (st != GG_OK) return st;
    for (float f : tw)
      if (!std::isfinite(f)) return fail(GG_ERR_INVALID, "non-finite twist");
  }
  for (const HostBody& b : s->bodies)
    if (b.shape == GG_GRID && (b.grid < 0 || b.grid >= (int32_t)s->grids.size()))
      return fail(GG_ERR_INVALID, "a grid body refers to a grid that is no longer registered");
  // Automatic capacity (max_contacts_per_particle 0): a step that would exceed
  // the current capacity is abandoned before any impulse, as always; the
  // capacity then grows (at most to the packing bound) and the call goes on
  // from that step -- a differentiable call from its start, restored from its
  // first checkpoint, so that its record is one pass.  Contact lists do not
  // depend on the capacity, so neither do the results.
  const bool taped = (s->p.flags & GG_FLAG_TAPE) != 0;
  const std::vector<HostBody> bodies0 = s->bodies;
  int first = 0;
  for (;;) {
    std::vector<float> rest;
    if (!tw.empty()) rest.assign(tw.begin() + (size_t)first * nb * 6, tw.end());
    const gg_status r = run_steps(s, n_steps - first, rest);
    const int done = (int)s->stats.steps_done;
    const int bound = bound_K(s);
    if (r != GG_ERR_CAPACITY || s->p.max_contacts_per_particle != 0 || s->K >= bound ||
        !slots_fit(s->n_pad, std::min(bound, std::max(2 * s->K, (int)s->stats.max_contacts)))) {
      s->stats.steps_done += first;
      return r;
    }
    const int K = std::min(bound, (std::max(2 * s->K, (int)s->stats.max_contacts) + 1) & ~1);
    s->K_floor = std::max(s->K_floor, K);
    gg_status e = ensure_ell(s, K);
    if (e != GG_OK) return e;
    if (taped) {
      // back to the call's start: the first checkpoint and the first poses
      const size_t n4 = (size_t)s->n * s->es4;
      HIPCHK(s, hipMemcpyAsync(s->x, s->ck, n4, hipMemcpyDeviceToDevice, s->stream));
      HIPCHK(s, hipMemcpyAsync(s->v, (char*)s->ck + n4, n4, hipMemcpyDeviceToDevice, s->stream));
      HIPCHK(s, hipStreamSynchronize(s->stream));
      s->bodies = bodies0;
      s->stats.steps_total -= done;
      first = 0;
    } else {
      first += done;
    }
    g_detail.clear();
  }
}

// Left Jacobian of SO(3): Exp(phi + d) ~= Exp([J_l(phi) d]x) Exp(phi).
static void so3_left_jacobian(const double phi[3], double J[9]) {
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  const double th = std::sqrt(th2);
  double a, b;
  if (th < 1e-6) {
    a = 0.5 - th2 / 24.0;
    b = 1.0 / 6.0 - th2 / 120.0;
  } else {
    a = (1.0 - std::cos(th)) / th2;
    b = (th - std::sin(th)) / (th2 * th);
  }
  const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double kk = 0;
      for (int m = 0; m < 3; ++m) kk += K[3 * r + m] * K[3 * m + c];
      J[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * kk;
    }
}

static void so3_exp(const double phi[3], double E[9]) {
  HostBody tmp{};
  for (int q = 0; q < 9; ++q) tmp.R[q] = (q % 4 == 0) ? 1.0 : 0.0;
  for (int q = 0; q < 3; ++q) tmp.om[q] = phi[q];
  advance_pose(tmp, 1.0);
  std::memcpy(E, tmp.R, sizeof(tmp.R));
}

gg_status gg_step_backward(gg_sim* s, const float* dL_dx, const float* dL_dv, float* dL_dx0, float* dL_dv0,
                           float* dL_dtwists, gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  if (!(s->p.flags & GG_FLAG_TAPE)) return fail(GG_ERR_NO_TAPE, "the simulation was created without GG_FLAG_TAPE");
  if (!s->tape_ok || s->tape_steps <= 0) return fail(GG_ERR_NO_TAPE, "no successful differentiable gg_step to reverse");
  if (s->n_envs != 1) return fail(GG_ERR_UNSUPPORTED, "the adjoint is built for one environment");
  return s->fp64 ? backward_t<double>(s, dL_dx, dL_dv, dL_dx0, dL_dv0, dL_dtwists, where)
                 : backward_t<float>(s, dL_dx, dL_dv, dL_dx0, dL_dv0, dL_dtwists, where);
}

}  // extern "C"

namespace {

// Reverse pass of the last recorded call in the build's precision R.
template <typename R>
gg_status backward_t(gg_sim* s, const float* dL_dx, const float* dL_dv, float* dL_dx0, float* dL_dv0,
                     float* dL_dtwists, gg_mem where) {
  using V = ggk::V4<R>;
  const int n = (int)s->n;
  const int nb = (int)s->bodies.size();
  const int N = s->tape_steps;
  const int I = s->p.n_iters;
  const int C = s->p.checkpoint_every;
  const int K = s->K;
  const size_t slots = (size_t)s->n_pad * K;
  const int grid = (n + ggk::kBlock - 1) / ggk::kBlock;
  hipStream_t S = s->stream;
  DeviceGuard g(s->dev);
  if (!g.ok) return fail(GG_ERR_HIP, "hipSetDevice failed");

  // ---- device buffers for one segment of recorded steps and the adjoint
  std::vector<void*> owned;
  auto alloc = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) return nullptr;
    owned.push_back(p);
    return p;
  };
  auto release = [&]() {
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
  };
  const size_t n4 = (size_t)n * sizeof(V);
  // half contacts of every recorded step (a pair counts in both rows)
  std::vector<size_t> hc(N);
  size_t hc_max_seg = 1, hc_max = 1;
  for (int st = 0; st < N; ++st) {
    hc[st] = 2 * (size_t)s->tape_counts[2 * st] + (size_t)s->tape_counts[2 * st + 1];
    hc_max = std::max(hc_max, hc[st]);
  }
  for (int seg = 0; seg * C < N; ++seg) {
    size_t sum = 0;
    for (int st = seg * C; st < std::min(N, seg * C + C); ++st) sum += hc[st];
    hc_max_seg = std::max(hc_max_seg, sum);
  }
  const size_t nsw = (size_t)std::max(I - 1, 1);
  V* tx = (V*)alloc(n4 * C);
  V* tv = (V*)alloc(n4 * C);
  int32_t* tncon = (int32_t*)alloc((size_t)n * 4 * C);
  int32_t* tpart = (int32_t*)alloc(slots * 4 * C);
  R* tpsi = (R*)alloc(slots * sizeof(R) * C);
  V* tw = (V*)alloc(n4 * (size_t)I * C);
  R* tP = (R*)alloc(hc_max_seg * sizeof(R) * 3 * nsw);
  R* Plast = (R*)alloc(hc_max * sizeof(R) * 3);
  int32_t* tpofs = (int32_t*)alloc(((size_t)n + 1) * 4 * C);
  int32_t* pbsum = (int32_t*)alloc(((size_t)n + ggk::kScanTile) / ggk::kScanTile * 4 + 16);
  V* xw = (V*)alloc(n4);
  V* vw = (V*)alloc(n4);
  V* xb = (V*)alloc(n4);
  V* vb = (V*)alloc(n4);
  V* xbn = (V*)alloc(n4);
  V* vbn = (V*)alloc(n4);
  V* wba = (V*)alloc(n4);
  V* wbb = (V*)alloc(n4);
  V* w0b = (V*)alloc(n4);
  // adjoint state: the carry per contact-table slot, the body-contact
  // accumulators per contact (compact index)
  const size_t aslots = (size_t)s->n_pad * (size_t)K;
  R* adj = (R*)alloc((aslots * 3 + hc_max * 7) * sizeof(R));
  R* part = (R*)alloc((size_t)grid * std::max(nb, 1) * 18 * sizeof(R));
  R* bgrad = (R*)alloc((size_t)std::max(nb, 1) * 18 * sizeof(R) * N);
  float* io3 = (float*)alloc((size_t)n * 12 * 2);
  for (void* p : owned)
    if (!p) {
      release();
      return fail(GG_ERR_OOM, "adjoint workspace allocation failed");
    }
  if (owned.size() != 23) {
    release();
    return fail(GG_ERR_OOM, "adjoint workspace allocation failed");
  }
  sample_memory(s);
  ggk::AdjSlots<R> A;
  A.cx = adj; A.cy = adj + aslots; A.cz = adj + 2 * aslots;
  R* const abody = adj + 3 * aslots;
  A.nx = abody; A.ny = abody + hc_max; A.nz = abody + 2 * hc_max;
  A.ps = abody + 3 * hc_max;
  A.vx = abody + 4 * hc_max; A.vy = abody + 5 * hc_max; A.vz = abody + 6 * hc_max;

  // ---- final-state adjoints into the internal order
  const hipMemcpyKind kin = where == GG_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  const hipMemcpyKind kout = where == GG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
#define BWCHK(expr)                         \
  do {                                      \
    hipError_t _e = (expr);                 \
    if (_e != hipSuccess) {                 \
      release();                            \
      return hip_fail(s, _e, #expr);        \
    }                                       \
  } while (0)
  if (dL_dx) BWCHK(hipMemcpyAsync(io3, dL_dx, (size_t)n * 12, kin, S));
  if (dL_dv) BWCHK(hipMemcpyAsync(io3 + 3 * (size_t)n, dL_dv, (size_t)n * 12, kin, S));
  ggk::k_gather3<R><<<grid, ggk::kBlock, 0, S>>>(n, s->orig, dL_dx ? io3 : nullptr, xbn);
  ggk::k_gather3<R><<<grid, ggk::kBlock, 0, S>>>(n, s->orig, dL_dv ? io3 + 3 * (size_t)n : nullptr, vbn);

  const R dt = (R)s->p.dt;
  const R alpha_dt = (R)s->p.alpha / (R)s->p.dt;
  const int nseg = (N + C - 1) / C;
  for (int seg = nseg - 1; seg >= 0; --seg) {
    const int s0 = seg * C, s1 = std::min(N, s0 + C);
    // recompute the segment from its checkpoint, recording every step
    BWCHK(hipMemcpyAsync(xw, (V*)s->ck + (size_t)seg * 2 * n, n4, hipMemcpyDeviceToDevice, S));
    BWCHK(hipMemcpyAsync(vw, (V*)s->ck + (size_t)seg * 2 * n + n, n4, hipMemcpyDeviceToDevice, S));
    std::vector<size_t> pstart(C + 1, 0);   // first recorded impulse of each step of the segment
    for (int st = s0; st < s1; ++st) pstart[st - s0 + 1] = pstart[st - s0] + hc[st] * 3 * nsw;
    for (int st = s0; st < s1; ++st) {
      const int r = st - s0;
      const ggk::DevBody* bod = s->d_bodies + (size_t)st * nb;
      BWCHK(hipMemcpyAsync(tx + (size_t)r * n, xw, n4, hipMemcpyDeviceToDevice, S));
      BWCHK(hipMemcpyAsync(tv + (size_t)r * n, vw, n4, hipMemcpyDeviceToDevice, S));
      StepIO<R> io;
      io.x = xw;
      io.v = vw;
      io.ncon = tncon + (size_t)r * n;
      io.imass = (R*)s->imass;
      io.partner = tpart + slots * r;
      io.Psi = tpsi + slots * r;
      io.w.resize(I + 1);
      io.Px.resize(I + 1); io.Py.resize(I + 1); io.Pz.resize(I + 1);
      for (int l = 0; l < I; ++l) io.w[l] = tw + ((size_t)r * I + l) * n;
      io.w[I] = wba;  // unused: the last sweep writes the velocity
      for (int l = 1; l <= I; ++l) {
        R* base = (l < I) ? tP + pstart[r] + (size_t)(l - 1) * 3 * hc[st] : Plast;
        io.Px[l] = base; io.Py[l] = base + hc[st]; io.Pz[l] = base + 2 * hc[st];
      }
      io.Px[0] = io.Px[1]; io.Py[0] = io.Py[1]; io.Pz[0] = io.Pz[1];
      io.dv = nullptr;
      io.pofs = tpofs + (size_t)r * (n + 1);
      launch_detect<R>(s, io, st, bod);
      // compact offsets of this step's contacts; the recorded count must match
      const int pnb = (n + ggk::kScanTile - 1) / ggk::kScanTile;
      ggk::k_scan_a<<<pnb, ggk::kBlock, 0, S>>>(n, io.ncon, io.pofs, pbsum, 0);
      ggk::k_scan_b<<<1, 1024, 0, S>>>(pnb, pbsum, n, io.pofs);
      ggk::k_scan_c<<<pnb, ggk::kBlock, 0, S>>>(n, pbsum, io.pofs);
      int32_t total = -1;
      BWCHK(hipMemcpyAsync(&total, io.pofs + n, 4, hipMemcpyDeviceToHost, S));
      BWCHK(hipStreamSynchronize(S));
      if ((size_t)total != hc[st]) {
        release();
        return fail(GG_ERR_HIP, "recomputed contacts differ from the recorded forward");
      }
      launch_sweeps<R>(s, io, bod);
      ggk::k_integrate<R><<<grid, ggk::kBlock, 0, S>>>(n, xw, vw, dt, cyc_lo<R>(s), cyc_span<R>(s), s->ctl,
                                                       s->det_part, detect_grid(s), nullptr);
    }
    // reverse the segment
    for (int st = s1 - 1; st >= s0; --st) {
      const int r = st - s0;
      const V* xk = tx + (size_t)r * n;
      const V* vk = tv + (size_t)r * n;
      const int32_t* nc = tncon + (size_t)r * n;
      const int32_t* pt = tpart + slots * r;
      const R* ps = tpsi + slots * r;
      const ggk::DevBody* bod = s->d_bodies + (size_t)st * nb;
      ggk::k_adj_begin<R><<<grid, ggk::kBlock, 0, S>>>(n, xbn, vbn, vk, dt, xb, wba, w0b);
      // (no zeroing of the adjoint state: the first reverse sweep, l = I >= 1,
      // writes every slot in use before anything reads it)
      V* win = wba;
      V* wout = wbb;
      const int32_t* po = tpofs + (size_t)r * (n + 1);
      for (int l = I; l >= 1; --l) {
        const V* wprev = tw + ((size_t)r * I + (l - 1)) * n;
        const R* Pp = (l >= 2) ? tP + pstart[r] + (size_t)(l - 2) * 3 * hc[st] : nullptr;
        const int Ln = s->p.pja_lanes;
        const int lg = (int)(((int64_t)n * Ln + ggk::kBlock - 1) / ggk::kBlock);
        if (Ln == 1)
          ggk::k_pja_adj<R><<<grid, ggk::kBlock, 0, S>>>(n, K, xk, vk, wprev, win, wout, w0b, nc, pt, ps, Pp,
                                                      Pp ? Pp + hc[st] : nullptr, Pp ? Pp + 2 * hc[st] : nullptr,
                                                      A, bod, alpha_dt, (R)s->p.mu, (R)s->p.relax, l == 1 ? 1 : 0,
                                                      l == I ? 1 : 0, po, xb);
        else if (Ln == 2)
          ggk::k_pja_adj_lanes<R, 2><<<lg, ggk::kBlock, 0, S>>>(
              n, K, xk, vk, wprev, win, wout, w0b, nc, pt, ps, Pp, Pp ? Pp + hc[st] : nullptr,
              Pp ? Pp + 2 * hc[st] : nullptr, A, bod, alpha_dt, (R)s->p.mu, (R)s->p.relax, l == 1 ? 1 : 0,
              l == I ? 1 : 0, po, xb);
        else
          ggk::k_pja_adj_lanes<R, 4><<<lg, ggk::kBlock, 0, S>>>(
              n, K, xk, vk, wprev, win, wout, w0b, nc, pt, ps, Pp, Pp ? Pp + hc[st] : nullptr,
              Pp ? Pp + 2 * hc[st] : nullptr, A, bod, alpha_dt, (R)s->p.mu, (R)s->p.relax, l == 1 ? 1 : 0,
              l == I ? 1 : 0, po, xb);
        std::swap(win, wout);
      }
      ggk::k_adj_vbar<R><<<grid, ggk::kBlock, 0, S>>>(n, w0b, win, vb);
      ggk::k_geom_adj<R><<<grid, ggk::kBlock, 0, S>>>(n, K, xk, nc, pt, ps, A, bod, nb, po, xb, part);
      if (nb > 0)
        ggk::k_body_reduce<R><<<nb * 18, ggk::kBlock, 0, S>>>(grid, nb, part, bgrad + (size_t)st * nb * 18);
      std::swap(xb, xbn);
      std::swap(vb, vbn);
    }
  }
  BWCHK(hipGetLastError());
  // ---- outputs
  ggk::k_unpermute3<R><<<grid, 256, 0, S>>>(n, s->orig, xbn, io3);
  ggk::k_unpermute3<R><<<grid, 256, 0, S>>>(n, s->orig, vbn, io3 + 3 * (size_t)n);
  if (dL_dx0) BWCHK(hipMemcpyAsync(dL_dx0, io3, (size_t)n * 12, kout, S));
  if (dL_dv0) BWCHK(hipMemcpyAsync(dL_dv0, io3 + 3 * (size_t)n, (size_t)n * 12, kout, S));
  std::vector<R> hb((size_t)std::max(nb, 1) * 18 * N, R(0));
  if (nb > 0) BWCHK(hipMemcpyAsync(hb.data(), bgrad, hb.size() * sizeof(R), hipMemcpyDeviceToHost, S));
  BWCHK(hipStreamSynchronize(S));
  release();
#undef BWCHK

  // ---- twists: direct (body point velocity) plus the pose chain, in double
  if (dL_dtwists) {
    std::vector<float> out((size_t)N * nb * 6, 0.0f);
    for (int b = 0; b < nb; ++b) {
      double Racc[9] = {0}, tacc[3] = {0};  // adjoint of the pose after step st
      for (int st = N - 1; st >= 0; --st) {
        const HostBody& P0 = s->tape_poses[(size_t)st * nb + b];      // pose at step st
        const HostBody& P1 = s->tape_poses[(size_t)(st + 1) * nb + b];  // pose after step st
        const R* gq = &hb[((size_t)st * nb + b) * 18];
        double gnu[3], gom[3];
        for (int q = 0; q < 3; ++q) {
          gnu[q] = gq[q] + dt * tacc[q];
          gom[q] = gq[3 + q];
        }
        // R1 = E R0 with E = Exp(dt omega): d/d omega through the left Jacobian
        const double phi[3] = {dt * P0.om[0], dt * P0.om[1], dt * P0.om[2]};
        double M[9];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += Racc[3 * r + m] * P1.R[3 * c + m];
            M[3 * r + c] = acc;
          }
        const double gxi[3] = {M[7] - M[5], M[2] - M[6], M[3] - M[1]};
        double J[9];
        so3_left_jacobian(phi, J);
        for (int q = 0; q < 3; ++q) gom[q] += dt * (J[q] * gxi[0] + J[3 + q] * gxi[1] + J[6 + q] * gxi[2]);
        for (int q = 0; q < 3; ++q) {
          out[((size_t)st * nb + b) * 6 + q] = (float)gnu[q];
          out[((size_t)st * nb + b) * 6 + 3 + q] = (float)gom[q];
        }
        // adjoint of the pose at step st: back through the advance, plus this step's geometry
        double E[9];
        so3_exp(phi, E);
        double R0b[9];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += E[3 * m + r] * Racc[3 * m + c];
            R0b[3 * r + c] = acc;
          }
        for (int q = 0; q < 9; ++q) Racc[q] = R0b[q] + gq[6 + q];
        for (int q = 0; q < 3; ++q) tacc[q] += gq[15 + q];
      }
    }
    if (where == GG_MEM_HOST) {
      std::memcpy(dL_dtwists, out.data(), out.size() * 4);
    } else {
      HIPCHK(s, hipMemcpy(dL_dtwists, out.data(), out.size() * 4, hipMemcpyHostToDevice));
    }
  }
  return GG_OK;
}


// Per-call workspace of the goal reward: partial sums per chunk, the staged
// boxes, and the staged results for host outputs.
struct RewardWork {
  double* part_d;
  int32_t* part_n;
  float* boxes;
  double* reward;
  int64_t* inside;
};

gg_status reward_check(gg_sim* s, const float* boxes, const double* reward, gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  if (!boxes || !reward) return fail(GG_ERR_INVALID, "boxes and reward are required");
  for (int e = 0; e < s->n_envs; ++e)
    for (int q = 0; q < 3; ++q) {
      const float lo = boxes[6 * e + q], hi = boxes[6 * e + 3 + q];
      if (!std::isfinite(lo) || !std::isfinite(hi) || lo > hi)
        return fail(GG_ERR_INVALID, "goal boxes must be finite with lo <= hi");
    }
  return GG_OK;
}

// Stage the boxes, sum each chunk, combine the chunks of each environment in
// order, copy host results out; returns after the results are written.
gg_status reward_run(gg_sim* s, const float* boxes, double* reward, int64_t* inside, gg_mem where,
                     const RewardWork& W) {
  const int ne = s->n_envs;
  HIPCHK(s, hipMemcpyAsync(W.boxes, boxes, (size_t)ne * 24, hipMemcpyHostToDevice, s->stream));
  if (s->n_chunks > 0) {
    if (s->fp64)
      ggk::k_reward_chunks<double><<<s->n_chunks, ggk::kBlock, 0, s->stream>>>((const double4*)s->x, s->d_chunks,
                                                                            W.boxes, W.part_d, W.part_n);
    else
      ggk::k_reward_chunks<float><<<s->n_chunks, ggk::kBlock, 0, s->stream>>>((const float4*)s->x, s->d_chunks,
                                                                           W.boxes, W.part_d, W.part_n);
    HIPCHK(s, hipGetLastError());
  }
  double* rw = where == GG_MEM_DEVICE ? reward : W.reward;
  int64_t* in = where == GG_MEM_DEVICE ? inside : (inside ? W.inside : nullptr);
  if (ne > 0) {
    ggk::k_reward_envs<<<(ne + 255) / 256, 256, 0, s->stream>>>(ne, s->d_env_chunk, s->d_env_count, W.part_d,
                                                                 W.part_n, rw, in);
    HIPCHK(s, hipGetLastError());
  }
  if (where == GG_MEM_HOST && ne > 0) {
    HIPCHK(s, hipMemcpyAsync(reward, W.reward, (size_t)ne * 8, hipMemcpyDeviceToHost, s->stream));
    if (inside) HIPCHK(s, hipMemcpyAsync(inside, W.inside, (size_t)ne * 8, hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return GG_OK;
}

// Address of this device's copy of the no-allocation workspace, taken once per
// device with that device current (the array's name in host code is not a
// device address).
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

gg_status scratch_address(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(GG_ERR_INVALID, "device index beyond the workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(GG_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return GG_OK;
}

}  // namespace

extern "C" {

gg_status gg_read(gg_sim* s, int32_t field, void* dst, int64_t capacity_bytes, int64_t* written, gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  const int64_t n = s->n;
  int64_t need = 0;
  const int64_t C = s->contacts_valid ? s->stats.n_pp + s->stats.n_pb : 0;
  switch (field) {
    case GG_FIELD_POS:
    case GG_FIELD_VEL:
    case GG_FIELD_DV: need = 12 * n; break;
    case GG_FIELD_RADIUS: need = 4 * n; break;
    case GG_FIELD_CELL_INDEX: need = 8 * n; break;
    case GG_FIELD_CONTACTS: need = 8 * C; break;
    case GG_FIELD_IMPULSES: need = 12 * C; break;
    case GG_FIELD_STATS: need = sizeof(gg_stats); break;
    case GG_FIELD_BODY_POSES: need = 48 * (int64_t)s->bodies.size(); break;
    default: return fail(GG_ERR_INVALID, "unknown field");
  }
  if (field == GG_FIELD_DV && !s->dv) return fail(GG_ERR_INVALID, "GG_FIELD_DV needs GG_FLAG_DIAGNOSTICS at creation");
  if (written) *written = need;
  if (!dst) return GG_OK;
  if (capacity_bytes < need) return fail(GG_ERR_INVALID, "destination too small");
  if (need == 0) return GG_OK;
  DeviceGuard g(s->dev);
  const hipMemcpyKind kind = where == GG_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (field == GG_FIELD_STATS) {
    if (where == GG_MEM_HOST) {
      std::memcpy(dst, &s->stats, sizeof(gg_stats));
    } else {
      HIPCHK(s, hipMemcpy(dst, &s->stats, sizeof(gg_stats), hipMemcpyHostToDevice));
    }
    return GG_OK;
  }
  if (field == GG_FIELD_BODY_POSES) {
    std::vector<float> poses(12 * s->bodies.size());
    for (size_t b = 0; b < s->bodies.size(); ++b)
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) poses[12 * b + 4 * r + c] = (float)s->bodies[b].R[3 * r + c];
        poses[12 * b + 4 * r + 3] = (float)s->bodies[b].t[r];
      }
    if (where == GG_MEM_HOST)
      std::memcpy(dst, poses.data(), (size_t)need);
    else
      HIPCHK(s, hipMemcpy(dst, poses.data(), (size_t)need, hipMemcpyHostToDevice));
    return GG_OK;
  }
  const int blocks = (int)((n + 255) / 256);
  if (field == GG_FIELD_POS || field == GG_FIELD_VEL || field == GG_FIELD_DV || field == GG_FIELD_RADIUS ||
      field == GG_FIELD_CELL_INDEX) {
    gg_status st = ensure_tmp(s, (size_t)need);
    if (st != GG_OK) return st;
    float* f = (float*)s->tmp;
    const void* src = field == GG_FIELD_POS ? s->x : field == GG_FIELD_VEL ? s->v : field == GG_FIELD_DV ? s->dv : s->x;
    if (field == GG_FIELD_POS || field == GG_FIELD_VEL || field == GG_FIELD_DV) {
      if (s->fp64)
        ggk::k_unpermute3<double><<<blocks, 256, 0, s->stream>>>((int)n, s->orig, (const double4*)src, f);
      else
        ggk::k_unpermute3<float><<<blocks, 256, 0, s->stream>>>((int)n, s->orig, (const float4*)src, f);
    }
    if (field == GG_FIELD_RADIUS) {
      if (s->fp64)
        ggk::k_unpermute_w<double><<<blocks, 256, 0, s->stream>>>((int)n, s->orig, (const double4*)s->x, f);
      else
        ggk::k_unpermute_w<float><<<blocks, 256, 0, s->stream>>>((int)n, s->orig, (const float4*)s->x, f);
    }
    if (field == GG_FIELD_CELL_INDEX)
      ggk::k_unpermute_i64<<<blocks, 256, 0, s->stream>>>((int)n, s->orig, s->h6, (int64_t*)s->tmp);
    HIPCHK(s, hipGetLastError());
    HIPCHK(s, hipMemcpyAsync(dst, s->tmp, (size_t)need, kind, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return GG_OK;
  }
  // contacts / impulses: gather the per-particle lists into the canonical order
  const size_t slots = (size_t)s->n_pad * s->K;
  std::vector<int32_t> cnt(n), part(slots), org(n);
  std::vector<unsigned char> px, py, pz;   // impulses as stored (R = float or double)
  HIPCHK(s, hipMemcpyAsync(cnt.data(), s->ncon, n * 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(part.data(), s->partner, slots * 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipMemcpyAsync(org.data(), s->orig, n * 4, hipMemcpyDeviceToHost, s->stream));
  if (field == GG_FIELD_IMPULSES) {
    px.resize(slots * s->es); py.resize(slots * s->es); pz.resize(slots * s->es);
    HIPCHK(s, hipMemcpyAsync(px.data(), s->Px, slots * s->es, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(py.data(), s->Py, slots * s->es, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(pz.data(), s->Pz, slots * s->es, hipMemcpyDeviceToHost, s->stream));
  }
  HIPCHK(s, hipStreamSynchronize(s->stream));
  auto imp_at = [&](const std::vector<unsigned char>& a, size_t sl) -> float {
    if (s->fp64) {
      double d;
      std::memcpy(&d, a.data() + sl * 8, 8);
      return (float)d;
    }
    float f;
    std::memcpy(&f, a.data() + sl * 4, 4);
    return f;
  };
  struct Rec {
    int32_t a, b;
    size_t slot;
  };
  std::vector<Rec> pp, pb;
  pp.reserve((size_t)s->stats.n_pp);
  const int K = s->K;
  // impulse index of contact k of particle i: its table slot, or with one lane
  // per particle the jagged rows of its 64-group's block (rec_row)
  std::vector<size_t> rows((size_t)64 * K);
  for (int64_t i = 0; i < n; ++i) {
    if (s->imp_rows && (i & 63) == 0) {
      size_t at = (size_t)(i >> 6) * ((size_t)K << 6);
      for (int k = 0; k < K; ++k)
        for (int64_t l = i; l < std::min<int64_t>(i + 64, n); ++l)
          if (cnt[l] > k) rows[(size_t)(l - i) * K + k] = at++;
    }
    for (int k = 0; k < cnt[i]; ++k) {
      const size_t sl = (size_t)(i >> 6) * ((size_t)K << 6) + ((size_t)k << 6) + (size_t)(i & 63);
      const size_t q = s->imp_rows ? rows[(size_t)(i & 63) * K + k] : sl;
      const int32_t code = part[sl];
      if (code >= 0) {
        if ((code & ggk::kHiFlag) == 0) pp.push_back({org[i], org[code & (ggk::kHiFlag - 1)], q});
      } else {
        pb.push_back({org[i], -1 - code, q});
      }
    }
  }
  auto by_pair = [](const Rec& u, const Rec& w) { return u.a != w.a ? u.a < w.a : u.b < w.b; };
  std::sort(pp.begin(), pp.end(), by_pair);
  std::sort(pb.begin(), pb.end(), by_pair);
  std::vector<int32_t> pairs;
  std::vector<float> imp;
  for (const auto* L : {&pp, &pb})
    for (const Rec& r : *L) {
      if (field == GG_FIELD_CONTACTS) {
        pairs.push_back(r.a);
        pairs.push_back(r.b);
      } else {
        imp.push_back(imp_at(px, r.slot));
        imp.push_back(imp_at(py, r.slot));
        imp.push_back(imp_at(pz, r.slot));
      }
    }
  const void* src = field == GG_FIELD_CONTACTS ? (const void*)pairs.data() : (const void*)imp.data();
  const int64_t have = field == GG_FIELD_CONTACTS ? (int64_t)pairs.size() * 4 : (int64_t)imp.size() * 4;
  if (have != need) return fail(GG_ERR_HIP, "contact list size disagrees with the detection counters");
  if (where == GG_MEM_HOST) {
    std::memcpy(dst, src, (size_t)need);
  } else {
    HIPCHK(s, hipMemcpy(dst, src, (size_t)need, hipMemcpyHostToDevice));
  }
  return GG_OK;
}

gg_status gg_render_depth(gg_sim* s, int32_t n_cams, const gg_camera* cams, float* depth, int64_t capacity_bytes,
                          gg_mem where) {
  g_detail.clear();
  if (!s) return fail(GG_ERR_INVALID, "sim is NULL");
  if (s->failed) return fail(GG_ERR_HIP, "simulation is in a failed state");
  if (where != GG_MEM_HOST && where != GG_MEM_DEVICE) return fail(GG_ERR_INVALID, "bad gg_mem");
  if (n_cams < 0 || n_cams > 65535) return fail(GG_ERR_INVALID, "n_cams must be in 0 .. 65535");
  if (n_cams > 0 && !cams) return fail(GG_ERR_INVALID, "cams is NULL");
  std::vector<ggk::DevCamera> hc(n_cams);
  std::vector<ggk::DevPlane> hp;
  int64_t total = 0;
  int max_px = 0, max_n = 0;
  for (int k = 0; k < n_cams; ++k) {
    const gg_camera& c = cams[k];
    if (c.kind != GG_CAM_ORTHO && c.kind != GG_CAM_PERSPECTIVE) return fail(GG_ERR_INVALID, "unknown camera kind");
    if (c.width < 1 || c.width > 8192 || c.height < 1 || c.height > 8192)
      return fail(GG_ERR_INVALID, "camera width and height must be in 1 .. 8192");
    if (c.env < 0 || c.env >= s->n_envs) return fail(GG_ERR_INVALID, "camera env out of range");
    for (int q = 0; q < 12; ++q)
      if (!std::isfinite(c.pose[q])) return fail(GG_ERR_INVALID, "camera pose must be finite");
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(c.params[q]) || !(c.params[q] > 0.0f))
        return fail(GG_ERR_INVALID, "camera params[0..2] must be finite and positive");
    ggk::DevCamera& d = hc[k];
    d.kind = c.kind;
    d.width = c.width;
    d.height = c.height;
    for (int r = 0; r < 3; ++r) {
      for (int q = 0; q < 3; ++q) d.R[3 * r + q] = c.pose[4 * r + q];
      d.t[r] = c.pose[4 * r + 3];
    }
    d.p0 = c.params[0];
    d.p1 = c.params[1];
    d.far = c.params[2];
    d.su = (float)(2.0 / c.width);
    d.sv = (float)(2.0 / c.height);
    d.i0 = (int32_t)s->env_off[c.env];
    d.i1 = (int32_t)s->env_off[c.env + 1];
    d.q0 = (int32_t)hp.size();
    for (const HostBody& b : s->bodies) {
      if (b.shape != GG_PLANE || b.env != c.env) continue;
      ggk::DevPlane pl;
      for (int q = 0; q < 3; ++q) {
        pl.n[q] = (float)b.R[3 * q + 2];
        pl.t[q] = (float)b.t[q];
      }
      hp.push_back(pl);
    }
    d.q1 = (int32_t)hp.size();
    d.base = total;
    total += (int64_t)c.width * c.height;
    max_px = std::max(max_px, c.width * c.height);
    max_n = std::max(max_n, d.i1 - d.i0);
  }
  if (total > 0 && !depth) return fail(GG_ERR_INVALID, "depth is NULL");
  if (capacity_bytes < total * 4) return fail(GG_ERR_INVALID, "destination too small");
  if (total == 0) return GG_OK;
  DeviceGuard g(s->dev);
  auto grow = [&](void** buf, int64_t& cap, int64_t need_bytes) -> gg_status {
    if (need_bytes <= cap) return GG_OK;
    if (*buf) HIPCHK(s, hipFree(*buf));
    *buf = nullptr;
    cap = 0;
    if (hipMalloc(buf, (size_t)need_bytes) != hipSuccess) return fail(GG_ERR_OOM, "observation buffer allocation failed");
    cap = need_bytes;
    return GG_OK;
  };
  gg_status st = grow((void**)&s->d_cams, s->d_cams_cap, (int64_t)(n_cams * sizeof(ggk::DevCamera)));
  if (st == GG_OK) st = grow((void**)&s->d_planes, s->d_planes_cap, (int64_t)(std::max<size_t>(1, hp.size()) * sizeof(ggk::DevPlane)));
  if (st == GG_OK && where == GG_MEM_HOST) st = grow((void**)&s->obs_img, s->obs_img_cap, total * 4);
  if (st != GG_OK) return st;
  HIPCHK(s, hipMemcpyAsync(s->d_cams, hc.data(), n_cams * sizeof(ggk::DevCamera), hipMemcpyHostToDevice, s->stream));
  if (!hp.empty())
    HIPCHK(s, hipMemcpyAsync(s->d_planes, hp.data(), hp.size() * sizeof(ggk::DevPlane), hipMemcpyHostToDevice, s->stream));
  float* out = where == GG_MEM_DEVICE ? depth : s->obs_img;
  const int gx = std::max(1, std::min((max_px + ggk::kBlock - 1) / ggk::kBlock, 1024));
  ggk::k_depth_planes<<<dim3(gx, n_cams), ggk::kBlock, 0, s->stream>>>(s->d_cams, s->d_planes, out);
  HIPCHK(s, hipGetLastError());
  if (max_n > 0) {
    const int gs = std::max(1, std::min((max_n + ggk::kBlock - 1) / ggk::kBlock, 4096));
    if (s->fp64)
      ggk::k_depth_spheres<double><<<dim3(gs, n_cams), ggk::kBlock, 0, s->stream>>>(s->d_cams, (const double4*)s->x, out);
    else
      ggk::k_depth_spheres<float><<<dim3(gs, n_cams), ggk::kBlock, 0, s->stream>>>(s->d_cams, (const float4*)s->x, out);
    HIPCHK(s, hipGetLastError());
  }
  if (where == GG_MEM_HOST)
    HIPCHK(s, hipMemcpyAsync(depth, s->obs_img, (size_t)total * 4, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(s, hipStreamSynchronize(s->stream));
  return GG_OK;
}

gg_status gg_goal_reward(gg_sim* s, const float* boxes, double* reward, int64_t* inside, gg_mem where) {
  gg_status st = reward_check(s, boxes, reward, where);
  if (st != GG_OK) return st;
  const int ne = s->n_envs;
  DeviceGuard g(s->dev);
  if (!s->d_part_d) {
    const size_t nc = (size_t)std::max(1, s->n_chunks);
    bool ok = dev_alloc(&s->d_part_n, nc) == hipSuccess && dev_alloc(&s->d_part_d, nc) == hipSuccess &&
              dev_alloc(&s->d_boxes, (size_t)std::max(1, ne) * 6) == hipSuccess &&
              dev_alloc(&s->d_reward, (size_t)std::max(1, ne)) == hipSuccess &&
              dev_alloc(&s->d_inside, (size_t)std::max(1, ne)) == hipSuccess;
    if (!ok) return fail(GG_ERR_OOM, "reward buffer allocation failed");
  }
  return reward_run(s, boxes, reward, inside, where,
                    RewardWork{s->d_part_d, s->d_part_n, s->d_boxes, s->d_reward, s->d_inside});
}

gg_status gg_goal_reward_noalloc(gg_sim* s, const float* boxes, double* reward, int64_t* inside, gg_mem where) {
  gg_status st = reward_check(s, boxes, reward, where);
  if (st != GG_OK) return st;
  // the workspace carved from the device array: partial sums per chunk,
  // staged boxes, staged results (host outputs only)
  const size_t nc = (size_t)std::max(1, s->n_chunks), ne = (size_t)std::max(1, s->n_envs);
  auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t o_n = up(nc * 8), o_b = o_n + up(nc * 4), o_r = o_b + up(ne * 24), o_i = o_r + up(ne * 8);
  const size_t need = o_i + up(ne * 8);
  if (need > kNoAllocScratchBytes)
    return fail(GG_ERR_INVALID, "goal reward of " + std::to_string(s->n_chunks) + " chunks and " +
                                    std::to_string(s->n_envs) + " environments needs " + std::to_string(need) +
                                    " bytes of workspace; the no-allocation call has " +
                                    std::to_string(kNoAllocScratchBytes));
  DeviceGuard g(s->dev);
  if (!g.ok) return fail(GG_ERR_HIP, "hipSetDevice failed");
  unsigned char* w = nullptr;
  st = scratch_address(s->dev, &w);
  if (st != GG_OK) return st;
  return reward_run(s, boxes, reward, inside, where,
                    RewardWork{(double*)w, (int32_t*)(w + o_n), (float*)(w + o_b), (double*)(w + o_r),
                               (int64_t*)(w + o_i)});
}
void gg_destroy(gg_sim* s) {
  if (!s) return;
  {
    DeviceGuard g(s->dev);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_all(s);
  }
  delete s;
}

}  // extern "C"
