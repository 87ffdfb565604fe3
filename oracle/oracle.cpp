// Reference oracle for the granular contact step -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of one timestep of the method of
// "GranularGym" (arXiv 2306.01369), Sec. II:
//   * cell coordinates and the spatial hash of Eq. (6)                (Sec. II-B)
//   * the parallel linked hashmap of Alg. 2, built here sequentially
//     (push-front into table[h] / next[i])                             (Sec. II-B)
//   * the 3^3 neighbour-cell query and the sphere test ||xi-xj||^2 <= (ri+rj)^2
//                                                                      (Sec. II-B, II-C)
//   * particle-body contact through closed-form SDFs, or SDF samples on a
//     regular grid with trilinear interpolation, psi = f_G(x) - r,
//     evaluated at the inverse body pose                               (Eq. (7), Sec. II-C)
//   * contact frame (e1 = normal, e2/e3 any tangent basis)             (Fig. contact-frame)
//   * projected Jacobi over the stored contact list (Alg. 1) for the NCP of
//     Eqs. (1)-(3), with Baumgarte bias alpha*psi/dt                  (Sec. II-A)
//   * symplectic Euler: velocity first, then position                 (Eqs. (4)-(5))
//
// Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
// this library.  It shares no code, header or constant table with the GPU path.
//
// Readings taken where the paper is silent or garbled (all documented in the
// design notes):
//   - the impulse opposes the velocity residual: y = lam - mt*(u + bias*e1),
//     normal n points from j to i, psi <= 0 for touching pairs;
//   - relative velocity of a pair is w_i - w_j (gamma = 1), both sides carry
//     gravity and all impulses accumulated so far (symmetric Jacobi);
//   - each contact carries its own accumulated impulse lam_c, and the total is
//     projected (clamp normal at 0, then scale the tangential part radially to
//     radius mu*lam_n, as the listing of Alg. 1 does);
//   - per-contact effective mass by mass splitting, mt = 1/(n_i/m_i + n_j/m_j)
//     (n_i = contacts touching i), or mt = m_i/n_i for a body contact;
//   - integrator v' = v + dt*g + dv, x' = x + dt*v';
//   - cell size c is a parameter (c >= max(ri+rj)); cells kappa = rne(fl32(x*inv_c));
//     hash products in 64-bit integers, floored (non-negative) modulus;
//   - the contact decision is taken in binary32 with a fixed operation order
//     (no fused multiply-add), everything downstream is FP64.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Loops over fewer items than this run on one thread.  Every item of a loop is
// computed on its own (no shared accumulation), so the thread count never
// changes a result; tiny systems iterated thousands of times skip the
// fork-join cost.
const int64_t kOmpMin = 4096;

// ---------------------------------------------------------------- Eq. (6)
const int64_t kP1 = 73856093, kP2 = 19349663, kP3 = 83492791, kQ = 100;

int64_t floor_mod(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

int64_t hash_cell(int64_t k0, int64_t k1, int64_t k2, int64_t n_h) {
  int64_t v = (kP1 * (k0 - kQ)) ^ (kP2 * (k1 - kQ)) ^ (kP3 * (k2 - kQ));
  return floor_mod(v, n_h);
}

// round(x / c): the product is rounded once to binary32, then to the nearest
// integer with ties to even (the IEEE default rounding mode).
int64_t cell_coord(float x, float inv_c) {
  volatile float s = x * inv_c;
  return (int64_t)std::nearbyint((float)s);
}

// ---------------------------------------------------------------- bodies
enum Shape { PLANE = 0, BOX = 1, CAPSULE = 2, GRID = 3 };

struct Body {          // mirrored by the Python wrapper (ctypes)
  int32_t shape;
  int32_t env;
  float params[4];     // box: half extents; capsule: radius, half length
  double R[9];         // world <- body rotation, row major
  double t[3];         // body origin in world
  double nu[3];        // linear velocity of the body origin (world)
  double omega[3];     // angular velocity (world)
  const float* gv;     // GRID: knot values, x fastest ((c*ny + b)*nx + a)
  int32_t gn[3];       // GRID: knots per axis
  float go[3];         // GRID: body-frame position of knot (0, 0, 0)
  float gih;           // GRID: 1 / knot spacing
  int32_t gpad;
};

// Pre-computed SDF on a regular grid, trilinearly interpolated (Sec. II-C).
// Per axis u = (p - origin) * inv_spacing; cell i = min(floor(u), n - 2),
// t = u - i; the interpolant lerps a + t (b - a) along x, then y, then z.
// In binary32 (the contact decision) a point with u outside [0, n - 1] on any
// axis is outside the geometry; in FP64 u is clamped into the grid.
const float kGridOutside = 3.0e38f;

float grid_f32(const Body& b, const float p[3]) {
  int i[3];
  float t[3];
  for (int a = 0; a < 3; ++a) {
    volatile float d = p[a] - b.go[a];
    volatile float u = d * b.gih;
    if (!(u >= 0.0f && u <= (float)(b.gn[a] - 1))) return kGridOutside;
    int k = (int)std::floor((float)u);
    if (k > b.gn[a] - 2) k = b.gn[a] - 2;
    i[a] = k;
    t[a] = (float)u - (float)k;
  }
  auto V = [&](int a, int c, int e) {
    return b.gv[((int64_t)(i[2] + e) * b.gn[1] + (i[1] + c)) * b.gn[0] + (i[0] + a)];
  };
  auto lerp = [](float x, float y, float t) {
    volatile float d = y - x;
    volatile float m = t * d;
    return (float)(x + m);
  };
  float c00 = lerp(V(0, 0, 0), V(1, 0, 0), t[0]);
  float c10 = lerp(V(0, 1, 0), V(1, 1, 0), t[0]);
  float c01 = lerp(V(0, 0, 1), V(1, 0, 1), t[0]);
  float c11 = lerp(V(0, 1, 1), V(1, 1, 1), t[0]);
  float c0 = lerp(c00, c10, t[1]);
  float c1 = lerp(c01, c11, t[1]);
  return lerp(c0, c1, t[2]);
}

// FP64 value of the interpolant and its gradient with respect to p.
double grid_f64(const Body& b, const double p[3], double grad[3]) {
  int i[3];
  double t[3];
  for (int a = 0; a < 3; ++a) {
    double u = (p[a] - (double)b.go[a]) * (double)b.gih;
    u = std::min(std::max(u, 0.0), (double)(b.gn[a] - 1));
    int k = std::min((int)std::floor(u), b.gn[a] - 2);
    i[a] = k;
    t[a] = u - (double)k;
  }
  auto V = [&](int a, int c, int e) -> double {
    return b.gv[((int64_t)(i[2] + e) * b.gn[1] + (i[1] + c)) * b.gn[0] + (i[0] + a)];
  };
  // value: lerps along x, y, z
  double c00 = V(0, 0, 0) + t[0] * (V(1, 0, 0) - V(0, 0, 0));
  double c10 = V(0, 1, 0) + t[0] * (V(1, 1, 0) - V(0, 1, 0));
  double c01 = V(0, 0, 1) + t[0] * (V(1, 0, 1) - V(0, 0, 1));
  double c11 = V(0, 1, 1) + t[0] * (V(1, 1, 1) - V(0, 1, 1));
  double c0 = c00 + t[1] * (c10 - c00);
  double c1 = c01 + t[1] * (c11 - c01);
  // partial derivatives of the interpolant with respect to t, times du/dp
  double dx0 = (V(1, 0, 0) - V(0, 0, 0)) + t[1] * ((V(1, 1, 0) - V(0, 1, 0)) - (V(1, 0, 0) - V(0, 0, 0)));
  double dx1 = (V(1, 0, 1) - V(0, 0, 1)) + t[1] * ((V(1, 1, 1) - V(0, 1, 1)) - (V(1, 0, 1) - V(0, 0, 1)));
  double ih = (double)b.gih;
  grad[0] = (dx0 + t[2] * (dx1 - dx0)) * ih;
  grad[1] = ((c10 - c00) + t[2] * ((c11 - c01) - (c10 - c00))) * ih;
  grad[2] = (c1 - c0) * ih;
  return c0 + t[2] * (c1 - c0);
}

struct Params {
  double dt, alpha, mu, relax, density;
  double g[3];
  int32_t n_iters, mass_split;
  float inv_c;
  int32_t pad;
  int64_t n_h;
  double cyc_lo, cyc_hi;  // cyclic vertical boundary (off unless cyc_hi > cyc_lo)
};

// binary32 SDF with a fixed operation order (the contact decision).
float sdf_f32(const Body& b, const float x[3]) {
  float R[9], t[3];
  for (int k = 0; k < 9; ++k) R[k] = (float)b.R[k];
  for (int k = 0; k < 3; ++k) t[k] = (float)b.t[k];
  float d0 = x[0] - t[0], d1 = x[1] - t[1], d2 = x[2] - t[2];
  float p[3];
  for (int c = 0; c < 3; ++c) {
    float a0 = R[0 * 3 + c] * d0;
    float a1 = R[1 * 3 + c] * d1;
    float a2 = R[2 * 3 + c] * d2;
    float s = a0 + a1;
    p[c] = s + a2;
  }
  if (b.shape == PLANE) return p[2];
  if (b.shape == GRID) return grid_f32(b, p);
  if (b.shape == BOX) {
    float q[3], m[3];
    for (int c = 0; c < 3; ++c) {
      q[c] = std::fabs(p[c]) - b.params[c];
      m[c] = q[c] > 0.0f ? q[c] : 0.0f;
    }
    float s0 = m[0] * m[0];
    float s1 = m[1] * m[1];
    float s2 = m[2] * m[2];
    float ss = s0 + s1;
    ss = ss + s2;
    float outside = std::sqrt(ss);
    float inside = std::max(q[0], std::max(q[1], q[2]));
    inside = inside < 0.0f ? inside : 0.0f;
    return outside + inside;
  }
  // capsule
  float h = b.params[1];
  float cz = std::min(std::max(p[2], -h), h);
  float dz = p[2] - cz;
  float s0 = p[0] * p[0];
  float s1 = p[1] * p[1];
  float s2 = dz * dz;
  float ss = s0 + s1;
  ss = ss + s2;
  return std::sqrt(ss) - b.params[0];
}

bool body_touch_f32(const Body& b, const float x[3], float r) {
  float f = sdf_f32(b, x);
  float psi = f - r;
  return psi <= 0.0f;
}

// binary32 sphere-sphere decision ||xi - xj||^2 <= (ri + rj)^2 (Sec. II-C).
bool pair_touch_f32(const float xi[3], const float xj[3], float ri, float rj) {
  float dx = xi[0] - xj[0], dy = xi[1] - xj[1], dz = xi[2] - xj[2];
  float a = dx * dx, b = dy * dy, c = dz * dz;
  float D = a + b;
  D = D + c;
  float s = ri + rj;
  float S = s * s;
  return D <= S;
}

// FP64 SDF in the body frame and its unit gradient.  Ties at non-smooth points
// go to the lowest axis index; sign(0) = +1.
double sdf_f64(const Body& b, const double p[3], double grad[3]) {
  if (b.shape == PLANE) {
    grad[0] = 0; grad[1] = 0; grad[2] = 1;
    return p[2];
  }
  if (b.shape == GRID) {
    double f = grid_f64(b, p, grad);
    if (!(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2] > 0)) {
      grad[0] = 1; grad[1] = 0; grad[2] = 0;
    }
    return f;
  }
  if (b.shape == BOX) {
    double q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = std::fabs(p[c]) - (double)b.params[c];
      m[c] = q[c] > 0 ? q[c] : 0.0;
      if (q[c] > 0) outside = true;
    }
    if (outside) {
      double L = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int c = 0; c < 3; ++c) grad[c] = (p[c] < 0 ? -1.0 : 1.0) * m[c] / L;
      return L;
    }
    int a = 0;
    for (int c = 1; c < 3; ++c)
      if (q[c] > q[a]) a = c;
    grad[0] = grad[1] = grad[2] = 0;
    grad[a] = p[a] < 0 ? -1.0 : 1.0;
    return q[a];
  }
  double h = b.params[1];
  double cz = std::min(std::max(p[2], -h), h);
  double e[3] = {p[0], p[1], p[2] - cz};
  double L = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (L > 0) {
    for (int c = 0; c < 3; ++c) grad[c] = e[c] / L;
  } else {
    grad[0] = 1; grad[1] = 0; grad[2] = 0;
  }
  return L - (double)b.params[0];
}

// Any orthonormal tangent pair for the unit normal n (Frisvad's construction
// as revised by Duff et al., "Building an Orthonormal Basis, Revisited").
void tangent_basis(const double n[3], double t1[3], double t2[3]) {
  double sgn = n[2] >= 0 ? 1.0 : -1.0;
  double a = -1.0 / (sgn + n[2]);
  double b = n[0] * n[1] * a;
  t1[0] = 1.0 + sgn * n[0] * n[0] * a; t1[1] = sgn * b; t1[2] = -sgn * n[0];
  t2[0] = b; t2[1] = sgn + n[1] * n[1] * a; t2[2] = -n[1];
}

double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

struct Contact {
  int32_t i, j;      // j >= 0: particle, j < 0: body (-1 - body index)
  double n[3], t1[3], t2[3];
  double psi;
  double vel[3];     // body point velocity (body contacts)
};

// Sequential linked hashmap of Alg. 2: table[h] holds the most recently
// inserted particle of bucket h, next[i] the one inserted before i.
struct LinkedHashmap {
  std::vector<int64_t> table, next, kappa;
  void build(int64_t n, const float* x, float inv_c, int64_t n_h) {
    table.assign(n_h, -1);
    next.assign(n, -1);
    kappa.resize(3 * n);
    for (int64_t i = 0; i < n; ++i) {
      for (int a = 0; a < 3; ++a) kappa[3 * i + a] = cell_coord(x[3 * i + a], inv_c);
      int64_t h = hash_cell(kappa[3 * i], kappa[3 * i + 1], kappa[3 * i + 2], n_h);
      next[i] = table[h];
      table[h] = i;
    }
  }
};

// Particle-particle contact set through the hashmap: for each particle, the
// lists of its own cell and its 26 neighbours; a candidate counts only if it
// really lies in the queried cell (buckets may alias).  Pairs come out as
// (i, j), i < j, sorted.
void pp_contacts_grid(int64_t n, const float* x, const float* r, const int32_t* env,
                      float inv_c, int64_t n_h, std::vector<std::pair<int32_t, int32_t>>& out,
                      int64_t* candidates) {
  LinkedHashmap hm;
  hm.build(n, x, inv_c, n_h);
  std::vector<std::vector<int32_t>> partners(n);
  int64_t cand_total = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : cand_total) if (n > kOmpMin)
  for (int64_t i = 0; i < n; ++i) {
    const int64_t* ki = &hm.kappa[3 * i];
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          int64_t c0 = ki[0] + dx, c1 = ki[1] + dy, c2 = ki[2] + dz;
          int64_t h = hash_cell(c0, c1, c2, n_h);
          for (int64_t j = hm.table[h]; j >= 0; j = hm.next[j]) {
            if (j == i) continue;
            const int64_t* kj = &hm.kappa[3 * j];
            if (kj[0] != c0 || kj[1] != c1 || kj[2] != c2) continue;
            if (env && env[i] != env[j]) continue;
            ++cand_total;
            if (j > i && pair_touch_f32(&x[3 * i], &x[3 * j], r[i], r[j]))
              partners[i].push_back((int32_t)j);
          }
        }
    std::sort(partners[i].begin(), partners[i].end());
  }
  out.clear();
  for (int64_t i = 0; i < n; ++i)
    for (int32_t j : partners[i]) out.emplace_back((int32_t)i, j);
  if (candidates) *candidates = cand_total;
}

void pb_contacts(int64_t n, const float* x, const float* r, const int32_t* env, int nb,
                 const Body* bodies, std::vector<std::pair<int32_t, int32_t>>& out) {
  out.clear();
  for (int64_t i = 0; i < n; ++i)
    for (int b = 0; b < nb; ++b) {
      if (env && bodies[b].env != env[i]) continue;
      if (body_touch_f32(bodies[b], &x[3 * i], r[i])) out.emplace_back((int32_t)i, (int32_t)b);
    }
}

double particle_mass(double radius, double density) {
  return density * (4.0 / 3.0) * M_PI * radius * radius * radius;
}

}  // namespace

extern "C" {

// Eq. (6) for single cells (tests evaluate it against other sources).
int64_t ggo_hash(int64_t k0, int64_t k1, int64_t k2, int64_t n_h) { return hash_cell(k0, k1, k2, n_h); }

// Cell coordinates and bucket of every particle; env_bucket_offset/env_n_h
// (may be NULL) give per-particle bucket offsets and table sizes for
// segmented (multi-environment) tables.
void ggo_cell_index(int64_t n, const float* x, float inv_c, int64_t n_h, const int64_t* bucket_offset,
                    const int64_t* env_n_h, int64_t* kappa, int64_t* h) {
  for (int64_t i = 0; i < n; ++i) {
    int64_t k[3];
    for (int a = 0; a < 3; ++a) k[a] = cell_coord(x[3 * i + a], inv_c);
    if (kappa)
      for (int a = 0; a < 3; ++a) kappa[3 * i + a] = k[a];
    int64_t nh = env_n_h ? env_n_h[i] : n_h;
    h[i] = hash_cell(k[0], k[1], k[2], nh) + (bucket_offset ? bucket_offset[i] : 0);
  }
}

// Decisions in binary32, exposed for tests.
int32_t ggo_pair_touch(const float* xi, const float* xj, float ri, float rj) {
  return pair_touch_f32(xi, xj, ri, rj) ? 1 : 0;
}
float ggo_sdf_f32(const Body* b, const float* x) { return sdf_f32(*b, x); }
double ggo_sdf_f64(const Body* b, const double* p_body, double* grad) { return sdf_f64(*b, p_body, grad); }

// O(n^2) particle-particle contact set: every pair i < j tested directly.
int64_t ggo_pp_bruteforce(int64_t n, const float* x, const float* r, const int32_t* env, int64_t cap,
                          int32_t* pairs) {
  int64_t k = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      if (env && env[i] != env[j]) continue;
      if (pair_touch_f32(&x[3 * i], &x[3 * j], r[i], r[j])) {
        if (k < cap) {
          pairs[2 * k] = (int32_t)i;
          pairs[2 * k + 1] = (int32_t)j;
        }
        ++k;
      }
    }
  return k;
}

// Particle-particle contact set through the linked hashmap (Alg. 2 + 27-cell query).
int64_t ggo_pp_hashgrid(int64_t n, const float* x, const float* r, const int32_t* env, float inv_c,
                        int64_t n_h, int64_t cap, int32_t* pairs, int64_t* candidates) {
  std::vector<std::pair<int32_t, int32_t>> out;
  pp_contacts_grid(n, x, r, env, inv_c, n_h, out, candidates);
  for (int64_t k = 0; k < (int64_t)out.size() && k < cap; ++k) {
    pairs[2 * k] = out[k].first;
    pairs[2 * k + 1] = out[k].second;
  }
  return (int64_t)out.size();
}

int64_t ggo_pb_contacts(int64_t n, const float* x, const float* r, const int32_t* env, int32_t nb,
                        const Body* bodies, int64_t cap, int32_t* pairs) {
  std::vector<std::pair<int32_t, int32_t>> out;
  pb_contacts(n, x, r, env, nb, bodies, out);
  for (int64_t k = 0; k < (int64_t)out.size() && k < cap; ++k) {
    pairs[2 * k] = out[k].first;
    pairs[2 * k + 1] = out[k].second;
  }
  return (int64_t)out.size();
}

// Advance kinematic body poses by one step: t += dt*nu, R = Exp(dt*[omega]x) R.
void ggo_advance_bodies(int32_t nb, Body* bodies, double dt) {
  for (int b = 0; b < nb; ++b) {
    Body& B = bodies[b];
    for (int a = 0; a < 3; ++a) B.t[a] += dt * B.nu[a];
    double w[3] = {B.omega[0] * dt, B.omega[1] * dt, B.omega[2] * dt};
    double th = std::sqrt(dot3(w, w));
    if (th == 0) continue;
    double k[3] = {w[0] / th, w[1] / th, w[2] / th};
    double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
    double K2[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int m = 0; m < 3; ++m) s += K[3 * r + m] * K[3 * m + c];
        K2[3 * r + c] = s;
      }
    double E[9];
    for (int q = 0; q < 9; ++q) E[q] = (q % 4 == 0 ? 1.0 : 0.0) + std::sin(th) * K[q] + (1 - std::cos(th)) * K2[q];
    double Rn[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int m = 0; m < 3; ++m) s += E[3 * r + m] * B.R[3 * m + c];
        Rn[3 * r + c] = s;
      }
    std::memcpy(B.R, Rn, sizeof(Rn));
  }
}

// One timestep.  State x, v (n x 3, FP64) is updated in place; contact
// decisions use the binary32 rounding of x and of the body poses.
// Outputs (each may be NULL):
//   pairs      [cap x 2]  canonical list: pp (i<j) by (i,j), then pb (i, body) by (i, body)
//   impulses   [cap x 3]  world impulse on the first member, R_c * lam_c
//   psi        [cap]      signed gap of each contact
//   normals    [cap x 3]  unit contact normal e1 (from the second member to the first)
//   dv         [n x 3]    w - w0 after the last iteration (velocity change by impulses)
//   lam_hist   [n_hist x cap x 3] world impulses after iterations 1..n_hist (n_hist <= n_iters)
//   stats      [4]        candidates, pp count, pb count, 0
// Returns the number of contacts (which may exceed cap; arrays then hold the
// first cap entries and the state is still advanced).
int64_t ggo_step(const Params* P, int64_t n, double* x, double* v, const float* radius,
                 const int32_t* env, int32_t nb, Body* bodies, int32_t advance_bodies, int64_t cap,
                 int32_t* pairs, double* impulses, double* psi_out, double* normals, double* dv, int32_t n_hist,
                 double* lam_hist, int64_t* stats, const int32_t* fixed_pairs, int64_t fixed_pp,
                 int64_t fixed_pb) {
  // ---- detection on binary32 positions, or a given contact list (to
  // differentiate with the contact set held fixed)
  std::vector<float> xf(3 * n);
  for (int64_t q = 0; q < 3 * n; ++q) xf[q] = (float)x[q];
  std::vector<std::pair<int32_t, int32_t>> pp, pb;
  int64_t cand = 0;
  if (fixed_pairs) {
    for (int64_t c = 0; c < fixed_pp; ++c) pp.emplace_back(fixed_pairs[2 * c], fixed_pairs[2 * c + 1]);
    for (int64_t c = fixed_pp; c < fixed_pp + fixed_pb; ++c) pb.emplace_back(fixed_pairs[2 * c], fixed_pairs[2 * c + 1]);
  } else {
    pp_contacts_grid(n, xf.data(), radius, env, P->inv_c, P->n_h, pp, &cand);
    pb_contacts(n, xf.data(), radius, env, nb, bodies, pb);
  }
  const int64_t C = (int64_t)(pp.size() + pb.size());
  if (stats) {
    stats[0] = cand;
    stats[1] = (int64_t)pp.size();
    stats[2] = (int64_t)pb.size();
    stats[3] = 0;
  }

  // ---- contact geometry (FP64)
  std::vector<Contact> cs(C);
  std::vector<int32_t> count(n, 0);
  for (int64_t c = 0; c < (int64_t)pp.size(); ++c) {
    Contact& K = cs[c];
    K.i = pp[c].first;
    K.j = pp[c].second;
    double d[3];
    for (int a = 0; a < 3; ++a) d[a] = x[3 * K.i + a] - x[3 * K.j + a];
    double L = std::sqrt(dot3(d, d));
    double rs = (double)radius[K.i] + (double)radius[K.j];
    if (L > 0) {
      for (int a = 0; a < 3; ++a) K.n[a] = d[a] / L;
    } else {
      K.n[0] = 0; K.n[1] = 0; K.n[2] = 1;
    }
    K.psi = L - rs;
    K.vel[0] = K.vel[1] = K.vel[2] = 0;
    count[K.i]++;
    count[K.j]++;
  }
  for (int64_t q = 0; q < (int64_t)pb.size(); ++q) {
    Contact& K = cs[pp.size() + q];
    K.i = pb[q].first;
    int b = pb[q].second;
    K.j = -1 - b;
    const Body& B = bodies[b];
    double d[3], p[3], g[3];
    for (int a = 0; a < 3; ++a) d[a] = x[3 * K.i + a] - B.t[a];
    for (int c = 0; c < 3; ++c) p[c] = B.R[0 * 3 + c] * d[0] + B.R[1 * 3 + c] * d[1] + B.R[2 * 3 + c] * d[2];
    double f = sdf_f64(B, p, g);
    for (int a = 0; a < 3; ++a) K.n[a] = B.R[3 * a + 0] * g[0] + B.R[3 * a + 1] * g[1] + B.R[3 * a + 2] * g[2];
    double nn = std::sqrt(dot3(K.n, K.n));
    for (int a = 0; a < 3; ++a) K.n[a] /= nn;
    K.psi = f - (double)radius[K.i];
    double pc[3], arm[3];
    for (int a = 0; a < 3; ++a) {
      pc[a] = x[3 * K.i + a] - f * K.n[a];
      arm[a] = pc[a] - B.t[a];
    }
    K.vel[0] = B.nu[0] + B.omega[1] * arm[2] - B.omega[2] * arm[1];
    K.vel[1] = B.nu[1] + B.omega[2] * arm[0] - B.omega[0] * arm[2];
    K.vel[2] = B.nu[2] + B.omega[0] * arm[1] - B.omega[1] * arm[0];
    count[K.i]++;
  }
  for (auto& K : cs) tangent_basis(K.n, K.t1, K.t2);

  // ---- masses and split masses
  std::vector<double> mass(n), mt(C);
  for (int64_t i = 0; i < n; ++i) mass[i] = particle_mass((double)radius[i], P->density);
  for (int64_t c = 0; c < C; ++c) {
    const Contact& K = cs[c];
    double ni = P->mass_split ? (double)count[K.i] : 1.0;
    if (K.j >= 0) {
      double nj = P->mass_split ? (double)count[K.j] : 1.0;
      mt[c] = 1.0 / (ni / mass[K.i] + nj / mass[K.j]);
    } else {
      mt[c] = mass[K.i] / ni;
    }
  }

  // ---- projected Jacobi (Alg. 1): every contact reads iterate l-1
  std::vector<double> w0(3 * n), w(3 * n), lam(3 * C, 0.0), lam_new(3 * C);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) w0[3 * i + a] = v[3 * i + a] + P->dt * P->g[a];
  w = w0;
  // incident contacts of each particle, in contact-list order
  std::vector<int64_t> start(n + 1, 0), inc;
  for (int64_t c = 0; c < C; ++c) {
    start[cs[c].i + 1]++;
    if (cs[c].j >= 0) start[cs[c].j + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
  inc.resize(start[n]);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t c = 0; c < C; ++c) {
      inc[fill[cs[c].i]++] = c;
      if (cs[c].j >= 0) inc[fill[cs[c].j]++] = c;
    }
  }
  const double mu = P->mu, om = P->relax;
  for (int32_t l = 1; l <= P->n_iters; ++l) {
#pragma omp parallel for schedule(static) if (C > kOmpMin)
    for (int64_t c = 0; c < C; ++c) {
      const Contact& K = cs[c];
      double u[3];
      for (int a = 0; a < 3; ++a)
        u[a] = w[3 * K.i + a] - (K.j >= 0 ? w[3 * K.j + a] : K.vel[a]);
      const double* L = &lam[3 * c];
      double ln = dot3(K.n, L), l1 = dot3(K.t1, L), l2 = dot3(K.t2, L);
      double yn = ln - mt[c] * (dot3(K.n, u) + P->alpha * K.psi / P->dt);
      double y1 = l1 - mt[c] * dot3(K.t1, u);
      double y2 = l2 - mt[c] * dot3(K.t2, u);
      yn = yn > 0 ? yn : 0.0;
      double s = std::sqrt(y1 * y1 + y2 * y2);
      if (s > mu * yn) {
        double f = mu * yn / s;
        y1 *= f;
        y2 *= f;
      }
      for (int a = 0; a < 3; ++a) {
        double yw = yn * K.n[a] + y1 * K.t1[a] + y2 * K.t2[a];
        lam_new[3 * c + a] = (1.0 - om) * L[a] + om * yw;
      }
    }
    lam.swap(lam_new);
#pragma omp parallel for schedule(static) if (n > kOmpMin)
    for (int64_t i = 0; i < n; ++i) {
      double acc[3] = {0, 0, 0};
      for (int64_t q = start[i]; q < start[i + 1]; ++q) {
        int64_t c = inc[q];
        double sg = (cs[c].i == i) ? 1.0 : -1.0;
        for (int a = 0; a < 3; ++a) acc[a] += sg * lam[3 * c + a];
      }
      for (int a = 0; a < 3; ++a) w[3 * i + a] = w0[3 * i + a] + acc[a] / mass[i];
    }
    if (lam_hist && l <= n_hist)
      for (int64_t c = 0; c < C && c < cap; ++c)
        for (int a = 0; a < 3; ++a) lam_hist[((int64_t)(l - 1) * cap + c) * 3 + a] = lam[3 * c + a];
  }

  // ---- outputs
  for (int64_t c = 0; c < C && c < cap; ++c) {
    if (pairs) {
      pairs[2 * c] = cs[c].i;
      pairs[2 * c + 1] = cs[c].j >= 0 ? cs[c].j : -1 - cs[c].j;
    }
    if (impulses)
      for (int a = 0; a < 3; ++a) impulses[3 * c + a] = lam[3 * c + a];
    if (psi_out) psi_out[c] = cs[c].psi;
    if (normals)
      for (int a = 0; a < 3; ++a) normals[3 * c + a] = cs[c].n[a];
  }
  if (dv)
    for (int64_t q = 0; q < 3 * n; ++q) dv[q] = w[q] - w0[q];

  // ---- symplectic Euler (Eqs. (4)-(5)): velocity first, then position; the
  // tower benchmark's cyclic boundary moves a particle that falls below the
  // bottom cap up by the tower height, velocity unchanged
  for (int64_t q = 0; q < 3 * n; ++q) {
    v[q] = w[q];
    x[q] = x[q] + P->dt * v[q];
    if (q % 3 == 2 && P->cyc_hi > P->cyc_lo && x[q] < P->cyc_lo) x[q] += P->cyc_hi - P->cyc_lo;
  }
  if (advance_bodies) ggo_advance_bodies(nb, bodies, P->dt);
  return C;
}

int32_t ggo_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int32_t ggo_sizeof_body() { return (int32_t)sizeof(Body); }
int32_t ggo_sizeof_params() { return (int32_t)sizeof(Params); }

}  // extern "C"

namespace {

// ------------------------------------------------------- forward-mode JVP
// The same step carried out on dual numbers (value, tangent): the tangent part
// is the exact directional derivative of the step along the input tangents,
// with every discrete decision (the contact set, the normal clamp max(y_n, 0)
// with derivative [y_n > 0], the strict test for scaling the tangential part,
// the SDF branch) taken on the value part.  The value part repeats the plain
// step's operations in the same order, so it equals ggo_step's result bit for
// bit (the tests check this).  Tangents of the body twists are inputs of each
// step; tangents of the poses are carried along with the poses.

struct Dual {
  double v, d;
};
inline Dual mkd(double v) { return {v, 0.0}; }
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual operator/(double a, Dual b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
inline Dual dsqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, s > 0 ? a.d / (2.0 * s) : 0.0};
}
inline Dual dsin(Dual a) { return {std::sin(a.v), std::cos(a.v) * a.d}; }
inline Dual dcos(Dual a) { return {std::cos(a.v), -std::sin(a.v) * a.d}; }
inline Dual dabs(Dual a) { return a.v < 0 ? -a : a; }
inline Dual dot3d(const Dual a[3], const Dual b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

struct BodyTan {       // tangents of a body's pose and twist (mirrored by the Python wrapper)
  double R[9], t[3], nu[3], omega[3];
};

struct DBody {
  int32_t shape;
  const float* params;
  Dual R[9], t[3], nu[3], om[3];
  const Body* body;   // grid data (values, knots, origin, inv_spacing)
};

// grid_f64 on duals (the cell chosen on values).
Dual grid_dual(const Body& b, const Dual p[3], Dual grad[3]) {
  int i[3];
  Dual t[3];
  for (int a = 0; a < 3; ++a) {
    Dual u = (p[a] - (double)b.go[a]) * (double)b.gih;
    if (u.v < 0) u = mkd(0.0);
    if (u.v > (double)(b.gn[a] - 1)) u = mkd((double)(b.gn[a] - 1));
    int k = std::min((int)std::floor(u.v), b.gn[a] - 2);
    i[a] = k;
    t[a] = u - (double)k;
  }
  auto V = [&](int a, int c, int e) -> double {
    return b.gv[((int64_t)(i[2] + e) * b.gn[1] + (i[1] + c)) * b.gn[0] + (i[0] + a)];
  };
  Dual c00 = V(0, 0, 0) + t[0] * (V(1, 0, 0) - V(0, 0, 0));
  Dual c10 = V(0, 1, 0) + t[0] * (V(1, 1, 0) - V(0, 1, 0));
  Dual c01 = V(0, 0, 1) + t[0] * (V(1, 0, 1) - V(0, 0, 1));
  Dual c11 = V(0, 1, 1) + t[0] * (V(1, 1, 1) - V(0, 1, 1));
  Dual c0 = c00 + t[1] * (c10 - c00);
  Dual c1 = c01 + t[1] * (c11 - c01);
  Dual dx0 = (V(1, 0, 0) - V(0, 0, 0)) + t[1] * ((V(1, 1, 0) - V(0, 1, 0)) - (V(1, 0, 0) - V(0, 0, 0)));
  Dual dx1 = (V(1, 0, 1) - V(0, 0, 1)) + t[1] * ((V(1, 1, 1) - V(0, 1, 1)) - (V(1, 0, 1) - V(0, 0, 1)));
  double ih = (double)b.gih;
  grad[0] = (dx0 + t[2] * (dx1 - dx0)) * ih;
  grad[1] = ((c10 - c00) + t[2] * ((c11 - c01) - (c10 - c00))) * ih;
  grad[2] = (c1 - c0) * ih;
  if (!(grad[0].v * grad[0].v + grad[1].v * grad[1].v + grad[2].v * grad[2].v > 0)) {
    grad[0] = mkd(1.0); grad[1] = mkd(0.0); grad[2] = mkd(0.0);
  }
  return c0 + t[2] * (c1 - c0);
}

// sdf_f64 on duals (same branches, decided on values).
Dual sdf_dual(const DBody& b, const Dual p[3], Dual grad[3]) {
  const Dual zero = mkd(0.0), one = mkd(1.0);
  if (b.shape == PLANE) {
    grad[0] = zero; grad[1] = zero; grad[2] = one;
    return p[2];
  }
  if (b.shape == GRID) return grid_dual(*b.body, p, grad);
  if (b.shape == BOX) {
    Dual q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = dabs(p[c]) - (double)b.params[c];
      m[c] = q[c].v > 0 ? q[c] : zero;
      if (q[c].v > 0) outside = true;
    }
    if (outside) {
      Dual L = dsqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int c = 0; c < 3; ++c) grad[c] = (p[c].v < 0 ? -1.0 : 1.0) * m[c] / L;
      return L;
    }
    int a = 0;
    for (int c = 1; c < 3; ++c)
      if (q[c].v > q[a].v) a = c;
    grad[0] = grad[1] = grad[2] = zero;
    grad[a] = mkd(p[a].v < 0 ? -1.0 : 1.0);
    return q[a];
  }
  double h = b.params[1];
  Dual cz = p[2].v < -h ? mkd(-h) : (p[2].v > h ? mkd(h) : p[2]);
  Dual e[3] = {p[0], p[1], p[2] - cz};
  Dual L = dsqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (L.v > 0) {
    for (int c = 0; c < 3; ++c) grad[c] = e[c] / L;
  } else {
    grad[0] = one; grad[1] = zero; grad[2] = zero;
  }
  return L - (double)b.params[0];
}

void tangent_basis_dual(const Dual n[3], Dual t1[3], Dual t2[3]) {
  double sgn = n[2].v >= 0 ? 1.0 : -1.0;
  Dual a = -1.0 / (sgn + n[2]);
  Dual b = n[0] * n[1] * a;
  t1[0] = 1.0 + sgn * n[0] * n[0] * a; t1[1] = sgn * b; t1[2] = -sgn * n[0];
  t2[0] = b; t2[1] = sgn + n[1] * n[1] * a; t2[2] = -n[1];
}

struct DContact {
  int32_t i, j;
  Dual n[3], t1[3], t2[3];
  Dual psi;
  Dual vel[3];
};

// Rodrigues update of one body on duals (ggo_advance_bodies): t += dt nu,
// R = Exp(dt [omega]x) R.  At a zero rotation the exponential is I + [w]x to
// first order, which carries the tangent of w exactly.
void advance_body_dual(DBody& B, double dt) {
  for (int a = 0; a < 3; ++a) B.t[a] = B.t[a] + dt * B.nu[a];
  Dual w[3] = {B.om[0] * dt, B.om[1] * dt, B.om[2] * dt};
  Dual th = dsqrt(dot3d(w, w));
  Dual E[9];
  if (th.v == 0) {
    const Dual zero = mkd(0.0);
    Dual K[9] = {zero, -w[2], w[1], w[2], zero, -w[0], -w[1], w[0], zero};
    for (int q = 0; q < 9; ++q) E[q] = (q % 4 == 0 ? 1.0 : 0.0) + K[q];
  } else {
    Dual k[3] = {w[0] / th, w[1] / th, w[2] / th};
    const Dual zero = mkd(0.0);
    Dual K[9] = {zero, -k[2], k[1], k[2], zero, -k[0], -k[1], k[0], zero};
    Dual K2[9];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        Dual sum = mkd(0.0);
        for (int m = 0; m < 3; ++m) sum = sum + K[3 * r + m] * K[3 * m + c];
        K2[3 * r + c] = sum;
      }
    for (int q = 0; q < 9; ++q) E[q] = (q % 4 == 0 ? 1.0 : 0.0) + dsin(th) * K[q] + (1.0 - dcos(th)) * K2[q];
  }
  Dual Rn[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      Dual sum = mkd(0.0);
      for (int m = 0; m < 3; ++m) sum = sum + E[3 * r + m] * B.R[3 * m + c];
      Rn[3 * r + c] = sum;
    }
  for (int q = 0; q < 9; ++q) B.R[q] = Rn[q];
}

}  // namespace

extern "C" {

// One timestep with tangents: x, v (values) and dx, dv (tangents) are updated
// in place, as are the bodies and their tangents dbodies (the caller sets the
// twist tangents of this step in dbodies[b].nu / .omega).  The contact list is
// detected on the values, or given (fixed_*), as in ggo_step.  stats as there.
int64_t ggo_step_jvp(const Params* P, int64_t n, double* x, double* v, double* dx, double* dv,
                     const float* radius, const int32_t* env, int32_t nb, Body* bodies, BodyTan* dbodies,
                     int32_t advance_bodies, const int32_t* fixed_pairs, int64_t fixed_pp, int64_t fixed_pb,
                     int64_t* stats) {
  std::vector<float> xf(3 * n);
  for (int64_t q = 0; q < 3 * n; ++q) xf[q] = (float)x[q];
  std::vector<std::pair<int32_t, int32_t>> pp, pb;
  int64_t cand = 0;
  if (fixed_pairs) {
    for (int64_t c = 0; c < fixed_pp; ++c) pp.emplace_back(fixed_pairs[2 * c], fixed_pairs[2 * c + 1]);
    for (int64_t c = fixed_pp; c < fixed_pp + fixed_pb; ++c) pb.emplace_back(fixed_pairs[2 * c], fixed_pairs[2 * c + 1]);
  } else {
    pp_contacts_grid(n, xf.data(), radius, env, P->inv_c, P->n_h, pp, &cand);
    pb_contacts(n, xf.data(), radius, env, nb, bodies, pb);
  }
  const int64_t C = (int64_t)(pp.size() + pb.size());
  if (stats) {
    stats[0] = cand;
    stats[1] = (int64_t)pp.size();
    stats[2] = (int64_t)pb.size();
    stats[3] = 0;
  }
  std::vector<Dual> X(3 * n), V(3 * n);
  for (int64_t q = 0; q < 3 * n; ++q) {
    X[q] = {x[q], dx[q]};
    V[q] = {v[q], dv[q]};
  }
  std::vector<DBody> DB(nb);
  for (int b = 0; b < nb; ++b) {
    DB[b].shape = bodies[b].shape;
    DB[b].params = bodies[b].params;
    DB[b].body = &bodies[b];
    for (int q = 0; q < 9; ++q) DB[b].R[q] = {bodies[b].R[q], dbodies[b].R[q]};
    for (int q = 0; q < 3; ++q) {
      DB[b].t[q] = {bodies[b].t[q], dbodies[b].t[q]};
      DB[b].nu[q] = {bodies[b].nu[q], dbodies[b].nu[q]};
      DB[b].om[q] = {bodies[b].omega[q], dbodies[b].omega[q]};
    }
  }

  // ---- contact geometry
  std::vector<DContact> cs(C);
  std::vector<int32_t> count(n, 0);
  for (int64_t c = 0; c < (int64_t)pp.size(); ++c) {
    DContact& K = cs[c];
    K.i = pp[c].first;
    K.j = pp[c].second;
    Dual d[3];
    for (int a = 0; a < 3; ++a) d[a] = X[3 * K.i + a] - X[3 * K.j + a];
    Dual L = dsqrt(dot3d(d, d));
    double rs = (double)radius[K.i] + (double)radius[K.j];
    if (L.v > 0) {
      for (int a = 0; a < 3; ++a) K.n[a] = d[a] / L;
    } else {
      K.n[0] = mkd(0); K.n[1] = mkd(0); K.n[2] = mkd(1);
    }
    K.psi = L - rs;
    K.vel[0] = K.vel[1] = K.vel[2] = mkd(0);
    count[K.i]++;
    count[K.j]++;
  }
  for (int64_t q = 0; q < (int64_t)pb.size(); ++q) {
    DContact& K = cs[pp.size() + q];
    K.i = pb[q].first;
    int b = pb[q].second;
    K.j = -1 - b;
    const DBody& B = DB[b];
    Dual d[3], p[3], g[3];
    for (int a = 0; a < 3; ++a) d[a] = X[3 * K.i + a] - B.t[a];
    for (int c = 0; c < 3; ++c) p[c] = B.R[0 * 3 + c] * d[0] + B.R[1 * 3 + c] * d[1] + B.R[2 * 3 + c] * d[2];
    Dual f = sdf_dual(B, p, g);
    for (int a = 0; a < 3; ++a) K.n[a] = B.R[3 * a + 0] * g[0] + B.R[3 * a + 1] * g[1] + B.R[3 * a + 2] * g[2];
    Dual nn = dsqrt(dot3d(K.n, K.n));
    for (int a = 0; a < 3; ++a) K.n[a] = K.n[a] / nn;
    K.psi = f - (double)radius[K.i];
    Dual pc[3], arm[3];
    for (int a = 0; a < 3; ++a) {
      pc[a] = X[3 * K.i + a] - f * K.n[a];
      arm[a] = pc[a] - B.t[a];
    }
    K.vel[0] = B.nu[0] + B.om[1] * arm[2] - B.om[2] * arm[1];
    K.vel[1] = B.nu[1] + B.om[2] * arm[0] - B.om[0] * arm[2];
    K.vel[2] = B.nu[2] + B.om[0] * arm[1] - B.om[1] * arm[0];
    count[K.i]++;
  }
  for (auto& K : cs) tangent_basis_dual(K.n, K.t1, K.t2);

  // ---- masses (no tangents: radii are fixed)
  std::vector<double> mass(n), mt(C);
  for (int64_t i = 0; i < n; ++i) mass[i] = particle_mass((double)radius[i], P->density);
  for (int64_t c = 0; c < C; ++c) {
    const DContact& K = cs[c];
    double ni = P->mass_split ? (double)count[K.i] : 1.0;
    if (K.j >= 0) {
      double nj = P->mass_split ? (double)count[K.j] : 1.0;
      mt[c] = 1.0 / (ni / mass[K.i] + nj / mass[K.j]);
    } else {
      mt[c] = mass[K.i] / ni;
    }
  }

  // ---- projected Jacobi on duals
  std::vector<Dual> w0(3 * n), w(3 * n), lam(3 * C, mkd(0.0)), lam_new(3 * C);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) w0[3 * i + a] = V[3 * i + a] + P->dt * P->g[a];
  w = w0;
  std::vector<int64_t> start(n + 1, 0), inc;
  for (int64_t c = 0; c < C; ++c) {
    start[cs[c].i + 1]++;
    if (cs[c].j >= 0) start[cs[c].j + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
  inc.resize(start[n]);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t c = 0; c < C; ++c) {
      inc[fill[cs[c].i]++] = c;
      if (cs[c].j >= 0) inc[fill[cs[c].j]++] = c;
    }
  }
  const double mu = P->mu, om = P->relax;
  for (int32_t l = 1; l <= P->n_iters; ++l) {
#pragma omp parallel for schedule(static) if (C > kOmpMin)
    for (int64_t c = 0; c < C; ++c) {
      const DContact& K = cs[c];
      Dual u[3];
      for (int a = 0; a < 3; ++a) u[a] = w[3 * K.i + a] - (K.j >= 0 ? w[3 * K.j + a] : K.vel[a]);
      const Dual* L = &lam[3 * c];
      Dual ln = dot3d(K.n, L), l1 = dot3d(K.t1, L), l2 = dot3d(K.t2, L);
      Dual yn = ln - mt[c] * (dot3d(K.n, u) + P->alpha * K.psi / P->dt);
      Dual y1 = l1 - mt[c] * dot3d(K.t1, u);
      Dual y2 = l2 - mt[c] * dot3d(K.t2, u);
      yn = yn.v > 0 ? yn : mkd(0.0);
      Dual s = dsqrt(y1 * y1 + y2 * y2);
      if (s.v > mu * yn.v) {
        Dual f = mu * yn / s;
        y1 = y1 * f;
        y2 = y2 * f;
      }
      if (!(mu * yn.v > 0)) {
        // A friction disk of radius zero (a non-positive normal part, or no
        // friction) maps the tangential part to zero, and so it does on a
        // neighbourhood: its tangent is zero.  The tangential test alone
        // would keep the tangents of y_t where y_t is exactly zero (0 > 0 is
        // false), which is not the derivative of the projection.
        y1.d = 0.0;
        y2.d = 0.0;
      }
      for (int a = 0; a < 3; ++a) {
        Dual yw = yn * K.n[a] + y1 * K.t1[a] + y2 * K.t2[a];
        lam_new[3 * c + a] = (1.0 - om) * L[a] + om * yw;
      }
    }
    lam.swap(lam_new);
#pragma omp parallel for schedule(static) if (n > kOmpMin)
    for (int64_t i = 0; i < n; ++i) {
      Dual acc[3] = {mkd(0), mkd(0), mkd(0)};
      for (int64_t q = start[i]; q < start[i + 1]; ++q) {
        int64_t c = inc[q];
        double sg = (cs[c].i == i) ? 1.0 : -1.0;
        for (int a = 0; a < 3; ++a) acc[a] = acc[a] + sg * lam[3 * c + a];
      }
      for (int a = 0; a < 3; ++a) w[3 * i + a] = w0[3 * i + a] + acc[a] / mass[i];
    }
  }

  // ---- symplectic Euler
  for (int64_t q = 0; q < 3 * n; ++q) {
    V[q] = w[q];
    X[q] = X[q] + P->dt * V[q];
    if (q % 3 == 2 && P->cyc_hi > P->cyc_lo && X[q].v < P->cyc_lo) X[q] = X[q] + (P->cyc_hi - P->cyc_lo);
    x[q] = X[q].v;
    dx[q] = X[q].d;
    v[q] = V[q].v;
    dv[q] = V[q].d;
  }
  if (advance_bodies)
    for (int b = 0; b < nb; ++b) advance_body_dual(DB[b], P->dt);
  for (int b = 0; b < nb; ++b) {
    for (int q = 0; q < 9; ++q) {
      bodies[b].R[q] = DB[b].R[q].v;
      dbodies[b].R[q] = DB[b].R[q].d;
    }
    for (int q = 0; q < 3; ++q) {
      bodies[b].t[q] = DB[b].t[q].v;
      dbodies[b].t[q] = DB[b].t[q].d;
    }
  }
  return C;
}

int32_t ggo_sizeof_body_tan() { return (int32_t)sizeof(BodyTan); }

}  // extern "C"

// ======================================================= observations
// The Gym-style environment of Sec. III-A ("Bulldozing") observes the scene
// through two depth cameras computed on the simulating device -- a
// perspective camera riding on the tool and an orthographic camera looking
// down on the whole bed -- and rewards material inside a goal box.  The paper
// gives no camera model; the readings taken here:
//   - a camera has a pose [R | t] (camera -> world) and looks along its +z
//     axis; pixel (u, v) of a W x H image has the centre coordinates
//     g_u = (u + 1/2) * fl32(2/W) - 1 and g_v likewise, in binary32;
//   - orthographic: the ray of pixel (u, v) starts at (p0 g_u, p1 g_v, 0) and
//     runs along (0, 0, 1); perspective: it starts at the camera origin and
//     runs along (p0 g_u, p1 g_v, 1) (p0, p1 = tangents of the half angles);
//   - depth = camera-frame z of the first surface the ray meets (the ray
//     parameter along those directions), at most `far` (= p2); `far` when the
//     ray meets nothing;
//   - surfaces drawn: the particles of the camera's environment (spheres) and
//     its plane bodies (the solid half space below the body-frame xy plane);
//     tool bodies are not drawn;
//   - whether a ray meets a sphere is decided in binary32 with a fixed
//     operation order and no fused multiply-add (the camera-frame centre
//     c = R^T (x - t) summed as the SDF transform is; orthographic:
//     c_z > 0 and (o_x - c_x)^2 + (o_y - c_y)^2 <= r^2; perspective: c_z > 0,
//     E = |c|^2 - r^2 > 0 (the camera is outside the sphere), D = d.c > 0 and
//     |d|^2 E <= D^2); the depth itself is FP64 from those binary32 values;
//   - a plane is met when the ray runs into its solid side (n.d < 0) at a
//     non-negative parameter.
struct Camera {        // mirrored by the Python wrapper (ctypes)
  int32_t env, kind;   // kind 0: orthographic, 1: perspective
  int32_t width, height;
  float pose[12];      // row-major [R | t], camera -> world
  float params[4];     // p0, p1 (see above), far, unused
};

float pixel_centre(int idx, int size) {
  const float s = (float)(2.0 / size);
  float a = (float)idx + 0.5f;
  float b = a * s;
  return b - 1.0f;
}

// Depth of one pixel: every particle of the environment and every plane body
// of it, smallest parameter wins.
double pixel_depth(const Camera& C, int u, int v, const float* x, const float* r, int64_t i0, int64_t i1,
                   int32_t nb, const Body* bodies) {
  const float gu = pixel_centre(u, C.width), gv = pixel_centre(v, C.height);
  const float a = C.params[0] * gu, b = C.params[1] * gv;
  const bool ortho = C.kind == 0;
  const float Rc[9] = {C.pose[0], C.pose[1], C.pose[2], C.pose[4], C.pose[5],
                       C.pose[6], C.pose[8], C.pose[9], C.pose[10]};
  const float tc[3] = {C.pose[3], C.pose[7], C.pose[11]};
  double best = C.params[2];
  for (int64_t i = i0; i < i1; ++i) {
    // camera-frame centre, binary32
    float d0 = x[3 * i] - tc[0], d1 = x[3 * i + 1] - tc[1], d2 = x[3 * i + 2] - tc[2];
    float c[3];
    for (int k = 0; k < 3; ++k) {
      float s0 = Rc[0 * 3 + k] * d0;
      float s1 = Rc[1 * 3 + k] * d1;
      float s2 = Rc[2 * 3 + k] * d2;
      float s = s0 + s1;
      c[k] = s + s2;
    }
    if (!(c[2] > 0.0f)) continue;
    const float ri = r[i];
    const float r2 = ri * ri;
    double tau;
    if (ortho) {
      float ex = a - c[0], ey = b - c[1];
      float q0 = ex * ex;
      float q1 = ey * ey;
      float q = q0 + q1;
      if (!(q <= r2)) continue;
      const double ex64 = (double)a - c[0], ey64 = (double)b - c[1];
      const double h = (double)ri * ri - (ex64 * ex64 + ey64 * ey64);
      tau = (double)c[2] - std::sqrt(std::max(h, 0.0));
      tau = std::max(tau, 0.0);
    } else {
      float aa = a * a;
      float bb = b * b;
      float A = aa + bb;
      A = A + 1.0f;
      float c00 = c[0] * c[0];
      float c11 = c[1] * c[1];
      float c22 = c[2] * c[2];
      float B = c00 + c11;
      B = B + c22;
      float ac = a * c[0];
      float bc = b * c[1];
      float D = ac + bc;
      D = D + c[2];
      float E = B - r2;
      if (!(E > 0.0f) || !(D > 0.0f)) continue;
      float lhs = A * E;
      float rhs = D * D;
      if (!(lhs <= rhs)) continue;
      // |t d - c|^2 = r^2, nearer root, written without cancellation
      const double A6 = (double)a * a + (double)b * b + 1.0;
      const double B6 = (double)c[0] * c[0] + (double)c[1] * c[1] + (double)c[2] * c[2];
      const double D6 = (double)a * c[0] + (double)b * c[1] + (double)c[2];
      const double E6 = B6 - (double)ri * ri;
      const double disc = std::max(D6 * D6 - A6 * E6, 0.0);
      tau = E6 / (D6 + std::sqrt(disc));
    }
    best = std::min(best, tau);
  }
  // planes, in FP64
  double o[3] = {0, 0, 0}, d[3] = {0, 0, 1};
  if (ortho) {
    o[0] = a; o[1] = b;
  } else {
    d[0] = a; d[1] = b;
  }
  double ow[3], dw[3];
  for (int k = 0; k < 3; ++k) {
    ow[k] = tc[k] + ((double)Rc[3 * k] * o[0] + (double)Rc[3 * k + 1] * o[1] + (double)Rc[3 * k + 2] * o[2]);
    dw[k] = (double)Rc[3 * k] * d[0] + (double)Rc[3 * k + 1] * d[1] + (double)Rc[3 * k + 2] * d[2];
  }
  for (int q = 0; q < nb; ++q) {
    const Body& B = bodies[q];
    if (B.shape != PLANE || B.env != C.env) continue;
    const double nrm[3] = {B.R[2], B.R[5], B.R[8]};
    const double den = dot3(nrm, dw);
    if (!(den < 0)) continue;
    const double rel[3] = {B.t[0] - ow[0], B.t[1] - ow[1], B.t[2] - ow[2]};
    const double tau = dot3(nrm, rel) / den;
    if (tau >= 0) best = std::min(best, tau);
  }
  return best;
}

extern "C" {

int32_t ggo_sizeof_camera() { return (int32_t)sizeof(Camera); }

// Depth images of n_cams cameras, concatenated (camera k: height x width,
// row v, column u at v*width + u), rounded to binary32.  env_off: n_envs + 1
// particle offsets.  pixels: NULL for every pixel, else n_pix indices into the
// concatenated output; only those entries are written.
void ggo_render_depth(int64_t n, const float* x, const float* r, int32_t n_envs, const int64_t* env_off,
                      int32_t nb, const Body* bodies, int32_t n_cams, const Camera* cams, float* out,
                      int64_t n_pix, const int64_t* pixels) {
  std::vector<int64_t> base(n_cams + 1, 0);
  for (int k = 0; k < n_cams; ++k) base[k + 1] = base[k] + (int64_t)cams[k].width * cams[k].height;
  const int64_t total = pixels ? n_pix : base[n_cams];
#pragma omp parallel for schedule(dynamic, 16) if (total > kOmpMin)
  for (int64_t q = 0; q < total; ++q) {
    const int64_t p = pixels ? pixels[q] : q;
    const int k = (int)(std::upper_bound(base.begin(), base.end(), p) - base.begin()) - 1;
    const Camera& C = cams[k];
    const int64_t loc = p - base[k];
    const int u = (int)(loc % C.width), v = (int)(loc / C.width);
    const int e = C.env;
    const int64_t i0 = (e >= 0 && e < n_envs) ? env_off[e] : 0, i1 = (e >= 0 && e < n_envs) ? env_off[e + 1] : 0;
    out[p] = (float)pixel_depth(C, u, v, x, r, i0, i1, nb, bodies);
  }
  (void)n;
}

// Goal-box reward (Sec. III-A): per environment, 100/n_e for every particle in
// the closed box [lo, hi] (binary32 comparisons of the binary32 positions)
// and -d/n_e for every other, d = FP64 distance to the nearest point of the
// box.  boxes: n_envs x 6 (lo xyz, hi xyz).  reward: n_envs; inside: n_envs
// (may be NULL).  An empty environment has reward 0.
void ggo_goal_reward(int64_t n, const float* x, int32_t n_envs, const int64_t* env_off, const float* boxes,
                     double* reward, int64_t* inside) {
  for (int e = 0; e < n_envs; ++e) {
    const float* lo = boxes + 6 * e;
    const float* hi = lo + 3;
    int64_t cnt = 0;
    double dist = 0;
    for (int64_t i = env_off[e]; i < env_off[e + 1]; ++i) {
      const float* p = x + 3 * i;
      bool in = true;
      double s = 0;
      for (int k = 0; k < 3; ++k) {
        in = in && lo[k] <= p[k] && p[k] <= hi[k];
        const double q = std::min(std::max((double)p[k], (double)lo[k]), (double)hi[k]);
        s += ((double)p[k] - q) * ((double)p[k] - q);
      }
      if (in)
        ++cnt;
      else
        dist += std::sqrt(s);
    }
    const int64_t ne = env_off[e + 1] - env_off[e];
    reward[e] = ne > 0 ? (100.0 * (double)cnt - dist) / (double)ne : 0.0;
    if (inside) inside[e] = cnt;
  }
  (void)n;
}

}  // extern "C"
