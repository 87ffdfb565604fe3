// Device kernels of the granular contact step for gfx950 (CDNA4, wave64).
//
// Per timestep (arXiv 2306.01369, Sec. II):
//   k_morton_keys, k_rs_*, k_permute
//              (every few steps) re-sort the particle state along a Z-order
//              curve over the cells, a 64-bit LSD radix sort with wave64
//              ballot ranking; the order only affects memory locality
//   k_key      cell coordinates and spatial hash (Eq. (6)); bucket counters
//   k_scan_*   exclusive prefix sum of the bucket counters -> bucket_start
//   k_scatter  particles into hash-bucket order (stands in for Alg. 2's lists)
//   k_detect   27-cell query from LDS-staged cell tiles, sphere test, SDF body
//              tests (Sec. II-B, II-C, Eq. (7)); writes each particle's partners
//   k_pja      one projected-Jacobi sweep (Alg. 1) over all contacts, gathered
//              per particle; the last sweep also writes the new velocity
//              (k_pja_lanes: the same with 2 or 4 lanes per particle)
//   k_integrate  positions from the new velocities (Eq. (5))
//
// Precision.  Every state-carrying kernel is a template over the real type R:
// float (the production build) or double (a build for gradient and parity
// checks against an FP64 reference).  The discrete decisions (cell index, the
// sphere and SDF contact predicates) are binary32 in both, on the state rounded
// to binary32, so both builds take the same decisions from the same state.
//
// Layout.  Particle state is structure-of-arrays float4: x = (x, y, z, r),
// v = (vx, vy, vz, 1/m), w = (wx, wy, wz, s) with s = n_i/m_i (the split inverse
// mass), orig = the caller's index of each (internally reordered) particle,
// and 1/m alone for the sweeps.  Every contact is stored once per member ("half contacts") in an
// ELL table of K slots per particle, laid out slot-major within groups of 64
// particles: slot(i, k) = (i/64)*64K + 64k + i%64, so the k-th contact of the 64
// lanes of a wavefront is one contiguous 256-byte row.  Each half contact holds
// the partner (>= 0 particle, with a flag when this particle has the higher
// original index; < 0 body -1-b), the gap psi and the world-frame impulse on
// the member with the lower original index; both halves compute it with
// identical arithmetic from identical inputs, so the two copies agree bit for
// bit and no atomics or second pass are needed.  Partners are listed in a
// canonical order (neighbour cell, then original index), so results are
// deterministic and independent of the internal order and launch shape.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstddef>

namespace ggk {

constexpr int kBlock = 256;
constexpr int kRsBits = 8;
constexpr int kDetBlock = 128;  // default detection workgroup (and work item) size
constexpr int kScanTile = 1024;  // elements per block of the bucket scan
constexpr int kQ = 100;
constexpr int kQueueStride = 32;  // int32 slots between two work-queue counters

struct DevBody {  // one body at one step; 312 bytes
  int32_t shape, env;
  float params[4];
  float R[9];  // world <- body, row major
  float t[3];
  float nu[3];
  float om[3];
  double Rd[9], td[3], nud[3], omd[3];  // the same pose and twist in double (FP64 build geometry)
  const float* gv;                      // grid bodies: knot values, x fastest
  int32_t gn[3];                        // knots per axis
  float go[3];                          // body-frame position of knot (0, 0, 0)
  float gih;                            // 1 / knot spacing
  int32_t cull;                         // 1: particles outside [lo, hi] cannot touch the body
  float lo[3], hi[3];                   // world box holding every point within r_max of the body
  int32_t pad2;
};

// Four-vectors of the real type R.
template <typename R> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename R> using V4 = typename Vec4<R>::type;

template <typename R>
__device__ __forceinline__ V4<R> mk4(R a, R b, R c, R d) {
  V4<R> q;
  q.x = a; q.y = b; q.z = c; q.w = d;
  return q;
}

// The state rounded to binary32 (identity for the binary32 build).
__device__ __forceinline__ float4 f32of(const float4 p) { return p; }
__device__ __forceinline__ float4 f32of(const double4 p) {
  return make_float4((float)p.x, (float)p.y, (float)p.z, (float)p.w);
}

// Body pose and twist in the precision of the geometry: binary32 fields for the
// binary32 build, double fields for the double build.
template <typename R> struct PoseOf;
template <> struct PoseOf<float> {
  static __device__ __forceinline__ const float* R(const DevBody& B) { return B.R; }
  static __device__ __forceinline__ const float* t(const DevBody& B) { return B.t; }
  static __device__ __forceinline__ const float* nu(const DevBody& B) { return B.nu; }
  static __device__ __forceinline__ const float* om(const DevBody& B) { return B.om; }
};
template <> struct PoseOf<double> {
  static __device__ __forceinline__ const double* R(const DevBody& B) { return B.Rd; }
  static __device__ __forceinline__ const double* t(const DevBody& B) { return B.td; }
  static __device__ __forceinline__ const double* nu(const DevBody& B) { return B.nud; }
  static __device__ __forceinline__ const double* om(const DevBody& B) { return B.omd; }
};

struct Ctl {                    // device control block, one per simulation
  int32_t err;                  // first failure of the current call (gg_status), 0 = none
  int32_t fail_step;            // step index of that failure
  int32_t steps_done;           // steps completed in the current call
  int32_t max_cnt;              // largest contact count (last detection)
  unsigned long long n_pp;      // pair contacts (last detection)
  unsigned long long n_pb;      // body contacts (last detection)
  unsigned long long cand;      // ordered candidate pairs (last detection)
  unsigned long long summed;    // contacts summed over the steps of the current call
  int32_t fallback;             // detection work items that took the per-particle path (last detection)
  int32_t items;                // detection work items (set when they are built)
  int32_t pad_[18];
  // detection work queues, one per XCD, each on a 128-byte line of its own
  // (zeroed by the key kernels): next_item[q * kQueueStride]
  int32_t next_item[8 * kQueueStride];
};
static_assert(offsetof(Ctl, next_item) == 128, "work-queue counters start a cache line");

// Counts of one detection workgroup, stored once when it ends and summed by
// detect_stats_block (workgroup 0 of the step's k_integrate, or k_detect_stats
// after the fused step): device-scope atomics from every workgroup on the control
// block cost more time than the rest of the statistics by far (they queue on
// one address, and loads and stores of the workgroups still running wait
// behind them).
struct DetPart {
  unsigned long long n_pp, n_pb, cand;
  int32_t max_cnt;
  int32_t fb_ran;  // (fallback items << 1) | 1; 0: the workgroup stopped at an earlier failure
};

struct EnvTables {   // per-environment tables (batched form)
  const int32_t* env_of;       // particle -> env (nullptr: one env)
  const int32_t* nh;           // Eq. (6) buckets per env (the reported cell index)
  const int32_t* boff;         // Eq. (6) bucket offset per env
  const int32_t* tblk;         // internal table: blocks of 64 buckets per env
  const int32_t* toff;         // internal table: first bucket of env
  const int32_t* body_lo;      // first body of env (bodies sorted by env)
  const int32_t* body_hi;      // one past last body of env
};

// Blocks are handed to the 8 XCDs round robin; remap so each XCD works on a
// contiguous range of particles and keeps its neighbours in its own L2.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int per = nb >> 3, rem = nb & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * per + min(xcd, rem) + idx;
}

__device__ __forceinline__ int ell_slot(int i, int k, int K) {
  return (i >> 6) * (K << 6) + (k << 6) + (i & 63);
}

// ------------------------------------------------------------------ Eq. (6)
// round(x / c) as rne(fl32(x * inv_c)); ok = false when out of the hashable range.
__device__ __forceinline__ int cell_coord(float x, float inv_c, bool& ok) {
#pragma clang fp contract(off)
  float s = x * inv_c;
  float r = __builtin_rintf(s);
  ok = ok && (fabsf(r) < 1073741824.0f);  // |kappa| < 2^30; false for NaN too
  return ok ? (int)r : 0;
}

// Bucket of cell (k0, k1, k2) in a table of nh buckets: XOR of p_a*(k_a - q),
// floored modulo nh.  64-bit products; for a power-of-two nh the low bits of
// 32-bit wrap-around products are the same bits.
__device__ __forceinline__ int hash_cell(int k0, int k1, int k2, int nh) {
  if ((nh & (nh - 1)) == 0) {
    uint32_t a = (uint32_t)(k0 - kQ) * 73856093u;
    uint32_t b = (uint32_t)(k1 - kQ) * 19349663u;
    uint32_t c = (uint32_t)(k2 - kQ) * 83492791u;
    return (int)((a ^ b ^ c) & (uint32_t)(nh - 1));
  }
  long long a = (long long)(k0 - kQ) * 73856093LL;
  long long b = (long long)(k1 - kQ) * 19349663LL;
  long long c = (long long)(k2 - kQ) * 83492791LL;
  long long v = (a ^ b ^ c) % (long long)nh;
  return (int)(v < 0 ? v + nh : v);
}

// --------------------------------------------------------- contact decisions
// ||xi - xj||^2 <= (ri + rj)^2 in binary32, each operation rounded as written.
__device__ __forceinline__ bool pair_touch(const float4 a, const float4 b) {
#pragma clang fp contract(off)
  float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
  float D = dx * dx + dy * dy;
  D = D + dz * dz;
  float s = a.w + b.w;
  float S = s * s;
  return D <= S;
}

// Body-frame point p = R^T (x - t), fixed summation order (binary32 pose and
// arithmetic for R = float, double for R = double).
template <typename R>
__device__ __forceinline__ void to_body(const DevBody& B, R x0, R x1, R x2, R p[3]) {
#pragma clang fp contract(off)
  const auto* Rm = PoseOf<R>::R(B);
  const auto* tv = PoseOf<R>::t(B);
  R d0 = x0 - tv[0], d1 = x1 - tv[1], d2 = x2 - tv[2];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    R a0 = Rm[0 * 3 + c] * d0;
    R a1 = Rm[1 * 3 + c] * d1;
    R a2 = Rm[2 * 3 + c] * d2;
    R s = a0 + a1;
    p[c] = s + a2;
  }
}

// ---------------------------------------------------------- grid SDF bodies
// Trilinear interpolation of SDF samples on a regular grid (Sec. II-C).  The
// binary32 form decides contact: u = (p - origin) * inv_spacing per axis (a
// point with u outside [0, n - 1] is outside the geometry), cell
// i = min(floor(u), n - 2), t = u - i, lerps a + t (b - a) along x, y, z.
constexpr float kOutside = 3.0e38f;

__device__ __forceinline__ float grid_sdf_f32(const DevBody& B, const float p[3]) {
#pragma clang fp contract(off)
  float t[3];
  int i[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float d = p[a] - B.go[a];
    const float u = d * B.gih;
    if (!(u >= 0.0f && u <= (float)(B.gn[a] - 1))) return kOutside;
    const int k = min((int)floorf(u), B.gn[a] - 2);
    i[a] = k;
    t[a] = u - (float)k;
  }
  const long long sy = B.gn[0], sz = (long long)B.gn[0] * B.gn[1];
  const float* v = B.gv + ((long long)i[2] * sz + (long long)i[1] * sy + i[0]);
  const float c00 = v[0] + t[0] * (v[1] - v[0]);
  const float c10 = v[sy] + t[0] * (v[sy + 1] - v[sy]);
  const float c01 = v[sz] + t[0] * (v[sz + 1] - v[sz]);
  const float c11 = v[sz + sy] + t[0] * (v[sz + sy + 1] - v[sz + sy]);
  const float c0 = c00 + t[1] * (c10 - c00);
  const float c1 = c01 + t[1] * (c11 - c01);
  return c0 + t[2] * (c1 - c0);
}

// The interpolant and its gradient (with respect to the body-frame point) in
// precision Q, with u clamped into the grid (the point was inside when the
// contact was detected).
template <typename Q>
__device__ __forceinline__ Q grid_sdf_grad(const DevBody& B, const Q p[3], Q g[3]) {
  Q t[3];
  int i[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Q u = (p[a] - (Q)B.go[a]) * (Q)B.gih;
    u = fmin(fmax(u, Q(0)), (Q)(B.gn[a] - 1));
    const int k = min((int)floor(u), B.gn[a] - 2);
    i[a] = k;
    t[a] = u - (Q)k;
  }
  const long long sy = B.gn[0], sz = (long long)B.gn[0] * B.gn[1];
  const float* v = B.gv + ((long long)i[2] * sz + (long long)i[1] * sy + i[0]);
  const Q v000 = v[0], v100 = v[1], v010 = v[sy], v110 = v[sy + 1];
  const Q v001 = v[sz], v101 = v[sz + 1], v011 = v[sz + sy], v111 = v[sz + sy + 1];
  const Q c00 = v000 + t[0] * (v100 - v000), c10 = v010 + t[0] * (v110 - v010);
  const Q c01 = v001 + t[0] * (v101 - v001), c11 = v011 + t[0] * (v111 - v011);
  const Q c0 = c00 + t[1] * (c10 - c00), c1 = c01 + t[1] * (c11 - c01);
  const Q e0 = (v100 - v000) + t[1] * ((v110 - v010) - (v100 - v000));
  const Q e1 = (v101 - v001) + t[1] * ((v111 - v011) - (v101 - v001));
  const Q ih = (Q)B.gih;
  g[0] = (e0 + t[2] * (e1 - e0)) * ih;
  g[1] = ((c10 - c00) + t[2] * ((c11 - c01) - (c10 - c00))) * ih;
  g[2] = (c1 - c0) * ih;
  return c0 + t[2] * (c1 - c0);
}

// Closed-form SDFs (Sec. II-C) in binary32 with a fixed operation order: the
// value that decides contact (psi = f - r <= 0, Eq. (7)).
__device__ __forceinline__ float sdf_decide(const DevBody& B, float x0, float x1, float x2) {
#pragma clang fp contract(off)
  float p[3];
  to_body<float>(B, x0, x1, x2, p);
  if (B.shape == 0) return p[2];
  if (B.shape == 3) return grid_sdf_f32(B, p);
  if (B.shape == 1) {
    float q0 = fabsf(p[0]) - B.params[0];
    float q1 = fabsf(p[1]) - B.params[1];
    float q2 = fabsf(p[2]) - B.params[2];
    float m0 = q0 > 0.0f ? q0 : 0.0f, m1 = q1 > 0.0f ? q1 : 0.0f, m2 = q2 > 0.0f ? q2 : 0.0f;
    float s0 = m0 * m0, s1 = m1 * m1, s2 = m2 * m2;
    float ss = s0 + s1;
    ss = ss + s2;
    float outside = __builtin_sqrtf(ss);
    float in = fmaxf(q0, fmaxf(q1, q2));
    in = in < 0.0f ? in : 0.0f;
    return outside + in;
  }
  float h = B.params[1];
  float cz = fminf(fmaxf(p[2], -h), h);
  float dz = p[2] - cz;
  float s0 = p[0] * p[0], s1 = p[1] * p[1], s2 = dz * dz;
  float ss = s0 + s1;
  ss = ss + s2;
  return __builtin_sqrtf(ss) - B.params[0];
}

__device__ __forceinline__ bool body_touch(const DevBody& B, const float4 xi) {
#pragma clang fp contract(off)
  float f = sdf_decide(B, xi.x, xi.y, xi.z);
  float psi = f - xi.w;
  return psi <= 0.0f;
}

// Signed gap of a particle pair, psi = ||xi - xj|| - (ri + rj) (Eq. (7) for two
// spheres), free of cancellation: differences and squares of binary32 inputs
// are exact in double precision, and psi = (D - S) / (sqrt(D) + s).  The
// expression is symmetric in (i, j) and evaluated without contraction, so
// every kernel and both members of a pair obtain the same bits (the sweeps
// recompute it rather than read it back).
template <typename Q>
__device__ __forceinline__ Q pair_gap(const Q a_x, const Q a_y, const Q a_z, const Q a_w, const Q b_x, const Q b_y,
                                      const Q b_z, const Q b_w) {
#pragma clang fp contract(off)
  const double d0 = (double)a_x - (double)b_x;
  const double d1 = (double)a_y - (double)b_y;
  const double d2 = (double)a_z - (double)b_z;
  const double D = d0 * d0 + d1 * d1 + d2 * d2;
  const double s = (double)a_w + (double)b_w;
  return (Q)((D - s * s) / (sqrt(D) + s));
}
__device__ __forceinline__ float pair_gap(const float4 a, const float4 b) {
  return pair_gap<float>(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
}
__device__ __forceinline__ double pair_gap(const double4 a, const double4 b) {
  return pair_gap<double>(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
}

// Signed gap f(X^-1 x) - r of a body contact in double precision (Eq. (7)),
// from the pose of the build's precision.
template <typename R>
__device__ __forceinline__ R body_gap(const DevBody& B, const V4<R> xi) {
  const auto* Rm = PoseOf<R>::R(B);
  const auto* tv = PoseOf<R>::t(B);
  double d[3] = {(double)xi.x - tv[0], (double)xi.y - tv[1], (double)xi.z - tv[2]};
  double p[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = (double)Rm[c] * d[0] + (double)Rm[3 + c] * d[1] + (double)Rm[6 + c] * d[2];
  double f;
  if (B.shape == 0) {
    f = p[2];
  } else if (B.shape == 3) {
    double g[3];
    f = grid_sdf_grad<double>(B, p, g);
  } else if (B.shape == 1) {
    double q0 = fabs(p[0]) - B.params[0], q1 = fabs(p[1]) - B.params[1], q2 = fabs(p[2]) - B.params[2];
    double m0 = fmax(q0, 0.0), m1 = fmax(q1, 0.0), m2 = fmax(q2, 0.0);
    f = sqrt(m0 * m0 + m1 * m1 + m2 * m2) + fmin(fmax(q0, fmax(q1, q2)), 0.0);
  } else {
    double h = B.params[1];
    double cz = fmin(fmax(p[2], -h), h);
    double e2 = p[2] - cz;
    f = sqrt(p[0] * p[0] + p[1] * p[1] + e2 * e2) - (double)B.params[0];
  }
  return (R)(f - (double)xi.w);
}

// Contact geometry for a body contact with stored gap psi: world normal
// n = R grad f / |R grad f| and the velocity of the body's material point at
// the contact point pc = x - f n, V = nu + om x (pc - t).
template <typename R>
__device__ __forceinline__ void body_geometry(const DevBody& B, const V4<R> xi, R psi, R n[3], R V[3]) {
  const auto* Rm = PoseOf<R>::R(B);
  const auto* tv = PoseOf<R>::t(B);
  const auto* nu = PoseOf<R>::nu(B);
  const auto* om = PoseOf<R>::om(B);
  R p[3];
  to_body<R>(B, xi.x, xi.y, xi.z, p);
  R g[3], f;
  if (B.shape == 0) {
    g[0] = R(0); g[1] = R(0); g[2] = R(1);
    f = p[2];
  } else if (B.shape == 3) {
    f = grid_sdf_grad<R>(B, p, g);
    if (!(g[0] * g[0] + g[1] * g[1] + g[2] * g[2] > R(0))) {
      g[0] = R(1); g[1] = R(0); g[2] = R(0);
    }
  } else if (B.shape == 1) {
    R q[3], m[3];
    bool outside = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[c] = fabs(p[c]) - (R)B.params[c];
      m[c] = fmax(q[c], R(0));
      outside = outside || (q[c] > R(0));
    }
    if (outside) {
      R L = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      R il = R(1) / L;
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = (p[c] < R(0) ? R(-1) : R(1)) * m[c] * il;
      f = L;
    } else {
      int a = 0;
      if (q[1] > q[a]) a = 1;
      if (q[2] > q[a]) a = 2;
      g[0] = g[1] = g[2] = R(0);
      g[a] = p[a] < R(0) ? R(-1) : R(1);
      f = q[a];
    }
  } else {
    R h = B.params[1];
    R cz = fmin(fmax(p[2], -h), h);
    R e0 = p[0], e1 = p[1], e2 = p[2] - cz;
    R L = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    if (L > R(0)) {
      R il = R(1) / L;
      g[0] = e0 * il; g[1] = e1 * il; g[2] = e2 * il;
    } else {
      g[0] = R(1); g[1] = R(0); g[2] = R(0);
    }
    f = L - (R)B.params[0];
  }
  R w0 = Rm[0] * g[0] + Rm[1] * g[1] + Rm[2] * g[2];
  R w1 = Rm[3] * g[0] + Rm[4] * g[1] + Rm[5] * g[2];
  R w2 = Rm[6] * g[0] + Rm[7] * g[1] + Rm[8] * g[2];
  R inl = R(1) / sqrt(w0 * w0 + w1 * w1 + w2 * w2);
  n[0] = w0 * inl; n[1] = w1 * inl; n[2] = w2 * inl;
  f = psi + xi.w;
  R a0 = xi.x - f * n[0] - tv[0];
  R a1 = xi.y - f * n[1] - tv[1];
  R a2 = xi.z - f * n[2] - tv[2];
  V[0] = nu[0] + om[1] * a2 - om[2] * a1;
  V[1] = nu[1] + om[2] * a0 - om[0] * a2;
  V[2] = nu[2] + om[0] * a1 - om[1] * a0;
}

// ------------------------------------------------------------- wave helpers
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_max_i32(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ void set_error(Ctl* ctl, int code, int step) {
  if (atomicCAS(&ctl->err, 0, code) == 0) atomicExch(&ctl->fail_step, step);
}

// ------------------------------------------------------------------ kernels

__global__ void k_begin(Ctl* ctl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->err = 0;
    ctl->fail_step = -1;
    ctl->steps_done = 0;
    ctl->summed = 0;
  }
}

// ------------------------------------------------- spatial (Morton) order
// The internal particle order follows a Z-order curve over the cells so that a
// workgroup's particles occupy a compact block of cells and their neighbours
// sit nearby in memory.  Keys: environment in the high bits, then the Morton
// code of the low 10 bits of each cell coordinate (wrap-around only costs
// locality, never correctness), its node part (all but the low `sh` bits)
// above and its within-node part below 8 bits that order the particles of a
// node by descending contact count at the last detection.  Within a
// wavefront, the particles that still have a k-th contact then sit side by
// side, so row k of the contact table is read and written as one run instead
// of scattered lanes (bytes move in whole 64-byte segments).

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t morton_cell(int k0, int k1, int k2) {
  return spread10((uint32_t)(k0 + 512)) | (spread10((uint32_t)(k1 + 512)) << 1) |
         (spread10((uint32_t)(k2 + 512)) << 2);
}

// Bucket of a cell in the internal table that the counting sort and the
// neighbour queries use (n_blk blocks of 64 buckets).  The Z-order node of
// 4 x 4 x 4 cells holding the cell picks a block through a mixing hash
// (Fibonacci hashing of the node number, then a multiply-shift range
// reduction); the node's 64 cells take consecutive buckets of that block in
// Z-order.  Cells that collide share a bucket and are told apart by their
// coordinates, as with any spatial hash; since neighbouring cells mostly
// share a block, a query's buckets and their members sit together in memory,
// which the XOR hash of Eq. (6) scatters.  The reported cell index is still
// Eq. (6).
__device__ __forceinline__ int table_bucket(int k0, int k1, int k2, int n_blk) {
  const uint32_t m = morton_cell(k0, k1, k2);
  unsigned long long z = (unsigned long long)(m >> 6) * 0x9E3779B97F4A7C15ull;
  z ^= z >> 31;
  const uint32_t blk = (uint32_t)(((z >> 32) * (unsigned long long)(uint32_t)n_blk) >> 32);
  return (int)(blk * 64u + (m & 63u));
}

constexpr int kCountBits = 8;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_morton_keys(int n, const V4<R>* __restrict__ x, float inv_c,
                                                        const int32_t* __restrict__ env_of,
                                                        const int32_t* __restrict__ ncon, int sh,
                                                        unsigned long long* __restrict__ keys) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 p = f32of(x[i]);
  bool ok = true;
  const int k0 = cell_coord(p.x, inv_c, ok), k1 = cell_coord(p.y, inv_c, ok), k2 = cell_coord(p.z, inv_c, ok);
  const unsigned long long m = morton_cell(k0, k1, k2);
  const unsigned long long e = env_of ? (unsigned long long)env_of[i] : 0ull;
  const unsigned long long c = (unsigned long long)(255 - min(max(ncon[i], 0), 255));
  const unsigned long long low = (1ull << sh) - 1;
  keys[i] = (e << (30 + kCountBits)) | ((m & ~low) << kCountBits) | (c << sh) | (m & low);
}

// LSD radix sort, 8-bit digits, stable.  Each block owns kRsItems consecutive
// keys, processed in rounds of 256 (item = base + 256*round + thread).
constexpr int kRsRounds = 16;
constexpr int kRsItems = kBlock * kRsRounds;

__global__ __launch_bounds__(kBlock) void k_rs_hist(int n, const unsigned long long* __restrict__ keys, int shift,
                                                    int nb, int32_t* __restrict__ ghist) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRsItems;
  for (int r = 0; r < kRsRounds; ++r) {
    const int it = base + r * kBlock + threadIdx.x;
    if (it < n) atomicAdd(&hist[(int)((keys[it] >> shift) & 255ull)], 1);
  }
  __syncthreads();
  ghist[threadIdx.x * nb + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter: within a round, a key's rank among equal digits is (equal
// digits in earlier wavefronts) + (equal digits in earlier lanes), the latter
// from an 8-ballot match of the digit.
__global__ __launch_bounds__(kBlock) void k_rs_scatter(int n, const unsigned long long* __restrict__ kin,
                                                       const int32_t* __restrict__ vin,
                                                       unsigned long long* __restrict__ kout,
                                                       int32_t* __restrict__ vout, int shift, int nb,
                                                       const int32_t* __restrict__ gscan) {
  __shared__ int base_d[256];
  __shared__ int wcnt[kBlock / 64][256];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  base_d[threadIdx.x] = gscan[threadIdx.x * nb + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) wcnt[w][threadIdx.x] = 0;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int base = blockIdx.x * kRsItems;
  for (int r = 0; r < kRsRounds; ++r) {
    const int it = base + r * kBlock + threadIdx.x;
    const bool valid = it < n;
    unsigned long long key = valid ? kin[it] : 0ull;
    const int val = valid ? (vin ? vin[it] : it) : 0;
    const int d = (int)((key >> shift) & 255ull);
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long bal = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[wid][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base_d[d] + rank;
      for (int w = 0; w < wid; ++w) pos += wcnt[w][d];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      add += wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = 0;
    }
    base_d[threadIdx.x] += add;
    __syncthreads();
  }
}

// Apply the permutation (new position k takes old index perm[k]) to the state.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_permute(int n, const int32_t* __restrict__ perm,
                                                    const V4<R>* __restrict__ xi, const V4<R>* __restrict__ vi,
                                                    const int32_t* __restrict__ oi, V4<R>* __restrict__ xo,
                                                    V4<R>* __restrict__ vo, int32_t* __restrict__ oo) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int j = perm[k];
  xo[k] = xi[j];
  vo[k] = vi[j];
  oo[k] = oi[j];
}

// ------------------------------------------------------ hash-bucket table
// Cell keys and bucket counters: the internal bucket (table_bucket) for the
// counting sort, and the cell index of Eq. (6) (h6, reported to the caller).
// rank[i] is the arrival order of i in its bucket; the order inside a bucket
// is irrelevant downstream because the members of each cell are re-sorted by
// original index when staged.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_key(int n, const V4<R>* __restrict__ x, float inv_c, int nh, int n_blk,
                                                EnvTables env, int32_t* __restrict__ h, int32_t* __restrict__ h6,
                                                int32_t* __restrict__ rank, int32_t* __restrict__ counts,
                                                Ctl* ctl, int step) {
  if (blockIdx.x == 0 && threadIdx.x == 0 && ctl->err == 0) {
    ctl->n_pp = 0; ctl->n_pb = 0; ctl->cand = 0; ctl->max_cnt = 0; ctl->fallback = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 8) ctl->next_item[threadIdx.x * kQueueStride] = 0;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 p = f32of(x[i]);
  bool ok = true;
  int k0 = cell_coord(p.x, inv_c, ok);
  int k1 = cell_coord(p.y, inv_c, ok);
  int k2 = cell_coord(p.z, inv_c, ok);
  int bucket, cell;
  if (env.env_of) {
    int e = env.env_of[i];
    cell = env.boff[e] + hash_cell(k0, k1, k2, env.nh[e]);
    bucket = env.toff[e] + table_bucket(k0, k1, k2, env.tblk[e]);
  } else {
    cell = hash_cell(k0, k1, k2, nh);
    bucket = table_bucket(k0, k1, k2, n_blk);
  }
  if (!ok) set_error(ctl, 5 /* GG_ERR_NONFINITE */, step);
  h[i] = bucket;
  h6[i] = cell;
  // a cell's particles are mostly consecutive (Z order), so each run of lanes
  // with the same bucket takes one atomic: the run's first lane adds its
  // length, and a lane's rank is the old count plus its place in the run
  // (lanes with i >= n have left, so the active lanes are a prefix).  The
  // shuffle and both ballots run on every active lane, outside any branch: a
  // ballot in a divergent branch sees only that branch's lanes.
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(bucket, 1, 64);
  const unsigned long long live = __ballot(1);
  const unsigned long long heads = __ballot(lane == 0 || prev != bucket);
  const bool head = (heads >> lane) & 1ull;
  const unsigned long long upto = (2ull << lane) - 1ull;  // lanes 0..lane
  const int first = 63 - __clzll(heads & upto);
  const unsigned long long later = heads & ~upto;
  const int end = later ? __ffsll((unsigned long long)later) - 1 : __popcll(live);
  int base = 0;
  if (head) base = atomicAdd(&counts[bucket], end - first);
  base = __shfl(base, first, 64);
  rank[i] = base + (lane - first);
}

// Block-local exclusive scan of kScanTile counters; zeroes the counters when
// asked (the bucket counters are reused next step) and writes the block total.
// Each thread takes four consecutive counters, with 16-byte loads and stores
// where both arrays are 16-byte aligned and the four lie inside [0, m).
__global__ __launch_bounds__(kBlock) void k_scan_a(int m, int32_t* __restrict__ counts,
                                                   int32_t* __restrict__ start, int32_t* __restrict__ bsum,
                                                   int zero) {
  __shared__ int wsum[kBlock / 64];
  const int base = blockIdx.x * kScanTile + threadIdx.x * 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(counts) | reinterpret_cast<uintptr_t>(start)) & 15) == 0 &&
                   base + 3 < m;
  int v[4];
  if (vec) {
    const int4 c4 = *reinterpret_cast<const int4*>(counts + base);
    v[0] = c4.x; v[1] = c4.y; v[2] = c4.z; v[3] = c4.w;
    if (zero) *reinterpret_cast<int4*>(counts + base) = make_int4(0, 0, 0, 0);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = base + q;
      v[q] = e < m ? counts[e] : 0;
      if (zero && e < m) counts[e] = 0;
    }
  }
  const int t = v[0] + v[1] + v[2] + v[3];
  const int s = wave_incl_scan(t);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 63) wsum[wid] = s;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wid; ++w) off += wsum[w];
  int run = off + s - t;
  if (vec) {
    const int r1 = run + v[0], r2 = r1 + v[1], r3 = r2 + v[2];
    *reinterpret_cast<int4*>(start + base) = make_int4(run, r1, r2, r3);
    run = r3 + v[3];
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int e = base + q;
      if (e < m) start[e] = run;
      run += v[q];
    }
  }
  if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = run;
}

// Small beds: the bucket table in one workgroup (k_key, the three scans and
// k_scatter of one step in a single launch).  The counters live in LDS (m + 1
// ints, m <= kSmallBuckets), so the global counters stay zero; the bucket
// starts written to `start` and the members' order within a bucket follow the
// same rules (arrival order within a bucket, which no result depends on).
// One workgroup beats five launches only for a few thousand particles
// (1,024: -14 us per step; 16,384 with 32k buckets: +54 us), hence the bound.
constexpr int kSmallBuckets = 8192;
constexpr int kSmallBlock = 1024;

template <typename R>
__global__ __launch_bounds__(kSmallBlock) void k_bucket_small(
    int n, int m, const V4<R>* __restrict__ x, float inv_c, int nh, int n_blk, EnvTables env,
    int32_t* __restrict__ h, int32_t* __restrict__ h6, int32_t* __restrict__ rank, int32_t* __restrict__ start,
    const int32_t* __restrict__ orig, int32_t* __restrict__ sidx, V4<R>* __restrict__ xs,
    int32_t* __restrict__ os, Ctl* ctl, int step) {
  extern __shared__ int cnt[];        // m + 1
  __shared__ int wsum[kSmallBlock / 64];
  const int tid = threadIdx.x;
  if (tid == 0 && ctl->err == 0) {
    ctl->n_pp = 0; ctl->n_pb = 0; ctl->cand = 0; ctl->max_cnt = 0; ctl->fallback = 0;
  }
  if (tid < 8) ctl->next_item[tid * kQueueStride] = 0;
  for (int e = tid; e <= m; e += kSmallBlock) cnt[e] = 0;
  __syncthreads();
  // cell keys (as k_key); arrival rank within the bucket from an LDS atomic
  for (int i = tid; i < n; i += kSmallBlock) {
    const float4 p = f32of(x[i]);
    bool ok = true;
    const int k0 = cell_coord(p.x, inv_c, ok);
    const int k1 = cell_coord(p.y, inv_c, ok);
    const int k2 = cell_coord(p.z, inv_c, ok);
    int bucket, cell;
    if (env.env_of) {
      const int e = env.env_of[i];
      cell = env.boff[e] + hash_cell(k0, k1, k2, env.nh[e]);
      bucket = env.toff[e] + table_bucket(k0, k1, k2, env.tblk[e]);
    } else {
      cell = hash_cell(k0, k1, k2, nh);
      bucket = table_bucket(k0, k1, k2, n_blk);
    }
    if (!ok) set_error(ctl, 5 /* GG_ERR_NONFINITE */, step);
    h[i] = bucket;
    h6[i] = cell;
    rank[i] = atomicAdd(&cnt[bucket], 1);
  }
  __syncthreads();
  // exclusive scan of the counters: each thread a contiguous chunk
  const int per = (m + kSmallBlock - 1) / kSmallBlock;
  const int b = min(m, tid * per), e = min(m, b + per);
  int t = 0;
  for (int q = b; q < e; ++q) t += cnt[q];
  const int sc = wave_incl_scan(t);
  if ((tid & 63) == 63) wsum[tid >> 6] = sc;
  __syncthreads();
  int run = sc - t;
  for (int w = 0; w < (tid >> 6); ++w) run += wsum[w];
  for (int q = b; q < e; ++q) {
    const int c = cnt[q];
    cnt[q] = run;
    start[q] = run;
    run += c;
  }
  if (tid == kSmallBlock - 1) start[m] = run;
  __syncthreads();
  // members into bucket order (as k_scatter)
  for (int i = tid; i < n; i += kSmallBlock) {
    const int q = cnt[h[i]] + rank[i];
    sidx[q] = i;
    xs[q] = x[i];
    os[q] = orig[i];
  }
}

// Exclusive scan of the block totals (one block); start[m] = total.
__global__ __launch_bounds__(1024) void k_scan_b(int nb, int32_t* __restrict__ bsum, int m,
                                                 int32_t* __restrict__ start) {
  __shared__ int wsum[16];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nb; base += 1024) {
    const int e = base + threadIdx.x;
    const int t = e < nb ? bsum[e] : 0;
    const int s = wave_incl_scan(t);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    int off = carry;
    for (int w = 0; w < wid; ++w) off += wsum[w];
    if (e < nb) bsum[e] = off + s - t;
    __syncthreads();
    if (threadIdx.x == 1023) carry = off + s;
    __syncthreads();
  }
  if (threadIdx.x == 0) start[m] = carry;
}

// Adds the scanned block totals: one workgroup per scan tile (grid
// ceil(m / kScanTile)), four counters per thread as in k_scan_a.
__global__ __launch_bounds__(kBlock) void k_scan_c(int m, const int32_t* __restrict__ bsum,
                                                   int32_t* __restrict__ start) {
  const int base = blockIdx.x * kScanTile + threadIdx.x * 4;
  const int add = bsum[blockIdx.x];
  if ((reinterpret_cast<uintptr_t>(start) & 15) == 0 && base + 3 < m) {
    int4 s4 = *reinterpret_cast<const int4*>(start + base);
    s4.x += add; s4.y += add; s4.z += add; s4.w += add;
    *reinterpret_cast<int4*>(start + base) = s4;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (base + q < m) start[base + q] += add;
  }
}

// Particles into bucket order: index, position and original index, so that a
// bucket's members are read with independent loads.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_scatter(int n, const int32_t* __restrict__ h,
                                                    const int32_t* __restrict__ rank,
                                                    const int32_t* __restrict__ start, const V4<R>* __restrict__ x,
                                                    const int32_t* __restrict__ orig, int32_t* __restrict__ sidx,
                                                    V4<R>* __restrict__ xs, int32_t* __restrict__ os) {
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= n) return;
  const int q = start[h[i]] + rank[i];
  sidx[q] = i;
  xs[q] = x[i];
  os[q] = orig[i];
}

// ----------------------------------------------- detection work items
// Work items are runs of at most TB (the detection workgroup size) consecutive particles of one
// Z-order node (2^node_shift cells), so each item's cells form a compact box.
// Built after every re-sort from the sorted keys.
__global__ __launch_bounds__(kBlock) void k_node_flags(int n, const unsigned long long* __restrict__ keys,
                                                       int node_shift, int32_t* __restrict__ f) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  f[k] = (k == 0 || (keys[k] >> node_shift) != (keys[k - 1] >> node_shift)) ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_node_first(int n, const int32_t* __restrict__ f,
                                                       const int32_t* __restrict__ e, int32_t* __restrict__ first) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < n && f[k]) first[e[k]] = k;
}

__global__ __launch_bounds__(kBlock) void k_item_flags(int n, const int32_t* __restrict__ f,
                                                       const int32_t* __restrict__ e,
                                                       const int32_t* __restrict__ first, int item,
                                                       int32_t* __restrict__ g) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const int node = e[k] + f[k] - 1;
  g[k] = ((k - first[node]) % item) == 0 ? 1 : 0;
}

// item_start[0 .. n_items] (n_items = scan total, item_start[n_items] = n)
__global__ __launch_bounds__(kBlock) void k_item_starts(int n, const int32_t* __restrict__ g,
                                                        const int32_t* __restrict__ hsc,
                                                        int32_t* __restrict__ item_start) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k < n && g[k]) item_start[hsc[k]] = k;
  if (k == 0) item_start[hsc[n]] = n;
}

// Fixed items of `item` particles (used until the first re-sort).
__global__ __launch_bounds__(kBlock) void k_item_fixed(int n, int item, int32_t* __restrict__ item_start,
                                                       int32_t* __restrict__ n_items) {
  const int k = blockIdx.x * kBlock + threadIdx.x;
  const int ni = (n + item - 1) / item;
  if (k < ni) item_start[k] = k * item;
  if (k == 0) {
    item_start[ni] = n;
    *n_items = ni;
  }
}

// ------------------------------------------------------------ detection
constexpr int32_t kHiFlag = 1 << 30;   // partner entry: this particle is the higher original index

__device__ __forceinline__ int block_min(int v, int* red) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[wid] = v;
  __syncthreads();
  int r = red[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = min(r, red[w]);
  return r;
}

__device__ __forceinline__ int block_max(int v, int* red) { return -block_min(-v, red); }

// In-place exclusive scan of a[0..m) in LDS by the whole block; a[m] = total.
__device__ void block_exclusive_scan(int* a, int m, int* red) {
  const int T = blockDim.x;
  const int per = (m + T - 1) / T;
  const int b = threadIdx.x * per, e = min(b + per, m);
  int loc = 0;
  for (int q = b; q < e; ++q) loc += a[q];
  const int incl = wave_incl_scan(loc);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 63) red[wid] = incl;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wid; ++w) off += red[w];
  int run = off + incl - loc;
  for (int q = b; q < e; ++q) {
    const int t = a[q];
    a[q] = run;
    run += t;
  }
  if (threadIdx.x == T - 1) a[m] = run;
  __syncthreads();
}

// Write contact k of particle i (when within capacity).
template <typename R>
__device__ __forceinline__ void put_contact(int i, int k, int K, int32_t code, R psi, int32_t* partner,
                                            R* Psi, bool gap = true) {
  if (k < K) {
    const int sl = ell_slot(i, k, K);
    partner[sl] = code;
    if (gap) Psi[sl] = psi;
  }
}

// Block-wide min of 8 integers (max via negation) with one pair of barriers.
__device__ __forceinline__ void block_min8(int v[8], int (*red)[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q)
    for (int o = 32; o > 0; o >>= 1) v[q] = min(v[q], __shfl_xor(v[q], o, 64));
  const int wid = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < 8; ++q) red[wid][q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    int r = red[0][q];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = min(r, red[w][q]);
    v[q] = r;
  }
}

// Contact detection over work items (runs of at most TB particles of one
// Z-order node); each workgroup takes a contiguous range of items.
// Tile path: the bounding box of the item's cells, widened by one cell, is
// looked up once per cell through the bucket table (table_bucket); the
// buckets' members are copied to LDS, marked by whether they lie in the cell
// queried (buckets alias), and each cell's members are sorted by original
// index; every particle then tests the 27 cells around it from LDS.  Fallback
// path (box or staging larger than the LDS budget, or an item spanning
// environments): each particle queries its 27 cells directly.  Both paths list
// partners in the same canonical order (neighbour cell, then original index),
// then bodies in body order, so results do not depend on the internal order or
// on the path taken.  Also seeds the Jacobi iterate w = v + dt g and the split
// inverse mass s_i = n_i / m_i.
// (five waves per SIMD: the tile's LDS allows five workgroups per CU, and the
// register budget that fits costs only a few bytes of spill)
// Work distribution: with `queue` set (k_detect), the items are cut into one
// contiguous range per XCD (workgroup b runs on XCD b mod 8), and the
// workgroups of an XCD take the items of its range one at a time from a
// counter (Ctl::next_item, zeroed by the key kernels of the step), so no
// workgroup idles while another still holds several items (item times vary
// several-fold); without it (the fused step kernel), workgroup `blk` of `nblk`
// takes a fixed contiguous share.  Either way each item's results depend only
// on its particles.
// pair_gaps: store the gap of every pair contact (the recorded forward needs
// them; the sweeps recompute a pair's gap from the positions, so plain steps
// skip the double-precision gap and its store).
// (k_detect and the fused step call it)
template <typename R, int TB>
__device__ __forceinline__ void detect_items(
    int n, int K, const V4<R>* __restrict__ x, const V4<R>* __restrict__ v, const int32_t* __restrict__ orig,
    float inv_c, int n_blk, EnvTables env, const int32_t* __restrict__ start, const int32_t* __restrict__ sidx,
    const V4<R>* __restrict__ xs, const int32_t* __restrict__ os, const int32_t* __restrict__ item_start,
    const int32_t* __restrict__ n_items_ptr, const DevBody* __restrict__ bodies, int n_bodies, R gx,
    R gy, R gz, R dt, int mass_split, int max_cells, int max_stage, int32_t* __restrict__ ncon,
    int32_t* __restrict__ partner, R* __restrict__ Psi, V4<R>* __restrict__ w, R* __restrict__ imass, Ctl* ctl,
    DetPart* __restrict__ part, int step, int blk, int nblk, bool queue, bool pair_gaps) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int red8[TB / 64][8];
  __shared__ int red[TB / 64];
  __shared__ int grabbed;
  int* cell_off = (int*)smem;                                  // max_cells + 1
  int* cell_s = cell_off + (max_cells + 1);                    // max_cells: first bucket entry
  V4<R>* st_x = (V4<R>*)(smem + ((((2 * max_cells + 1) * 4) + 31) & ~31));  // max_stage
  int2* st_jo = (int2*)(st_x + max_stage);                     // max_stage: (index (-1: other cell), original index)

  const int n_items = *n_items_ptr;
  int it0, it1, qx = 0;
  if (queue) {
    const int nq = min(8, nblk);   // every queue has a workgroup (b = qx)
    qx = (int)(blockIdx.x % (unsigned)nq);
    it0 = (int)((int64_t)qx * n_items / nq);
    it1 = (int)((int64_t)(qx + 1) * n_items / nq);
  } else {
    const int per = (n_items + nblk - 1) / nblk;
    it0 = min(blk * per, n_items);
    it1 = min(it0 + per, n_items);
  }
  int cand = 0, npp = 0, npb = 0, mx = 0, fb = 0;
  const int BIG = 0x3fffffff;
  // (thread 0 takes the next item while the workgroup works on the current one)
  int ahead = (queue && threadIdx.x == 0) ? atomicAdd(&ctl->next_item[qx * kQueueStride], 1) : 0;

  for (int item = it0;; ++item) {
    if (queue) {
      // the same item for the whole workgroup; the last barrier of the
      // previous item orders this write after every read of `grabbed`
      if (threadIdx.x == 0) grabbed = it0 + ahead;
      __syncthreads();
      item = grabbed;
      if (threadIdx.x == 0 && item < it1) ahead = atomicAdd(&ctl->next_item[qx * kQueueStride], 1);
    }
    if (item >= it1) break;
    const int i = item_start[item] + threadIdx.x;
    const bool active = i < item_start[item + 1];
    const V4<R> p = active ? x[i] : mk4<R>(R(0), R(0), R(0), R(0));
    const float4 p32 = f32of(p);
    const int oi = active ? orig[i] : 0;
    bool ok = true;
    const int k0 = cell_coord(p32.x, inv_c, ok), k1 = cell_coord(p32.y, inv_c, ok), k2 = cell_coord(p32.z, inv_c, ok);
    const int e_i = (env.env_of && active) ? env.env_of[i] : 0;
    int tab_n = n_blk, tab_off = 0, b_lo = 0, b_hi = n_bodies;
    if (env.env_of && active) {
      tab_n = env.tblk[e_i];
      tab_off = env.toff[e_i];
      b_lo = env.body_lo[e_i];
      b_hi = env.body_hi[e_i];
    }
    int bb[8] = {active ? k0 : BIG, active ? k1 : BIG, active ? k2 : BIG, active ? e_i : BIG,
                 active ? -k0 : BIG, active ? -k1 : BIG, active ? -k2 : BIG, active ? -e_i : BIG};
    block_min8(bb, red8);
    const int lo0 = bb[0], lo1 = bb[1], lo2 = bb[2], hi0 = -bb[4], hi1 = -bb[5], hi2 = -bb[6];
    bool tile = (bb[3] == -bb[7]) && (hi0 - lo0 < 256) && (hi1 - lo1 < 256) && (hi2 - lo2 < 256);
    const int Dx = hi0 - lo0 + 3, Dy = hi1 - lo1 + 3, Dz = hi2 - lo2 + 3;
    const int NC = tile ? Dx * Dy * Dz : 0;
    tile = tile && NC <= max_cells;
    const int ex = lo0 - 1, ey = lo1 - 1, ez = lo2 - 1;
    int t_n = n_blk, t_off = 0;
    if (env.env_of && tile) {
      t_n = env.tblk[bb[3]];
      t_off = env.toff[bb[3]];
    }
    if (tile) {
      // bucket extents of every cell of the box: independent loads
      for (int c = threadIdx.x; c < NC; c += TB) {
        const int cx = ex + c % Dx, cy = ey + (c / Dx) % Dy, cz = ez + c / (Dx * Dy);
        const int hb = t_off + table_bucket(cx, cy, cz, t_n);
        const int s0 = start[hb];
        cell_s[c] = s0;
        cell_off[c] = start[hb + 1] - s0;
      }
      __syncthreads();
      block_exclusive_scan(cell_off, NC, red);
      tile = cell_off[NC] <= max_stage;
    }
    int cnt = 0;
    if (tile) {
      // copy the members, mark those of other cells, sort by original index
      for (int c = threadIdx.x; c < NC; c += TB) {
        const int cx = ex + c % Dx, cy = ey + (c / Dx) % Dy, cz = ez + c / (Dx * Dy);
        const int s0 = cell_s[c], first = cell_off[c], m = cell_off[c + 1] - first;
        for (int u = 0; u < m; ++u) {
          const V4<R> pj = xs[s0 + u];
          const float4 pj32 = f32of(pj);
          bool okj = true;
          const bool mine = cell_coord(pj32.x, inv_c, okj) == cx && cell_coord(pj32.y, inv_c, okj) == cy &&
                            cell_coord(pj32.z, inv_c, okj) == cz;
          st_x[first + u] = pj;
          st_jo[first + u] = mine ? make_int2(sidx[s0 + u], os[s0 + u]) : make_int2(-1, 0x7fffffff);
        }
        for (int u = 1; u < m; ++u) {
          const V4<R> kx = st_x[first + u];
          const int2 kjo = st_jo[first + u];
          int at = first + u;
          while (at > first && st_jo[at - 1].y > kjo.y) {
            st_x[at] = st_x[at - 1];
            st_jo[at] = st_jo[at - 1];
            --at;
          }
          st_x[at] = kx;
          st_jo[at] = kjo;
        }
      }
      __syncthreads();
      if (active) {
        // the three cells dx = -1, 0, 1 of a row are consecutive in the tile,
        // and so are their staged members: one scan per row, skipping the
        // other cells' members (sorted last within each cell), visits the
        // partners in the same order as 27 cell scans.  The scan reads four
        // members at a time (their loads in flight together; past the row's
        // end the last member is read again and skipped) and tests them in
        // order.
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy) {
            const int c = ((k2 + dz - ez) * Dy + (k1 + dy - ey)) * Dx + (k0 - 1 - ex);
            const int s0 = cell_off[c], s1 = cell_off[c + 3];
            for (int q0 = s0; q0 < s1; q0 += 4) {
              int2 jo[4];
              V4<R> px[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int q = min(q0 + u, s1 - 1);
                jo[u] = st_jo[q];
                px[u] = st_x[q];
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int j = jo[u].x;
                if (q0 + u >= s1 || j < 0 || j == i) continue;
                ++cand;
                if (!pair_touch(p32, f32of(px[u]))) continue;
                const int oj = jo[u].y;
                npp += oi < oj;
                put_contact(i, cnt, K, j | (oi < oj ? 0 : kHiFlag), pair_gaps ? pair_gap(p, px[u]) : R(0), partner,
                            Psi, pair_gaps);
                ++cnt;
              }
            }
          }
      }
    } else {
      fb += (threadIdx.x == 0);
      if (active) {
        for (int dz = -1; dz <= 1; ++dz)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
              const int c0 = k0 + dx, c1 = k1 + dy, c2 = k2 + dz;
              const int hb = tab_off + table_bucket(c0, c1, c2, tab_n);
              const int s0 = start[hb], s1 = start[hb + 1];
              const int first = cnt;
              for (int q = s0; q < s1; ++q) {
                const V4<R> pj = xs[q];
                const float4 pj32 = f32of(pj);
                bool okj = true;
                if (cell_coord(pj32.x, inv_c, okj) != c0 || cell_coord(pj32.y, inv_c, okj) != c1 ||
                    cell_coord(pj32.z, inv_c, okj) != c2)
                  continue;
                const int j = sidx[q];
                if (j == i) continue;
                ++cand;
                if (!pair_touch(p32, pj32)) continue;
                const int oj = os[q];
                npp += oi < oj;
                // keep this cell's partners sorted by original index (in place)
                int at = cnt;
                if (cnt < K) {
                  while (at > first) {
                    const int prev = partner[ell_slot(i, at - 1, K)];
                    if (orig[prev & (kHiFlag - 1)] < oj) break;
                    partner[ell_slot(i, at, K)] = prev;
                    if (pair_gaps) Psi[ell_slot(i, at, K)] = Psi[ell_slot(i, at - 1, K)];
                    --at;
                  }
                }
                put_contact(i, at, K, j | (oi < oj ? 0 : kHiFlag), pair_gaps ? pair_gap(p, pj) : R(0), partner,
                            Psi, pair_gaps);
                ++cnt;
              }
            }
      }
    }
    if (active) {
      for (int b = b_lo; b < b_hi; ++b) {
        const DevBody& B = bodies[b];
        // a particle outside the body's box is farther than r_max from it
        if (B.cull && (p32.x < B.lo[0] || p32.x > B.hi[0] || p32.y < B.lo[1] || p32.y > B.hi[1] ||
                       p32.z < B.lo[2] || p32.z > B.hi[2]))
          continue;
        if (body_touch(B, p32)) {
          put_contact(i, cnt, K, -1 - b, body_gap<R>(bodies[b], p), partner, Psi);
          ++cnt;
          ++npb;
        }
      }
      ncon[i] = cnt < K ? cnt : K;
      if (cnt > K) set_error(ctl, 4 /* GG_ERR_CAPACITY */, step);
      mx = max(mx, cnt);
      const V4<R> vi = v[i];
      const R s_i = mass_split ? (R)cnt * vi.w : vi.w;
      w[i] = mk4<R>(vi.x + dt * gx, vi.y + dt * gy, vi.z + dt * gz, s_i);
      imass[i] = vi.w;
    }
    __syncthreads();  // LDS is reused by the next item
  }
  // statistics: summed over the wavefronts, then the workgroup's counts in its
  // own slot (every thread has passed the loop's last barrier)
  __shared__ unsigned long long st_sum[TB / 64][3];
  __shared__ int st_max[TB / 64];
  const unsigned long long a = wave_sum_u64((unsigned long long)npp);
  const unsigned long long b2 = wave_sum_u64((unsigned long long)npb);
  const unsigned long long c = wave_sum_u64((unsigned long long)cand);
  mx = wave_max_i32(mx);
  if ((threadIdx.x & 63) == 0) {
    st_sum[threadIdx.x >> 6][0] = a;
    st_sum[threadIdx.x >> 6][1] = b2;
    st_sum[threadIdx.x >> 6][2] = c;
    st_max[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    DetPart d{0ull, 0ull, 0ull, 0, (fb << 1) | 1};
    for (int q = 0; q < TB / 64; ++q) {
      d.n_pp += st_sum[q][0];
      d.n_pb += st_sum[q][1];
      d.cand += st_sum[q][2];
      d.max_cnt = max(d.max_cnt, st_max[q]);
    }
    part[blk] = d;
  }
}

template <typename R, int TB>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(5))) void k_detect(
    int n, int K, const V4<R>* __restrict__ x, const V4<R>* __restrict__ v, const int32_t* __restrict__ orig,
    float inv_c, int n_blk, EnvTables env, const int32_t* __restrict__ start, const int32_t* __restrict__ sidx,
    const V4<R>* __restrict__ xs, const int32_t* __restrict__ os, const int32_t* __restrict__ item_start,
    const int32_t* __restrict__ n_items_ptr, const DevBody* __restrict__ bodies, int n_bodies, R gx,
    R gy, R gz, R dt, int mass_split, int max_cells, int max_stage, int32_t* __restrict__ ncon,
    int32_t* __restrict__ partner, R* __restrict__ Psi, V4<R>* __restrict__ w, R* __restrict__ imass, Ctl* ctl,
    DetPart* __restrict__ part, int step, int queue, int pair_gaps) {
  // the error word is read once per workgroup: every wave of it takes the
  // same branch (the work queue needs all of them)
  __shared__ int err0;
  if (threadIdx.x == 0) err0 = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (err0) return;
  detect_items<R, TB>(n, K, x, v, orig, inv_c, n_blk, env, start, sidx, xs, os, item_start, n_items_ptr, bodies,
                      n_bodies, gx, gy, gz, dt, mass_split, max_cells, max_stage, ncon, partner, Psi, w, imass, ctl,
                      part, step, xcd_block(), gridDim.x, queue != 0, pair_gaps != 0);
}

// Totals of one detection from its workgroups' counts, which are cleared for
// the next detection; run by one whole workgroup of kBlock threads.  A
// detection whose workgroups all stopped at an earlier failure of the call
// leaves the control block as it was.  rec (differentiable calls, else null):
// the step's pair and body contact counts.
__device__ void detect_stats_block(int nblk, DetPart* __restrict__ part, Ctl* ctl,
                                   unsigned long long* __restrict__ rec) {
  __shared__ unsigned long long ws[kBlock / 64][5];
  __shared__ int wm[kBlock / 64];
  unsigned long long pp = 0, pb = 0, cd = 0, fb = 0, ran = 0;
  int mx = 0;
  for (int q = threadIdx.x; q < nblk; q += kBlock) {
    const DetPart d = part[q];
    pp += d.n_pp;
    pb += d.n_pb;
    cd += d.cand;
    mx = max(mx, d.max_cnt);
    fb += (unsigned)d.fb_ran >> 1;
    ran += d.fb_ran & 1;
    part[q] = DetPart{0ull, 0ull, 0ull, 0, 0};
  }
  pp = wave_sum_u64(pp);
  pb = wave_sum_u64(pb);
  cd = wave_sum_u64(cd);
  fb = wave_sum_u64(fb);
  ran = wave_sum_u64(ran);
  mx = wave_max_i32(mx);
  if ((threadIdx.x & 63) == 0) {
    const int w = threadIdx.x >> 6;
    ws[w][0] = pp; ws[w][1] = pb; ws[w][2] = cd; ws[w][3] = fb; ws[w][4] = ran;
    wm[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      pp += ws[w][0]; pb += ws[w][1]; cd += ws[w][2]; fb += ws[w][3]; ran += ws[w][4];
      mx = max(mx, wm[w]);
    }
    if (ran) {
      ctl->n_pp = pp;
      ctl->n_pb = pb;
      ctl->cand = cd;
      ctl->max_cnt = mx;
      ctl->fallback = (int32_t)fb;
      ctl->summed += pp + pb;
    }
    if (rec) {
      rec[0] = ctl->n_pp;
      rec[1] = ctl->n_pb;
    }
  }
}

// The statistics of the fused step's detection (the split step sums them in
// k_integrate).
__global__ __launch_bounds__(kBlock) void k_detect_stats(int nblk, DetPart* __restrict__ part, Ctl* ctl,
                                                         unsigned long long* __restrict__ rec) {
  detect_stats_block(nblk, part, ctl, rec);
}

// ------------------------------------------------------ projected Jacobi
// One sweep (Alg. 1).  Every contact reads the iterate of the previous sweep
// (w_in) and its own accumulated world impulse P (on the member with the lower
// original index, or on the particle for a body contact), forms the contact
// velocity u = w_lo - w_hi (or w_i - V for a body), and takes the step
// y = P - mt (u + alpha psi/dt n) in the contact frame (e1 = n): the normal
// part is clamped at 0 and the tangential part y - (y.n) n scaled to length at
// most mu y.n (Eqs. (2)-(3)); the frame's tangent axes never need to be built
// because the projection is isotropic in the tangent plane.  mt = 1/(s_lo +
// s_hi) for a pair, 1/s_i for a body (mass splitting).  The particle then sums
// its contacts' impulses in list order: w_i = w0_i + (1/m_i) sum sigma P_c.
// The gap psi of a pair is recomputed from the two positions (pair_gap, the
// bits detection stored), which saves streaming it; a body contact's is read.
// mode bit 0: first sweep (impulses start at 0); bit 1: last sweep (write v and
// optionally dv instead of w_out).  Impulses are read from Pi* and written to P*
// (the same arrays, or per-sweep arrays when the sweeps are recorded).  With
// one lane per particle they lie in jagged rows (rec_row): in each group's
// block of the contact table, or, recorded, from the group's compact offset
// pofs[64 g] (pofs: the prefix sum of the contact counts).  With several
// lanes: at the contact's table slot, or, recorded, at pofs[i] + k.
// One half contact of a sweep: the impulse Q of contact `code` (slot `slot`,
// impulse index `ps`) of particle i from the previous impulse P and iterate,
// stored to P*, P itself, and the sign sg with which it enters i's sum.  Multiply-adds
// are fused only within one expression (fp contract on), so every kernel that
// calls it computes the same bits.
template <typename R>
__device__ __forceinline__ void half_contact(int code, int slot, int ps, bool first, const V4<R>& xi,
                                             const V4<R>& wi, const V4<R>* __restrict__ x,
                                             const V4<R>* __restrict__ w_in, const R* __restrict__ Psi,
                                             const R* Pix, const R* Piy, const R* Piz, R* Px, R* Py, R* Pz,
                                             const DevBody* __restrict__ bodies, R alpha_dt, R mu, R relax,
                                             R& Q0, R& Q1, R& Q2, R& P0, R& P1, R& P2, R& sg) {
#pragma clang fp contract(on)
  R psi;
  P0 = R(0); P1 = R(0); P2 = R(0);
  if (!first) {
    P0 = Pix[ps]; P1 = Piy[ps]; P2 = Piz[ps];
  }
  R n0, n1, n2, u0, u1, u2, mt;
  if (code >= 0) {
    const int j = code & (kHiFlag - 1);
    const bool lo = (code & kHiFlag) == 0;
    const V4<R> xj = x[j];
    const V4<R> wj = w_in[j];
    psi = pair_gap(xi, xj);
    const V4<R> xl = lo ? xi : xj, xh = lo ? xj : xi;
    const V4<R> wl = lo ? wi : wj, wh = lo ? wj : wi;
    const R d0 = xl.x - xh.x, d1 = xl.y - xh.y, d2 = xl.z - xh.z;
    const R L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (L > R(0)) {
      const R il = R(1) / L;
      n0 = d0 * il; n1 = d1 * il; n2 = d2 * il;
    } else {
      n0 = R(0); n1 = R(0); n2 = R(1);
    }
    u0 = wl.x - wh.x; u1 = wl.y - wh.y; u2 = wl.z - wh.z;
    mt = R(1) / (wl.w + wh.w);
    sg = lo ? R(1) : R(-1);
  } else {
    R nb[3], V[3];
    psi = Psi[slot];
    body_geometry<R>(bodies[-1 - code], xi, psi, nb, V);
    n0 = nb[0]; n1 = nb[1]; n2 = nb[2];
    u0 = wi.x - V[0]; u1 = wi.y - V[1]; u2 = wi.z - V[2];
    mt = R(1) / wi.w;
    sg = R(1);
  }
  const R bias = alpha_dt * psi;
  const R y0 = P0 - mt * (u0 + bias * n0);
  const R y1 = P1 - mt * (u1 + bias * n1);
  const R y2 = P2 - mt * (u2 + bias * n2);
  const R yn = n0 * y0 + n1 * y1 + n2 * y2;
  R t0 = y0 - yn * n0, t1 = y1 - yn * n1, t2 = y2 - yn * n2;
  const R ynp = fmax(yn, R(0));
  const R ts = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
  if (ts > mu * ynp) {
    const R f = mu * ynp / ts;
    t0 *= f; t1 *= f; t2 *= f;
  }
  Q0 = ynp * n0 + t0; Q1 = ynp * n1 + t1; Q2 = ynp * n2 + t2;
  if (relax != R(1)) {
    Q0 = P0 + relax * (Q0 - P0);
    Q1 = P1 + relax * (Q1 - P1);
    Q2 = P2 + relax * (Q2 - P2);
  }
  Px[ps] = Q0; Py[ps] = Q1; Pz[ps] = Q2;
}

// The particle's new iterate.  Jacobi: w = w0 + im sum sigma Q; it is formed
// from the previous iterate as w = w_prev + im sum sigma (Q - P), which is the
// same in exact arithmetic and spares reading v (w0 = v + dt g) every sweep.
// d = sum sigma (Q - P); a = sum sigma Q (only for the velocity change dv).
// The last sweep writes the velocity.
template <typename R>
__device__ __forceinline__ void finish_particle(int i, bool last, R im, const V4<R>& wi, R d0, R d1, R d2, R a0,
                                                R a1, R a2, V4<R>* __restrict__ v, V4<R>* __restrict__ w_out,
                                                V4<R>* __restrict__ dv) {
#pragma clang fp contract(on)
  const R n0 = wi.x + im * d0;
  const R n1 = wi.y + im * d1;
  const R n2 = wi.z + im * d2;
  if (last) {
    v[i] = mk4<R>(n0, n1, n2, im);
    if (dv) dv[i] = mk4<R>(im * a0, im * a1, im * a2, R(0));
  } else {
    w_out[i] = mk4<R>(n0, n1, n2, wi.w);
  }
}

// Impulses with one lane per particle: the 64 particles of a wavefront (an
// aligned group) keep theirs in jagged rows -- row k holds, in lane order, the
// particles that have a contact k, and the rows follow each other without
// gaps from the group's base: its block of the contact table, 64 K g, or,
// recorded, its first compact offset pofs[64 g].  A group's impulses are then
// one contiguous run of its contact count, and each row is a contiguous part
// of it, so a wavefront's loads and stores touch no cache line that holds
// none of its impulses.  Called by the lanes that have contact k, once per k
// in increasing order; `rbase` starts at the group's base and is advanced past
// the row.  (The forward sweep and its reverse both call it, so they agree on
// every index; the host's reader of impulses follows the same rule.)
__device__ __forceinline__ int rec_row(int& rbase) {
  const unsigned long long row = __ballot(1);
  const unsigned long long below = (1ull << (threadIdx.x & 63)) - 1ull;
  const int q = rbase + __popcll(row & below);
  rbase += __popcll(row);
  return q;
}

// (one particle's part of a sweep; k_pja and the fused step call it)
template <typename R>
__device__ __forceinline__ void pja_particle(int i, int K, const V4<R>* __restrict__ x,
                                             V4<R>* __restrict__ v, const V4<R>* __restrict__ w_in,
                                             V4<R>* __restrict__ w_out, const int32_t* __restrict__ ncon,
                                             const int32_t* __restrict__ partner,
                                             const R* __restrict__ Psi, const R* Pix,
                                             const R* Piy, const R* Piz, R* Px, R* Py,
                                             R* Pz, const DevBody* __restrict__ bodies, R gx, R gy,
                                             R gz, R dt, R alpha_dt, R mu, R relax,
                                             int mode, V4<R>* __restrict__ dv, const int32_t* __restrict__ pofs,
                                             const R* __restrict__ imass) {
#pragma clang fp contract(on)
  const bool first = mode & 1, last = mode & 2;
  const V4<R> xi = x[i];
  const V4<R> wi = w_in[i];
  const R im = imass[i];
  R d0 = R(0), d1 = R(0), d2 = R(0), a0 = R(0), a1 = R(0), a2 = R(0);
  const int c = ncon[i];
  int rbase = pofs ? pofs[i & ~63] : (i >> 6) * (K << 6);
  for (int k = 0; k < c; ++k) {
    const int slot = ell_slot(i, k, K);
    const int ps = rec_row(rbase);   // impulse index (jagged rows)
    R Q0, Q1, Q2, P0, P1, P2, sg;
    half_contact<R>(partner[slot], slot, ps, first, xi, wi, x, w_in, Psi, Pix, Piy, Piz, Px, Py, Pz, bodies,
                    alpha_dt, mu, relax, Q0, Q1, Q2, P0, P1, P2, sg);
    const R D0 = Q0 - P0, D1 = Q1 - P1, D2 = Q2 - P2;
    d0 += sg * D0; d1 += sg * D1; d2 += sg * D2;
    if (last && dv) {
      a0 += sg * Q0; a1 += sg * Q1; a2 += sg * Q2;
    }
  }
  finish_particle<R>(i, last, im, wi, d0, d1, d2, a0, a1, a2, v, w_out, dv);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_pja(int n, int K, const V4<R>* __restrict__ x,
                                                V4<R>* __restrict__ v, const V4<R>* __restrict__ w_in,
                                                V4<R>* __restrict__ w_out, const int32_t* __restrict__ ncon,
                                                const int32_t* __restrict__ partner,
                                                const R* __restrict__ Psi, const R* Pix,
                                                const R* Piy, const R* Piz, R* Px, R* Py,
                                                R* Pz, const DevBody* __restrict__ bodies, R gx, R gy,
                                                R gz, R dt, R alpha_dt, R mu, R relax,
                                                int mode, V4<R>* __restrict__ dv, const int32_t* __restrict__ pofs,
                                                const R* __restrict__ imass, const Ctl* ctl) {
  if (ctl->err) return;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= n) return;
  pja_particle<R>(i, K, x, v, w_in, w_out, ncon, partner, Psi, Pix, Piy, Piz, Px, Py, Pz, bodies, gx, gy, gz, dt,
                  alpha_dt, mu, relax, mode, dv, pofs, imass);
}

// The same sweep with L lanes per particle (L = 2 or 4; small beds, where a
// sweep is bound by each lane's chain of dependent loads, not by bandwidth).
// Lane s of a particle takes its contacts s, s + L, s + 2L, ...; after every
// round of L contacts all lanes of the particle add the round's impulses in
// list order (cross-lane shuffles), so the sum -- and every result -- is
// bitwise that of k_pja, with a chain L times shorter.
template <typename R, int L>
__global__ __launch_bounds__(kBlock) void k_pja_lanes(int n, int K, const V4<R>* __restrict__ x,
                                                      V4<R>* __restrict__ v, const V4<R>* __restrict__ w_in,
                                                      V4<R>* __restrict__ w_out, const int32_t* __restrict__ ncon,
                                                      const int32_t* __restrict__ partner,
                                                      const R* __restrict__ Psi, const R* Pix, const R* Piy,
                                                      const R* Piz, R* Px, R* Py, R* Pz,
                                                      const DevBody* __restrict__ bodies, R gx, R gy, R gz, R dt,
                                                      R alpha_dt, R mu, R relax, int mode,
                                                      V4<R>* __restrict__ dv, const int32_t* __restrict__ pofs,
                                                      const R* __restrict__ imass, const Ctl* ctl) {
#pragma clang fp contract(on)
  static_assert(L == 2 || L == 4, "lanes per particle");
  if (ctl->err) return;
  const int t = xcd_block() * kBlock + threadIdx.x;
  const int i = t / L, sub = t % L;
  if (i >= n) return;  // (the L lanes of a particle leave together)
  const bool first = mode & 1, last = mode & 2;
  const int pbase = pofs ? pofs[i] : 0;
  const V4<R> xi = x[i];
  const V4<R> wi = w_in[i];
  const R im = imass[i];
  R d0 = R(0), d1 = R(0), d2 = R(0), a0 = R(0), a1 = R(0), a2 = R(0);
  const int c = ncon[i];
  for (int m = 0; m * L < c; ++m) {
    const int k = m * L + sub;
    R Q0 = R(0), Q1 = R(0), Q2 = R(0), P0 = R(0), P1 = R(0), P2 = R(0), sg = R(0);
    if (k < c) {
      const int slot = ell_slot(i, k, K);
      half_contact<R>(partner[slot], slot, pofs ? pbase + k : slot, first, xi, wi, x, w_in, Psi, Pix, Piy, Piz,
                      Px, Py, Pz, bodies, alpha_dt, mu, relax, Q0, Q1, Q2, P0, P1, P2, sg);
    }
    const R D0 = Q0 - P0, D1 = Q1 - P1, D2 = Q2 - P2;
#pragma unroll
    for (int q = 0; q < L; ++q) {
      const R g = __shfl(sg, q, L), e0 = __shfl(D0, q, L), e1 = __shfl(D1, q, L), e2 = __shfl(D2, q, L);
      if (m * L + q < c) {
        d0 += g * e0; d1 += g * e1; d2 += g * e2;
      }
      if (last && dv) {   // (the same for every lane of the launch)
        const R q0 = __shfl(Q0, q, L), q1 = __shfl(Q1, q, L), q2 = __shfl(Q2, q, L);
        if (m * L + q < c) {
          a0 += g * q0; a1 += g * q1; a2 += g * q2;
        }
      }
    }
  }
  if (sub == 0) finish_particle<R>(i, last, im, wi, d0, d1, d2, a0, a1, a2, v, w_out, dv);
}

// Positions from the new velocities (Eq. (5)), x' = x + dt v'; with a cyclic
// vertical boundary (zspan > 0) a particle below zlo moves up by zspan.
template <typename R>
__device__ __forceinline__ void integrate_particle(int i, V4<R>* __restrict__ x, const V4<R>* __restrict__ v, R dt,
                                                   R zlo, R zspan) {
  V4<R> p = x[i];
  const V4<R> q = v[i];
  p.x += dt * q.x; p.y += dt * q.y; p.z += dt * q.z;
  if (zspan > R(0) && p.z < zlo) p.z += zspan;
  x[i] = p;
}

// Positions of one step; workgroup 0 first sums the step's detection
// statistics (detect_stats_block over nblk slots; part null: none), also
// after a failure, which needs the largest contact count.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_integrate(int n, V4<R>* __restrict__ x,
                                                      const V4<R>* __restrict__ v, R dt, R zlo, R zspan,
                                                      Ctl* ctl, DetPart* __restrict__ part, int nblk,
                                                      unsigned long long* __restrict__ rec) {
  if (blockIdx.x == 0 && part) detect_stats_block(nblk, part, ctl, rec);
  if (ctl->err) return;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&ctl->steps_done, 1);
  if (i >= n) return;
  integrate_particle<R>(i, x, v, dt, zlo, zspan);
}

// ---------------------------------------------------------------- readout
// Internal (Z-ordered) arrays back to the caller's order: out[orig[k]] = a[k].
// (Values of the double build are rounded to binary32 on the way out.)
template <typename R>
__global__ void k_unpermute3(int n, const int32_t* __restrict__ orig, const V4<R>* __restrict__ a,
                             float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const V4<R> q = a[k];
  const int o = orig[k];
  out[3 * o] = (float)q.x; out[3 * o + 1] = (float)q.y; out[3 * o + 2] = (float)q.z;
}

template <typename R>
__global__ void k_unpermute_w(int n, const int32_t* __restrict__ orig, const V4<R>* __restrict__ a,
                              float* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[orig[k]] = (float)a[k].w;
}

__global__ void k_unpermute_i64(int n, const int32_t* __restrict__ orig, const int32_t* __restrict__ a,
                                int64_t* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[orig[k]] = a[k];
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

__global__ void k_iota(int n, int32_t* __restrict__ a) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = k;
}

}  // namespace ggk
