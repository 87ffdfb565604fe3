// Reverse-mode adjoint of the granular contact step (gfx950).
//
// The forward step (kernels.hip.h) maps the state (x, v) at the start of a step,
// the body poses and the body twists to the next state.  Its adjoint runs the
// projected-Jacobi sweeps of Alg. 1 backwards from recorded iterates, with the
// contact set frozen: d max(z, 0)/dz = [z > 0], the tangential scaling
// differentiated where it is active (strict '>' as in the forward), and the
// contact geometry (normals, gaps, body point velocities) differentiated with
// respect to positions, body poses and twists (SDF gradients and Hessians).
//
// Recorded impulses and the adjoint's per-contact state are indexed compactly,
// pofs[i] + k with pofs the prefix sum of the contact counts.
// Per half contact the adjoint keeps a carry (the adjoint of the impulse of the
// previous sweep, identical bits in both halves of a pair, as the forward's
// impulse copies) and accumulators of the adjoints of the normal, the gap and
// the body point velocity over all sweeps; per particle it keeps the adjoint
// of the iterate.  Like the forward, every particle gathers its own half
// contacts: no atomics, deterministic results.
#pragma once
#include "kernels.hip.h"

namespace ggk {

struct AdjSlots {         // per half-contact adjoint state (SoA)
  float *cx, *cy, *cz;    // carry: adjoint of the impulse of the previous sweep
  float *nx, *ny, *nz;    // accumulated adjoint of the contact normal (lower-index orientation)
  float *ps;              // accumulated adjoint of the gap psi
  float *vx, *vy, *vz;    // accumulated adjoint of the body point velocity V
};

__device__ __forceinline__ float dot3f(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Adjoint of the projection Q = proj(y, n) of the forward sweep, given Qbar.
// Returns ybar and adds the normal's share to nbar.
__device__ __forceinline__ void proj_adjoint(const float y[3], const float n[3], float mu, const float Qb[3],
                                             float yb[3], float nb[3]) {
  const float yn = dot3f(n, y);
  float t[3] = {y[0] - yn * n[0], y[1] - yn * n[1], y[2] - yn * n[2]};
  const float ynp = fmaxf(yn, 0.0f);
  const float ts = sqrtf(dot3f(t, t));
  const bool scaled = ts > mu * ynp;
  if (yn <= 0.0f) {
    if (scaled) {  // Q = 0 identically
      yb[0] = yb[1] = yb[2] = 0.0f;
      return;
    }
    // Q = y - (n.y) n
    const float qn = dot3f(Qb, n);
    for (int a = 0; a < 3; ++a) {
      yb[a] = Qb[a] - qn * n[a];
      nb[a] += -qn * y[a] - yn * Qb[a];
    }
    return;
  }
  if (!scaled) {  // Q = y
    for (int a = 0; a < 3; ++a) yb[a] = Qb[a];
    return;
  }
  // Q = yn n + mu yn t/|t|
  const float it = 1.0f / ts;
  const float th[3] = {t[0] * it, t[1] * it, t[2] * it};
  const float qt = dot3f(Qb, th);
  const float k = mu * yn * it;
  float g[3];
  for (int a = 0; a < 3; ++a) g[a] = k * (Qb[a] - qt * th[a]);
  const float acoef = dot3f(Qb, n) + mu * qt - dot3f(g, n);
  for (int a = 0; a < 3; ++a) {
    yb[a] = g[a] + acoef * n[a];
    nb[a] += yn * (Qb[a] - g[a]) + acoef * y[a];
  }
}

// One reverse sweep: from wbar_in (adjoint of iterate l) to wbar_out (adjoint of
// iterate l-1).  Recomputes y of sweep l from the recorded impulses P^(l-1) and
// iterate w^(l-1).  Also accumulates wbar_in into the adjoint of w0.
__global__ __launch_bounds__(kBlock) void k_pja_adj(
    int n, int K, const float4* __restrict__ x, const float4* __restrict__ v,
    const float4* __restrict__ w_prev, const float4* __restrict__ wbar_in, float4* __restrict__ wbar_out,
    float4* __restrict__ w0bar, const int32_t* __restrict__ ncon, const int32_t* __restrict__ partner,
    const float* __restrict__ Psi, const float* __restrict__ Ppx, const float* __restrict__ Ppy,
    const float* __restrict__ Ppz, AdjSlots A, const DevBody* __restrict__ bodies, float alpha_dt, float mu,
    float relax, int first_sweep, const int32_t* __restrict__ pofs) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int pbase = pofs[i];
  const float4 xi = x[i];
  const float4 vi = v[i];
  const float4 wi = w_prev[i];
  const float4 bi = wbar_in[i];
  float acc[3] = {0.f, 0.f, 0.f};
  const int c = ncon[i];
  for (int k = 0; k < c; ++k) {
    const int slot = ell_slot(i, k, K);
    const int q = pbase + k;   // compact index of the recorded impulse and adjoint state
    const int code = partner[slot];
    const float psi = Psi[slot];
    float P[3] = {0.f, 0.f, 0.f};
    if (!first_sweep) {
      P[0] = Ppx[q]; P[1] = Ppy[q]; P[2] = Ppz[q];
    }
    float nrm[3], u[3], mt, Pb[3];
    const float carry[3] = {A.cx[q], A.cy[q], A.cz[q]};
    bool lo = true, body = code < 0;
    if (!body) {
      const int j = code & (kHiFlag - 1);
      lo = (code & kHiFlag) == 0;
      const float4 xj = x[j];
      const float4 wj = w_prev[j];
      const float4 bj = wbar_in[j];
      const float imj = v[j].w;
      const float4 xl = lo ? xi : xj, xh = lo ? xj : xi;
      const float4 wl = lo ? wi : wj, wh = lo ? wj : wi;
      const float4 bl = lo ? bi : bj, bh = lo ? bj : bi;
      const float iml = lo ? vi.w : imj, imh = lo ? imj : vi.w;
      const float d0 = xl.x - xh.x, d1 = xl.y - xh.y, d2 = xl.z - xh.z;
      const float L = sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
      if (L > 0.0f) {
        const float il = 1.0f / L;
        nrm[0] = d0 * il; nrm[1] = d1 * il; nrm[2] = d2 * il;
      } else {
        nrm[0] = 0.f; nrm[1] = 0.f; nrm[2] = 1.f;
      }
      u[0] = wl.x - wh.x; u[1] = wl.y - wh.y; u[2] = wl.z - wh.z;
      mt = 1.0f / (wl.w + wh.w);
      Pb[0] = carry[0] + iml * bl.x - imh * bh.x;
      Pb[1] = carry[1] + iml * bl.y - imh * bh.y;
      Pb[2] = carry[2] + iml * bl.z - imh * bh.z;
    } else {
      float V[3];
      body_geometry(bodies[-1 - code], xi, psi, nrm, V);
      u[0] = wi.x - V[0]; u[1] = wi.y - V[1]; u[2] = wi.z - V[2];
      mt = 1.0f / wi.w;
      Pb[0] = carry[0] + vi.w * bi.x;
      Pb[1] = carry[1] + vi.w * bi.y;
      Pb[2] = carry[2] + vi.w * bi.z;
    }
    const float bias = alpha_dt * psi;
    float y[3];
    for (int a = 0; a < 3; ++a) y[a] = P[a] - mt * (u[a] + bias * nrm[a]);
    const float Qb[3] = {relax * Pb[0], relax * Pb[1], relax * Pb[2]};
    float yb[3], nb[3] = {0.f, 0.f, 0.f};
    proj_adjoint(y, nrm, mu, Qb, yb, nb);
    const float keep = 1.0f - relax;
    A.cx[q] = yb[0] + keep * Pb[0];
    A.cy[q] = yb[1] + keep * Pb[1];
    A.cz[q] = yb[2] + keep * Pb[2];
    const float ub[3] = {-mt * yb[0], -mt * yb[1], -mt * yb[2]};
    const float bb = -mt * dot3f(yb, nrm);
    A.nx[q] += nb[0] - mt * bias * yb[0];
    A.ny[q] += nb[1] - mt * bias * yb[1];
    A.nz[q] += nb[2] - mt * bias * yb[2];
    A.ps[q] += alpha_dt * bb;
    if (body) {
      A.vx[q] -= ub[0]; A.vy[q] -= ub[1]; A.vz[q] -= ub[2];
    }
    const float sg = lo ? 1.0f : -1.0f;
    acc[0] += sg * ub[0]; acc[1] += sg * ub[1]; acc[2] += sg * ub[2];
  }
  wbar_out[i] = make_float4(acc[0], acc[1], acc[2], 0.0f);
  float4 z = w0bar[i];
  z.x += bi.x; z.y += bi.y; z.z += bi.z;
  w0bar[i] = z;
}

// Start of the reverse of one step: xbar^k = xbar^{k+1} (positions pass through),
// wbar^(I) = vbar^{k+1} + dt xbar^{k+1}; clears the per-particle w0 adjoint.
__global__ __launch_bounds__(kBlock) void k_adj_begin(int n, const float4* __restrict__ xbar_next,
                                                      const float4* __restrict__ vbar_next, float dt,
                                                      float4* __restrict__ xbar, float4* __restrict__ wbar,
                                                      float4* __restrict__ w0bar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 a = xbar_next[i], b = vbar_next[i];
  xbar[i] = a;
  wbar[i] = make_float4(b.x + dt * a.x, b.y + dt * a.y, b.z + dt * a.z, 0.f);
  w0bar[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ __launch_bounds__(kBlock) void k_zero_f(size_t m, float* __restrict__ a) {
  const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < m) a[e] = 0.0f;
}

// vbar^k = adjoint of w0 (w0 = v + dt g), including the last reverse sweep's output.
__global__ __launch_bounds__(kBlock) void k_adj_vbar(int n, const float4* __restrict__ w0bar,
                                                     const float4* __restrict__ wbar0, float4* __restrict__ vbar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float4 a = w0bar[i], b = wbar0[i];
  vbar[i] = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, 0.f);
}

// Body-frame SDF Hessian applied to a vector (symmetric), at the point where
// the unit gradient g was evaluated (Sec. II-C primitives).
__device__ __forceinline__ void sdf_hess_apply(const DevBody& B, const float p[3], const float g[3],
                                               const float in[3], float out[3]) {
  out[0] = out[1] = out[2] = 0.0f;
  if (B.shape == 1) {
    float q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = fabsf(p[c]) - B.params[c];
      m[c] = fmaxf(q[c], 0.0f);
      outside = outside || (q[c] > 0.0f);
    }
    if (!outside) return;
    const float L = sqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    // H = S P_A (I - mh mh^T) P_A S / L,  mh = m / L, S = diag(sign p)
    float s[3], w[3];
    for (int c = 0; c < 3; ++c) {
      s[c] = p[c] < 0.0f ? -1.0f : 1.0f;
      w[c] = q[c] > 0.0f ? s[c] * in[c] : 0.0f;
    }
    const float mh[3] = {m[0] / L, m[1] / L, m[2] / L};
    const float d = mh[0] * w[0] + mh[1] * w[1] + mh[2] * w[2];
    for (int c = 0; c < 3; ++c) out[c] = q[c] > 0.0f ? s[c] * (w[c] - d * mh[c]) / L : 0.0f;
  } else if (B.shape == 2) {
    const float h = B.params[1];
    const float cz = fminf(fmaxf(p[2], -h), h);
    const float e[3] = {p[0], p[1], p[2] - cz};
    const float L = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(L > 0.0f)) return;
    const float dz = (p[2] > -h && p[2] < h) ? 0.0f : 1.0f;
    // H = D (I - g g^T) D / L, D = diag(1, 1, dz)
    const float w[3] = {in[0], in[1], dz * in[2]};
    const float gw = g[0] * w[0] + g[1] * w[1] + g[2] * w[2];
    out[0] = (w[0] - gw * g[0]) / L;
    out[1] = (w[1] - gw * g[1]) / L;
    out[2] = dz * (w[2] - gw * g[2]) / L;
  }
}

// Unit body-frame SDF gradient and value (same branches as the forward).
__device__ __forceinline__ float sdf_grad(const DevBody& B, const float p[3], float g[3]) {
  if (B.shape == 0) {
    g[0] = 0.f; g[1] = 0.f; g[2] = 1.f;
    return p[2];
  }
  if (B.shape == 1) {
    float q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = fabsf(p[c]) - B.params[c];
      m[c] = fmaxf(q[c], 0.0f);
      outside = outside || (q[c] > 0.0f);
    }
    if (outside) {
      const float L = sqrtf(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int c = 0; c < 3; ++c) g[c] = (p[c] < 0.0f ? -1.0f : 1.0f) * m[c] / L;
      return L;
    }
    int a = 0;
    if (q[1] > q[a]) a = 1;
    if (q[2] > q[a]) a = 2;
    g[0] = g[1] = g[2] = 0.f;
    g[a] = p[a] < 0.0f ? -1.0f : 1.0f;
    return q[a];
  }
  const float h = B.params[1];
  const float cz = fminf(fmaxf(p[2], -h), h);
  const float e[3] = {p[0], p[1], p[2] - cz};
  const float L = sqrtf(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (L > 0.0f) {
    for (int c = 0; c < 3; ++c) g[c] = e[c] / L;
  } else {
    g[0] = 1.f; g[1] = 0.f; g[2] = 0.f;
  }
  return L - B.params[0];
}

// Geometry adjoint of one step: positions from the accumulated normal / gap /
// body-velocity adjoints of every half contact; body pose and twist adjoints
// reduced per workgroup and body (LDS tree, fixed order) into
// part[block][body][18] = (nu, omega, R row-major, t).
__global__ __launch_bounds__(kBlock) void k_geom_adj(int n, int K, const float4* __restrict__ x,
                                                     const int32_t* __restrict__ ncon,
                                                     const int32_t* __restrict__ partner,
                                                     const float* __restrict__ Psi, AdjSlots A,
                                                     const DevBody* __restrict__ bodies, int n_bodies,
                                                     const int32_t* __restrict__ pofs, float4* __restrict__ xbar,
                                                     float* __restrict__ part) {
  __shared__ float red[kBlock];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  float4 xi = make_float4(0.f, 0.f, 0.f, 0.f);
  int c = 0;
  float xb[3] = {0.f, 0.f, 0.f};
  if (active) {
    xi = x[i];
    c = ncon[i];
    for (int k = 0; k < c; ++k) {
      const int slot = ell_slot(i, k, K);
      const int code = partner[slot];
      if (code < 0) continue;
      const int j = code & (kHiFlag - 1);
      const bool lo = (code & kHiFlag) == 0;
      const float4 xj = x[j];
      const float4 xl = lo ? xi : xj, xh = lo ? xj : xi;
      const float d[3] = {xl.x - xh.x, xl.y - xh.y, xl.z - xh.z};
      const float L = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (!(L > 0.0f)) continue;
      const float nr[3] = {d[0] / L, d[1] / L, d[2] / L};
      const int q = pofs[i] + k;
      const float nb[3] = {A.nx[q], A.ny[q], A.nz[q]};
      const float psb = A.ps[q];
      const float nn = dot3f(nr, nb);
      const float sg = lo ? 1.0f : -1.0f;
      for (int a = 0; a < 3; ++a) xb[a] += sg * ((nb[a] - nn * nr[a]) / L + psb * nr[a]);
    }
  }
  // body contacts: one pass per body so the block reduction has a fixed order
  for (int b = 0; b < n_bodies; ++b) {
    float acc[18];
    for (int q = 0; q < 18; ++q) acc[q] = 0.f;
    const DevBody& B = bodies[b];
    if (active) {
      for (int k = 0; k < c; ++k) {
        const int slot = ell_slot(i, k, K);
        if (partner[slot] != -1 - b) continue;
        float pnt[3];
        {
          const float dd[3] = {xi.x - B.t[0], xi.y - B.t[1], xi.z - B.t[2]};
          for (int cc = 0; cc < 3; ++cc) pnt[cc] = B.R[cc] * dd[0] + B.R[3 + cc] * dd[1] + B.R[6 + cc] * dd[2];
        }
        float g[3];
        sdf_grad(B, pnt, g);
        float nr[3];
        for (int r = 0; r < 3; ++r) nr[r] = B.R[3 * r] * g[0] + B.R[3 * r + 1] * g[1] + B.R[3 * r + 2] * g[2];
        const float psi = Psi[slot];
        const float f = psi + xi.w;
        const float a[3] = {xi.x - f * nr[0] - B.t[0], xi.y - f * nr[1] - B.t[1], xi.z - f * nr[2] - B.t[2]};
        const int qq = pofs[i] + k;
        const float Vb[3] = {A.vx[qq], A.vy[qq], A.vz[qq]};
        const float nb[3] = {A.nx[qq], A.ny[qq], A.nz[qq]};
        const float psb = A.ps[qq];
        // V = nu + om x a
        acc[0] += Vb[0]; acc[1] += Vb[1]; acc[2] += Vb[2];
        acc[3] += a[1] * Vb[2] - a[2] * Vb[1];
        acc[4] += a[2] * Vb[0] - a[0] * Vb[2];
        acc[5] += a[0] * Vb[1] - a[1] * Vb[0];
        const float om[3] = {B.om[0], B.om[1], B.om[2]};
        const float ab[3] = {Vb[1] * om[2] - Vb[2] * om[1], Vb[2] * om[0] - Vb[0] * om[2],
                             Vb[0] * om[1] - Vb[1] * om[0]};
        // a = pc - t, pc = x - f n
        float tb[3] = {-ab[0], -ab[1], -ab[2]};
        for (int q = 0; q < 3; ++q) xb[q] += ab[q];
        const float fb = psb - dot3f(nr, ab);
        float ntot[3];
        for (int q = 0; q < 3; ++q) ntot[q] = nb[q] - f * ab[q];
        // n = R g
        float Rb[9];
        float gb[3];
        for (int q = 0; q < 3; ++q) gb[q] = B.R[q] * ntot[0] + B.R[3 + q] * ntot[1] + B.R[6 + q] * ntot[2];
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) Rb[3 * r + q] = ntot[r] * g[q];
        // g = grad F(p), f = F(p)
        float pb[3];
        sdf_hess_apply(B, pnt, g, gb, pb);
        for (int q = 0; q < 3; ++q) pb[q] += fb * g[q];
        // p = R^T (x - t)
        float Rp[3];
        for (int r = 0; r < 3; ++r) Rp[r] = B.R[3 * r] * pb[0] + B.R[3 * r + 1] * pb[1] + B.R[3 * r + 2] * pb[2];
        const float dd[3] = {xi.x - B.t[0], xi.y - B.t[1], xi.z - B.t[2]};
        for (int q = 0; q < 3; ++q) {
          xb[q] += Rp[q];
          tb[q] -= Rp[q];
        }
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) Rb[3 * r + q] += dd[r] * pb[q];
        for (int q = 0; q < 9; ++q) acc[6 + q] += Rb[q];
        for (int q = 0; q < 3; ++q) acc[15 + q] += tb[q];
      }
    }
    for (int q = 0; q < 18; ++q) {
      red[threadIdx.x] = acc[q];
      __syncthreads();
      for (int st = kBlock / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((size_t)blockIdx.x * n_bodies + b) * 18 + q] = red[0];
      __syncthreads();
    }
  }
  if (active) {
    float4 z = xbar[i];
    z.x += xb[0]; z.y += xb[1]; z.z += xb[2];
    xbar[i] = z;
  }
}

// out[b][q] = sum over blocks of part[block][b][q], fixed order (one block per
// (body, component)).
__global__ __launch_bounds__(kBlock) void k_body_reduce(int nblocks, int n_bodies, const float* __restrict__ part,
                                                        float* __restrict__ out) {
  __shared__ float red[kBlock];
  const int bq = blockIdx.x;  // b * 18 + q
  const int b = bq / 18, q = bq % 18;
  float s = 0.f;
  for (int k = threadIdx.x; k < nblocks; k += kBlock) s += part[((size_t)k * n_bodies + b) * 18 + q];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = kBlock / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[bq] = red[0];
}

// caller order <-> internal order for adjoint vectors
__global__ void k_gather3(int n, const int32_t* __restrict__ orig, const float* __restrict__ in3,
                          float4* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = orig[k];
  out[k] = in3 ? make_float4(in3[3 * o], in3[3 * o + 1], in3[3 * o + 2], 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace ggk
