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
// Recorded impulses are indexed compactly from pofs, the prefix sum of the
// contact counts, as the forward sweep of the same lane count wrote them
// (jagged rows per wavefront with one lane per particle, rec_row; pofs[i] + k
// with several).  Per half contact the adjoint keeps a carry (the
// adjoint of the impulse of the previous sweep, identical bits in both halves
// of a pair, as the forward's impulse copies), read and written in every
// reverse sweep and indexed like the contact table (slot-major per 64
// particles), so that a wavefront's loads of it are whole rows.  The geometry
// of a pair (normal and gap, functions of the two positions) enters linearly
// in the adjoints of its normal and gap, so every reverse sweep adds its share
// of a pair's position adjoint straight into the particle's xbar; only body
// contacts accumulate the adjoints of their normal, gap and body point
// velocity over the sweeps (compact index), for the body pose and twist
// adjoints.  Per particle the adjoint keeps the adjoint of the iterate, whose
// w component carries the particle's inverse mass.  Like the forward, every
// particle gathers its own half contacts: no atomics, deterministic results.
#pragma once
#include "kernels.hip.h"

namespace ggk {

template <typename R>
struct AdjSlots {     // per half-contact adjoint state (SoA)
  R *cx, *cy, *cz;    // carry: adjoint of the impulse of the previous sweep (contact-table slot)
  // body contacts only, compact index pofs[i] + k:
  R *nx, *ny, *nz;    // accumulated adjoint of the contact normal
  R *ps;              // accumulated adjoint of the gap psi
  R *vx, *vy, *vz;    // accumulated adjoint of the body point velocity V
};

template <typename R>
__device__ __forceinline__ R dot3f(const R a[3], const R b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Adjoint of the projection Q = proj(y, n) of the forward sweep, given Qbar.
// Returns ybar and adds the normal's share to nbar.
template <typename R>
__device__ __forceinline__ void proj_adjoint(const R y[3], const R n[3], R mu, const R Qb[3],
                                             R yb[3], R nb[3]) {
  const R yn = dot3f(n, y);
  R t[3] = {y[0] - yn * n[0], y[1] - yn * n[1], y[2] - yn * n[2]};
  const R ynp = fmax(yn, R(0));
  const R ts = sqrt(dot3f(t, t));
  const bool scaled = ts > mu * ynp;
  if (yn <= R(0)) {
    // Q = 0, and so on a neighbourhood (the normal part stays clamped): also
    // where the tangential part is exactly zero and the strict test does not
    // scale it, the derivative is zero
    yb[0] = yb[1] = yb[2] = R(0);
    return;
  }
  if (!scaled) {
    if (mu * ynp > R(0)) {  // Q = y (inside the friction disk)
      for (int a = 0; a < 3; ++a) yb[a] = Qb[a];
      return;
    }
    // no friction and y_t exactly zero: Q = (n.y) n, the tangential part is
    // dropped on a neighbourhood too, so only the normal part has a derivative
    const R qn = dot3f(Qb, n);
    for (int a = 0; a < 3; ++a) {
      yb[a] = qn * n[a];
      nb[a] += qn * y[a] + yn * Qb[a];
    }
    return;
  }
  // Q = yn n + mu yn t/|t|
  const R it = R(1) / ts;
  const R th[3] = {t[0] * it, t[1] * it, t[2] * it};
  const R qt = dot3f(Qb, th);
  const R k = mu * yn * it;
  R g[3];
  for (int a = 0; a < 3; ++a) g[a] = k * (Qb[a] - qt * th[a]);
  const R acoef = dot3f(Qb, n) + mu * qt - dot3f(g, n);
  for (int a = 0; a < 3; ++a) {
    yb[a] = g[a] + acoef * n[a];
    nb[a] += yn * (Qb[a] - g[a]) + acoef * y[a];
  }
}

// One half contact of a reverse sweep: recomputes y of sweep l for contact
// `code` of particle i from the recorded impulse P^(l-1) (compact index q) and
// iterate w^(l-1) (recorded impulse at index qp, body accumulators at the
// per-particle compact index q), updates the contact's carry (at its contact-table slot, so
// that a wavefront's k-th contacts are one row) and returns ub (the adjoint of
// its velocity residual) with the sign sg it takes in i's sum, and xg, this
// sweep's share of a pair's adjoint of x_i through its normal n = d / |d| and
// gap psi = |d| - r_i - r_j (d = x_lo - x_hi): sg ((nbar - (nbar.n) n) / |d| +
// psibar n).  A body contact instead adds its shares to the accumulators at q.
// Multiply-adds are fused only within an expression (fp contract on), so every
// kernel that calls it computes the same bits.
template <typename R>
__device__ __forceinline__ void half_contact_adj(int code, int slot, int qp, int q, bool first_sweep, bool fresh,
                                                 const V4<R>& xi,
                                                 const V4<R>& vi, const V4<R>& wi, const V4<R>& bi,
                                                 const V4<R>* __restrict__ x, const V4<R>* __restrict__ v,
                                                 const V4<R>* __restrict__ w_prev,
                                                 const V4<R>* __restrict__ wbar_in, const R* __restrict__ Psi,
                                                 const R* __restrict__ Ppx, const R* __restrict__ Ppy,
                                                 const R* __restrict__ Ppz, AdjSlots<R>& A,
                                                 const DevBody* __restrict__ bodies, R alpha_dt, R mu, R relax,
                                                 R ub[3], R& sg, R xg[3]) {
#pragma clang fp contract(on)
  const R psi = Psi[slot];
  R P[3] = {R(0), R(0), R(0)};
  if (!first_sweep) {
    P[0] = Ppx[qp]; P[1] = Ppy[qp]; P[2] = Ppz[qp];
  }
  R nrm[3], u[3], mt, Pb[3], il = R(0);
  // (fresh: the first reverse sweep of a step, whose state starts at zero)
  const R carry[3] = {fresh ? R(0) : A.cx[slot], fresh ? R(0) : A.cy[slot], fresh ? R(0) : A.cz[slot]};
  bool lo = true, body = code < 0;
  if (!body) {
    const int j = code & (kHiFlag - 1);
    lo = (code & kHiFlag) == 0;
    const V4<R> xj = x[j];
    const V4<R> wj = w_prev[j];
    const V4<R> bj = wbar_in[j];
    const R imj = bj.w;
    const V4<R> xl = lo ? xi : xj, xh = lo ? xj : xi;
    const V4<R> wl = lo ? wi : wj, wh = lo ? wj : wi;
    const V4<R> bl = lo ? bi : bj, bh = lo ? bj : bi;
    const R iml = lo ? vi.w : imj, imh = lo ? imj : vi.w;
    const R d0 = xl.x - xh.x, d1 = xl.y - xh.y, d2 = xl.z - xh.z;
    const R L = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (L > R(0)) {
      il = R(1) / L;
      nrm[0] = d0 * il; nrm[1] = d1 * il; nrm[2] = d2 * il;
    } else {
      nrm[0] = R(0); nrm[1] = R(0); nrm[2] = R(1);
    }
    u[0] = wl.x - wh.x; u[1] = wl.y - wh.y; u[2] = wl.z - wh.z;
    mt = R(1) / (wl.w + wh.w);
    Pb[0] = carry[0] + iml * bl.x - imh * bh.x;
    Pb[1] = carry[1] + iml * bl.y - imh * bh.y;
    Pb[2] = carry[2] + iml * bl.z - imh * bh.z;
  } else {
    R V[3];
    body_geometry<R>(bodies[-1 - code], xi, psi, nrm, V);
    u[0] = wi.x - V[0]; u[1] = wi.y - V[1]; u[2] = wi.z - V[2];
    mt = R(1) / wi.w;
    Pb[0] = carry[0] + vi.w * bi.x;
    Pb[1] = carry[1] + vi.w * bi.y;
    Pb[2] = carry[2] + vi.w * bi.z;
  }
  const R bias = alpha_dt * psi;
  R y[3];
  for (int a = 0; a < 3; ++a) y[a] = P[a] - mt * (u[a] + bias * nrm[a]);
  const R Qb[3] = {relax * Pb[0], relax * Pb[1], relax * Pb[2]};
  R yb[3], nb[3] = {R(0), R(0), R(0)};
  proj_adjoint(y, nrm, mu, Qb, yb, nb);
  const R keep = R(1) - relax;
  A.cx[slot] = yb[0] + keep * Pb[0];
  A.cy[slot] = yb[1] + keep * Pb[1];
  A.cz[slot] = yb[2] + keep * Pb[2];
  ub[0] = -mt * yb[0]; ub[1] = -mt * yb[1]; ub[2] = -mt * yb[2];
  const R bb = -mt * dot3f(yb, nrm);
  const R ns[3] = {nb[0] - mt * bias * yb[0], nb[1] - mt * bias * yb[1], nb[2] - mt * bias * yb[2]};
  const R pss = alpha_dt * bb;
  sg = lo ? R(1) : R(-1);
  xg[0] = xg[1] = xg[2] = R(0);
  if (body) {
    A.nx[q] = (fresh ? R(0) : A.nx[q]) + ns[0];
    A.ny[q] = (fresh ? R(0) : A.ny[q]) + ns[1];
    A.nz[q] = (fresh ? R(0) : A.nz[q]) + ns[2];
    A.ps[q] = (fresh ? R(0) : A.ps[q]) + pss;
    A.vx[q] = (fresh ? R(0) : A.vx[q]) - ub[0];
    A.vy[q] = (fresh ? R(0) : A.vy[q]) - ub[1];
    A.vz[q] = (fresh ? R(0) : A.vz[q]) - ub[2];
  } else if (il > R(0)) {
    const R nn = dot3f(nrm, ns);
    for (int a = 0; a < 3; ++a) xg[a] = sg * ((ns[a] - nn * nrm[a]) * il + pss * nrm[a]);
  }
}

// One reverse sweep: from wbar_in (adjoint of iterate l) to wbar_out (adjoint of
// iterate l-1).  Recomputes y of sweep l from the recorded impulses P^(l-1) and
// iterate w^(l-1).  Also accumulates wbar_in into the adjoint of w0 and the
// sweep's pair geometry shares into xbar.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_pja_adj(
    int n, int K, const V4<R>* __restrict__ x, const V4<R>* __restrict__ v,
    const V4<R>* __restrict__ w_prev, const V4<R>* __restrict__ wbar_in, V4<R>* __restrict__ wbar_out,
    V4<R>* __restrict__ w0bar, const int32_t* __restrict__ ncon, const int32_t* __restrict__ partner,
    const R* __restrict__ Psi, const R* __restrict__ Ppx, const R* __restrict__ Ppy,
    const R* __restrict__ Ppz, AdjSlots<R> A, const DevBody* __restrict__ bodies, R alpha_dt, R mu,
    R relax, int first_sweep, int fresh, const int32_t* __restrict__ pofs, V4<R>* __restrict__ xbar) {
#pragma clang fp contract(on)
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int pbase = pofs[i];
  const V4<R> xi = x[i];
  const V4<R> vi = v[i];
  const V4<R> wi = w_prev[i];
  const V4<R> bi = wbar_in[i];
  R acc[3] = {R(0), R(0), R(0)}, gx[3] = {R(0), R(0), R(0)};
  const int c = ncon[i];
  int rbase = pofs[i & ~63];
  for (int k = 0; k < c; ++k) {
    const int slot = ell_slot(i, k, K);
    R ub[3], sg, xg[3];
    const int qp = rec_row(rbase);
    half_contact_adj<R>(partner[slot], slot, qp, pbase + k, first_sweep != 0, fresh != 0, xi, vi, wi, bi, x, v, w_prev, wbar_in,
                        Psi, Ppx, Ppy, Ppz, A, bodies, alpha_dt, mu, relax, ub, sg, xg);
    acc[0] += sg * ub[0]; acc[1] += sg * ub[1]; acc[2] += sg * ub[2];
    gx[0] += xg[0]; gx[1] += xg[1]; gx[2] += xg[2];
  }
  wbar_out[i] = mk4<R>(acc[0], acc[1], acc[2], vi.w);
  V4<R> z = w0bar[i];
  z.x += bi.x; z.y += bi.y; z.z += bi.z;
  w0bar[i] = z;
  V4<R> g = xbar[i];
  g.x += gx[0]; g.y += gx[1]; g.z += gx[2];
  xbar[i] = g;
}

// The same reverse sweep with L lanes per particle (L = 2 or 4): lane s takes
// contacts s, s + L, ...; the sum over contacts keeps list order (cross-lane
// shuffles after every round), so results are bitwise those of k_pja_adj.
template <typename R, int L>
__global__ __launch_bounds__(kBlock) void k_pja_adj_lanes(
    int n, int K, const V4<R>* __restrict__ x, const V4<R>* __restrict__ v,
    const V4<R>* __restrict__ w_prev, const V4<R>* __restrict__ wbar_in, V4<R>* __restrict__ wbar_out,
    V4<R>* __restrict__ w0bar, const int32_t* __restrict__ ncon, const int32_t* __restrict__ partner,
    const R* __restrict__ Psi, const R* __restrict__ Ppx, const R* __restrict__ Ppy,
    const R* __restrict__ Ppz, AdjSlots<R> A, const DevBody* __restrict__ bodies, R alpha_dt, R mu,
    R relax, int first_sweep, int fresh, const int32_t* __restrict__ pofs, V4<R>* __restrict__ xbar) {
#pragma clang fp contract(on)
  static_assert(L == 2 || L == 4, "lanes per particle");
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int i = t / L, sub = t % L;
  if (i >= n) return;  // (the L lanes of a particle leave together)
  const int pbase = pofs[i];
  const V4<R> xi = x[i];
  const V4<R> vi = v[i];
  const V4<R> wi = w_prev[i];
  const V4<R> bi = wbar_in[i];
  R acc[3] = {R(0), R(0), R(0)}, gx[3] = {R(0), R(0), R(0)};
  const int c = ncon[i];
  for (int m = 0; m * L < c; ++m) {
    const int k = m * L + sub;
    R ub[3] = {R(0), R(0), R(0)}, sg = R(0), xg[3] = {R(0), R(0), R(0)};
    if (k < c) {
      const int slot = ell_slot(i, k, K);
      half_contact_adj<R>(partner[slot], slot, pbase + k, pbase + k, first_sweep != 0, fresh != 0, xi, vi, wi, bi, x,
                          v, w_prev, wbar_in, Psi, Ppx, Ppy, Ppz, A, bodies, alpha_dt, mu, relax, ub, sg, xg);
    }
#pragma unroll
    for (int qq = 0; qq < L; ++qq) {
      const R g = __shfl(sg, qq, L), u0 = __shfl(ub[0], qq, L), u1 = __shfl(ub[1], qq, L),
              u2 = __shfl(ub[2], qq, L);
      const R e0 = __shfl(xg[0], qq, L), e1 = __shfl(xg[1], qq, L), e2 = __shfl(xg[2], qq, L);
      if (m * L + qq < c) {
        acc[0] += g * u0; acc[1] += g * u1; acc[2] += g * u2;
        gx[0] += e0; gx[1] += e1; gx[2] += e2;
      }
    }
  }
  if (sub == 0) {
    wbar_out[i] = mk4<R>(acc[0], acc[1], acc[2], vi.w);
    V4<R> z = w0bar[i];
    z.x += bi.x; z.y += bi.y; z.z += bi.z;
    w0bar[i] = z;
    V4<R> g = xbar[i];
    g.x += gx[0]; g.y += gx[1]; g.z += gx[2];
    xbar[i] = g;
  }
}

// Start of the reverse of one step: xbar^k = xbar^{k+1} (positions pass through),
// wbar^(I) = vbar^{k+1} + dt xbar^{k+1} (w: the inverse mass, v.w); clears the
// per-particle w0 adjoint.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_begin(int n, const V4<R>* __restrict__ xbar_next,
                                                      const V4<R>* __restrict__ vbar_next,
                                                      const V4<R>* __restrict__ v, R dt,
                                                      V4<R>* __restrict__ xbar, V4<R>* __restrict__ wbar,
                                                      V4<R>* __restrict__ w0bar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const V4<R> a = xbar_next[i], b = vbar_next[i];
  xbar[i] = a;
  wbar[i] = mk4<R>(b.x + dt * a.x, b.y + dt * a.y, b.z + dt * a.z, v[i].w);
  w0bar[i] = mk4<R>(R(0), R(0), R(0), R(0));
}


// vbar^k = adjoint of w0 (w0 = v + dt g), including the last reverse sweep's output.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_adj_vbar(int n, const V4<R>* __restrict__ w0bar,
                                                     const V4<R>* __restrict__ wbar0, V4<R>* __restrict__ vbar) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const V4<R> a = w0bar[i], b = wbar0[i];
  vbar[i] = mk4<R>(a.x + b.x, a.y + b.y, a.z + b.z, R(0));
}

// Body-frame SDF Hessian applied to a vector (symmetric), at the point where
// the unit gradient g was evaluated (Sec. II-C primitives).
template <typename R>
__device__ __forceinline__ void sdf_hess_apply(const DevBody& B, const R p[3], const R g[3],
                                               const R in[3], R out[3]) {
  out[0] = out[1] = out[2] = R(0);
  if (B.shape == 1) {
    R q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = fabs(p[c]) - B.params[c];
      m[c] = fmax(q[c], R(0));
      outside = outside || (q[c] > R(0));
    }
    if (!outside) return;
    const R L = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    // H = S P_A (I - mh mh^T) P_A S / L,  mh = m / L, S = diag(sign p)
    R s[3], w[3];
    for (int c = 0; c < 3; ++c) {
      s[c] = p[c] < R(0) ? R(-1) : R(1);
      w[c] = q[c] > R(0) ? s[c] * in[c] : R(0);
    }
    const R mh[3] = {m[0] / L, m[1] / L, m[2] / L};
    const R d = mh[0] * w[0] + mh[1] * w[1] + mh[2] * w[2];
    for (int c = 0; c < 3; ++c) out[c] = q[c] > R(0) ? s[c] * (w[c] - d * mh[c]) / L : R(0);
  } else if (B.shape == 2) {
    const R h = B.params[1];
    const R cz = fmin(fmax(p[2], -h), h);
    const R e[3] = {p[0], p[1], p[2] - cz};
    const R L = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    if (!(L > R(0))) return;
    const R dz = (p[2] > -h && p[2] < h) ? R(0) : R(1);
    // H = D (I - g g^T) D / L, D = diag(1, 1, dz)
    const R w[3] = {in[0], in[1], dz * in[2]};
    const R gw = g[0] * w[0] + g[1] * w[1] + g[2] * w[2];
    out[0] = (w[0] - gw * g[0]) / L;
    out[1] = (w[1] - gw * g[1]) / L;
    out[2] = dz * (w[2] - gw * g[2]) / L;
  }
}

// Hessian of a grid body's trilinear interpolant (with respect to the
// body-frame point) applied to w: zero on the diagonal inside a cell, the
// mixed second differences lerped along the third axis off it, times
// inv_spacing^2.
template <typename R>
__device__ __forceinline__ void grid_hess_apply(const DevBody& B, const R p[3], const R w[3], R out[3]) {
  R t[3];
  int i[3];
  for (int a = 0; a < 3; ++a) {
    R u = (p[a] - (R)B.go[a]) * (R)B.gih;
    u = fmin(fmax(u, R(0)), (R)(B.gn[a] - 1));
    const int k = min((int)floor(u), B.gn[a] - 2);
    i[a] = k;
    t[a] = u - (R)k;
  }
  const long long sy = B.gn[0], sz = (long long)B.gn[0] * B.gn[1];
  const float* v = B.gv + ((long long)i[2] * sz + (long long)i[1] * sy + i[0]);
  const R v000 = v[0], v100 = v[1], v010 = v[sy], v110 = v[sy + 1];
  const R v001 = v[sz], v101 = v[sz + 1], v011 = v[sz + sy], v111 = v[sz + sy + 1];
  const R Dz0 = v110 - v010 - v100 + v000, Dz1 = v111 - v011 - v101 + v001;   // d2f/dt0 dt1 at z0, z1
  const R Ey0 = v101 - v001 - v100 + v000, Ey1 = v111 - v011 - v110 + v010;   // d2f/dt0 dt2 at y0, y1
  const R Fx0 = v011 - v001 - v010 + v000, Fx1 = v111 - v101 - v110 + v100;   // d2f/dt1 dt2 at x0, x1
  const R ih2 = (R)B.gih * (R)B.gih;
  const R hxy = (Dz0 + t[2] * (Dz1 - Dz0)) * ih2;
  const R hxz = (Ey0 + t[1] * (Ey1 - Ey0)) * ih2;
  const R hyz = (Fx0 + t[0] * (Fx1 - Fx0)) * ih2;
  out[0] = hxy * w[1] + hxz * w[2];
  out[1] = hxy * w[0] + hyz * w[2];
  out[2] = hxz * w[0] + hyz * w[1];
}

// Unit body-frame SDF gradient and value (same branches as the forward).
template <typename R>
__device__ __forceinline__ R sdf_grad(const DevBody& B, const R p[3], R g[3]) {
  if (B.shape == 0) {
    g[0] = R(0); g[1] = R(0); g[2] = R(1);
    return p[2];
  }
  if (B.shape == 1) {
    R q[3], m[3];
    bool outside = false;
    for (int c = 0; c < 3; ++c) {
      q[c] = fabs(p[c]) - B.params[c];
      m[c] = fmax(q[c], R(0));
      outside = outside || (q[c] > R(0));
    }
    if (outside) {
      const R L = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
      for (int c = 0; c < 3; ++c) g[c] = (p[c] < R(0) ? R(-1) : R(1)) * m[c] / L;
      return L;
    }
    int a = 0;
    if (q[1] > q[a]) a = 1;
    if (q[2] > q[a]) a = 2;
    g[0] = g[1] = g[2] = R(0);
    g[a] = p[a] < R(0) ? R(-1) : R(1);
    return q[a];
  }
  const R h = B.params[1];
  const R cz = fmin(fmax(p[2], -h), h);
  const R e[3] = {p[0], p[1], p[2] - cz};
  const R L = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (L > R(0)) {
    for (int c = 0; c < 3; ++c) g[c] = e[c] / L;
  } else {
    g[0] = R(1); g[1] = R(0); g[2] = R(0);
  }
  return L - B.params[0];
}

// Geometry adjoint of the body contacts of one step (the reverse sweeps have
// added the pairs' shares to xbar): positions from the accumulated normal /
// gap / body-velocity adjoints of every body contact; body pose and twist
// adjoints reduced per workgroup and body (fixed order) into
// part[block][body][18] = (nu, omega, R row-major, t).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_geom_adj(int n, int K, const V4<R>* __restrict__ x,
                                                     const int32_t* __restrict__ ncon,
                                                     const int32_t* __restrict__ partner,
                                                     const R* __restrict__ Psi, AdjSlots<R> A,
                                                     const DevBody* __restrict__ bodies, int n_bodies,
                                                     const int32_t* __restrict__ pofs, V4<R>* __restrict__ xbar,
                                                     R* __restrict__ part) {
  __shared__ R wred[kBlock / 64][18];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < n;
  V4<R> xi = mk4<R>(R(0), R(0), R(0), R(0));
  int c = 0, pbase = 0;
  R xb[3] = {R(0), R(0), R(0)};
  if (active) {
    xi = x[i];
    c = ncon[i];
    pbase = pofs[i];
  }
  // a particle's body contacts follow its pairs, in body order
  int kb = c;
  while (kb > 0 && partner[ell_slot(i, kb - 1, K)] < 0) --kb;
  // body contacts: one pass per body so the block reduction has a fixed order
  for (int b = 0; b < n_bodies; ++b) {
    R acc[18];
    for (int q = 0; q < 18; ++q) acc[q] = R(0);
    const DevBody& B = bodies[b];
    const auto* BR = PoseOf<R>::R(B);
    const auto* Bt = PoseOf<R>::t(B);
    const auto* Bom = PoseOf<R>::om(B);
    bool touched = false;
    if (active) {
      for (int k = kb; k < c; ++k) {
        const int slot = ell_slot(i, k, K);
        if (partner[slot] != -1 - b) continue;
        touched = true;
        R pnt[3];
        {
          const R dd[3] = {xi.x - Bt[0], xi.y - Bt[1], xi.z - Bt[2]};
          for (int cc = 0; cc < 3; ++cc) pnt[cc] = BR[cc] * dd[0] + BR[3 + cc] * dd[1] + BR[6 + cc] * dd[2];
        }
        R g[3], G[3], Gn = R(1);
        if (B.shape == 3) {
          // grid: the interpolant's gradient G is not unit length; the
          // normal uses G / |G|
          grid_sdf_grad<R>(B, pnt, G);
          Gn = sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
          if (Gn > R(0)) {
            for (int q = 0; q < 3; ++q) g[q] = G[q] / Gn;
          } else {
            g[0] = R(1); g[1] = R(0); g[2] = R(0);
            G[0] = G[1] = G[2] = R(0);
            Gn = R(1);
          }
        } else {
          sdf_grad(B, pnt, g);
          for (int q = 0; q < 3; ++q) G[q] = g[q];
        }
        R nr[3];
        for (int r = 0; r < 3; ++r) nr[r] = BR[3 * r] * g[0] + BR[3 * r + 1] * g[1] + BR[3 * r + 2] * g[2];
        const R psi = Psi[slot];
        const R f = psi + xi.w;
        const R a[3] = {xi.x - f * nr[0] - Bt[0], xi.y - f * nr[1] - Bt[1], xi.z - f * nr[2] - Bt[2]};
        const int q = pbase + k;
        const R Vb[3] = {A.vx[q], A.vy[q], A.vz[q]};
        const R nb[3] = {A.nx[q], A.ny[q], A.nz[q]};
        const R psb = A.ps[q];
        // V = nu + om x a
        acc[0] += Vb[0]; acc[1] += Vb[1]; acc[2] += Vb[2];
        acc[3] += a[1] * Vb[2] - a[2] * Vb[1];
        acc[4] += a[2] * Vb[0] - a[0] * Vb[2];
        acc[5] += a[0] * Vb[1] - a[1] * Vb[0];
        const R om[3] = {Bom[0], Bom[1], Bom[2]};
        const R ab[3] = {Vb[1] * om[2] - Vb[2] * om[1], Vb[2] * om[0] - Vb[0] * om[2],
                             Vb[0] * om[1] - Vb[1] * om[0]};
        // a = pc - t, pc = x - f n
        R tb[3] = {-ab[0], -ab[1], -ab[2]};
        for (int q = 0; q < 3; ++q) xb[q] += ab[q];
        const R fb = psb - dot3f(nr, ab);
        R ntot[3];
        for (int q = 0; q < 3; ++q) ntot[q] = nb[q] - f * ab[q];
        // n = R g
        R Rb[9];
        R gb[3];
        for (int q = 0; q < 3; ++q) gb[q] = BR[q] * ntot[0] + BR[3 + q] * ntot[1] + BR[6 + q] * ntot[2];
        for (int r = 0; r < 3; ++r)
          for (int q = 0; q < 3; ++q) Rb[3 * r + q] = ntot[r] * g[q];
        // g = grad F(p) / |grad F(p)|, f = F(p)
        R pb[3];
        if (B.shape == 3) {
          const R gg = dot3f(g, gb);
          R Gb[3];
          for (int q = 0; q < 3; ++q) Gb[q] = (gb[q] - gg * g[q]) / Gn;
          grid_hess_apply<R>(B, pnt, Gb, pb);
        } else {
          sdf_hess_apply(B, pnt, g, gb, pb);
        }
        for (int q = 0; q < 3; ++q) pb[q] += fb * G[q];
        // p = R^T (x - t)
        R Rp[3];
        for (int r = 0; r < 3; ++r) Rp[r] = BR[3 * r] * pb[0] + BR[3 * r + 1] * pb[1] + BR[3 * r + 2] * pb[2];
        const R dd[3] = {xi.x - Bt[0], xi.y - Bt[1], xi.z - Bt[2]};
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
    // workgroup sum in a fixed order: a butterfly within each wavefront, then
    // the wavefronts in order; a workgroup none of whose particles touches the
    // body writes zeros
    R* out = part + ((size_t)blockIdx.x * n_bodies + b) * 18;
    if (!__syncthreads_or(touched ? 1 : 0)) {
      if (threadIdx.x < 18) out[threadIdx.x] = R(0);
      continue;
    }
    for (int q = 0; q < 18; ++q)
      for (int o = 32; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, 64);
    if ((threadIdx.x & 63) == 0)
      for (int q = 0; q < 18; ++q) wred[threadIdx.x >> 6][q] = acc[q];
    __syncthreads();
    if (threadIdx.x < 18) {
      R sum = R(0);
      for (int w = 0; w < kBlock / 64; ++w) sum += wred[w][threadIdx.x];
      out[threadIdx.x] = sum;
    }
    __syncthreads();   // (wred is written again for the next body)
  }
  if (active) {
    V4<R> z = xbar[i];
    z.x += xb[0]; z.y += xb[1]; z.z += xb[2];
    xbar[i] = z;
  }
}

// out[b][q] = sum over blocks of part[block][b][q], fixed order (one block per
// (body, component)).
template <typename R>
__global__ __launch_bounds__(kBlock) void k_body_reduce(int nblocks, int n_bodies, const R* __restrict__ part,
                                                        R* __restrict__ out) {
  __shared__ R red[kBlock];
  const int bq = blockIdx.x;  // b * 18 + q
  const int b = bq / 18, q = bq % 18;
  R s = R(0);
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
template <typename R>
__global__ void k_gather3(int n, const int32_t* __restrict__ orig, const float* __restrict__ in3,
                          V4<R>* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int o = orig[k];
  out[k] = in3 ? mk4<R>((R)in3[3 * o], (R)in3[3 * o + 1], (R)in3[3 * o + 2], R(0)) : mk4<R>(R(0), R(0), R(0), R(0));
}

}  // namespace ggk
