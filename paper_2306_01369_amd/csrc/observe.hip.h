// Observations of the Gym-style environment (arXiv 2306.01369, Sec. III-A,
// "Bulldozing"): depth images from cameras, computed on the device that holds
// the particles, and the goal-box reward.
//
// Camera model.  A camera has a pose [R | t] (camera -> world) and looks along
// its +z axis.  Pixel (u, v) of a W x H image has the binary32 centre
// coordinate g_u = fl(fl(u + 1/2) * su) - 1 with su = fl32(2 / W) (likewise
// g_v).  Orthographic: the pixel's ray starts at (p0 g_u, p1 g_v, 0) and runs
// along (0, 0, 1).  Perspective: it starts at the origin and runs along
// (p0 g_u, p1 g_v, 1).  Its depth is the camera-frame z of the first surface
// met (the ray parameter along those directions), at most `far`.  Surfaces:
// the particles of the camera's environment and its plane bodies.
//
// Whether a ray meets a sphere is decided in binary32, each operation rounded
// as written (camera-frame centre c = R^T (x - t) summed as the SDF transform
// is; orthographic: c_z > 0 and (o_x - c_x)^2 + (o_y - c_y)^2 <= r^2;
// perspective: c_z > 0, E = |c|^2 - r^2 > 0, D = d.c > 0, |d|^2 E <= D^2);
// the depth of a hit is computed in double from those binary32 values and
// rounded once to binary32.  A pixel keeps the smallest depth: positive
// binary32 values order like their bit patterns, so an unsigned atomicMin on
// the bits takes the minimum in any arrival order and the image is
// deterministic.
//
// Work decomposition.  k_depth_planes writes every pixel (far, or the nearest
// plane); k_depth_spheres then runs one thread per (camera, particle): the
// particle's footprint on the image -- the pixels whose rays can meet the
// sphere, from the extent of x/z and y/z over the ball (perspective) or of
// x, y (orthographic), widened by one pixel -- is tested pixel by pixel.
#pragma once
#include "kernels.hip.h"

namespace ggk {

struct DevCamera {
  int32_t kind, width, height, pad0;
  float R[9], t[3];       // camera -> world
  float p0, p1, far;      // half extents (orthographic) or tangents of the half angles
  float su, sv;           // fl32(2 / width), fl32(2 / height)
  int32_t i0, i1;         // particles of the environment (internal index range)
  int32_t q0, q1;         // its planes in the plane list
  int64_t base;           // first pixel of this camera in the output
};

struct DevPlane {         // a plane body: solid below the plane through t, normal n
  float n[3], t[3];
};

__device__ __forceinline__ float pixel_centre(int idx, float s) {
#pragma clang fp contract(off)
  const float a = (float)idx + 0.5f;
  const float b = a * s;
  return b - 1.0f;
}

// Pixel depths from the camera's planes (far where none is met).
__global__ __launch_bounds__(kBlock) void k_depth_planes(const DevCamera* __restrict__ cams,
                                                         const DevPlane* __restrict__ planes,
                                                         float* __restrict__ out) {
#pragma clang fp contract(off)
  const DevCamera& C = cams[blockIdx.y];
  const int npx = C.width * C.height;
  for (int p = blockIdx.x * kBlock + threadIdx.x; p < npx; p += gridDim.x * kBlock) {
    const int u = p % C.width, v = p / C.width;
    const float a = C.p0 * pixel_centre(u, C.su), b = C.p1 * pixel_centre(v, C.sv);
    double o[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 1.0};
    if (C.kind == 0) {
      o[0] = a; o[1] = b;
    } else {
      d[0] = a; d[1] = b;
    }
    double ow[3], dw[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double r0 = C.R[3 * k], r1 = C.R[3 * k + 1], r2 = C.R[3 * k + 2];
      ow[k] = (double)C.t[k] + (r0 * o[0] + r1 * o[1] + r2 * o[2]);
      dw[k] = r0 * d[0] + r1 * d[1] + r2 * d[2];
    }
    double best = C.far;
    for (int q = C.q0; q < C.q1; ++q) {
      const DevPlane& P = planes[q];
      const double n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
      const double den = n0 * dw[0] + n1 * dw[1] + n2 * dw[2];
      if (!(den < 0.0)) continue;
      const double num = n0 * ((double)P.t[0] - ow[0]) + n1 * ((double)P.t[1] - ow[1]) + n2 * ((double)P.t[2] - ow[2]);
      const double tau = num / den;
      if (tau >= 0.0) best = fmin(best, tau);
    }
    out[C.base + p] = (float)best;
  }
}

// Pixel index range whose centres can lie in [lo, hi] of the normalised
// coordinate g = (idx + 1/2) s - 1, widened by one pixel, clipped to the image.
__device__ __forceinline__ void pixel_range(double glo, double ghi, float s, int size, int& i0, int& i1) {
  const double a = (glo + 1.0) / (double)s - 0.5, b = (ghi + 1.0) / (double)s - 0.5;
  // (a NaN bound gives the whole axis; every index stays in [0, size - 1])
  i0 = a >= -1.0 ? (a <= (double)size ? max(0, (int)floor(a) - 1) : size) : 0;
  i1 = b <= (double)size ? (b >= -1.0 ? min(size - 1, (int)ceil(b) + 1) : -1) : size - 1;
}

// Extent of x/z over a disk of radius r centred at (cx, cz), cz > 0, as
// [tan(theta - alpha), tan(theta + alpha)]; unbounded when the disk reaches
// the plane z = 0.
__device__ __forceinline__ void slope_range(double cx, double cz, double r, double& lo, double& hi) {
  const double L = sqrt(cx * cx + cz * cz);
  if (cz <= r || L <= r) {
    lo = -1e300;
    hi = 1e300;
    return;
  }
  const double th = atan2(cx, cz), al = asin(r / L);
  const double half_pi = 1.5707963267948966;
  lo = th - al <= -half_pi ? -1e300 : tan(th - al);
  hi = th + al >= half_pi ? 1e300 : tan(th + al);
}

template <typename R>
__global__ __launch_bounds__(kBlock) void k_depth_spheres(const DevCamera* __restrict__ cams,
                                                          const V4<R>* __restrict__ x,
                                                          float* __restrict__ out) {
#pragma clang fp contract(off)
  const DevCamera& C = cams[blockIdx.y];
  const bool ortho = C.kind == 0;
  for (int i = C.i0 + blockIdx.x * kBlock + threadIdx.x; i < C.i1; i += gridDim.x * kBlock) {
    const float4 p = f32of(x[i]);
    const float d0 = p.x - C.t[0], d1 = p.y - C.t[1], d2 = p.z - C.t[2];
    float c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float s0 = C.R[0 * 3 + k] * d0;
      const float s1 = C.R[1 * 3 + k] * d1;
      const float s2 = C.R[2 * 3 + k] * d2;
      const float s = s0 + s1;
      c[k] = s + s2;
    }
    if (!(c[2] > 0.0f)) continue;
    const float r = p.w, r2 = r * r;
    int u0, u1, v0, v1;
    if (ortho) {
      pixel_range(((double)c[0] - r) / C.p0, ((double)c[0] + r) / C.p0, C.su, C.width, u0, u1);
      pixel_range(((double)c[1] - r) / C.p1, ((double)c[1] + r) / C.p1, C.sv, C.height, v0, v1);
    } else {
      double alo, ahi, blo, bhi;
      slope_range(c[0], c[2], r, alo, ahi);
      slope_range(c[1], c[2], r, blo, bhi);
      pixel_range(alo / C.p0, ahi / C.p0, C.su, C.width, u0, u1);
      pixel_range(blo / C.p1, bhi / C.p1, C.sv, C.height, v0, v1);
    }
    // binary32 terms that do not depend on the pixel
    const float c00 = c[0] * c[0];
    const float c11 = c[1] * c[1];
    const float c22 = c[2] * c[2];
    const float Bq = c00 + c11;
    const float B = Bq + c22;
    const float E = B - r2;
    if (!ortho && !(E > 0.0f)) continue;
    for (int v = v0; v <= v1; ++v) {
      const float b = C.p1 * pixel_centre(v, C.sv);
      for (int u = u0; u <= u1; ++u) {
        const float a = C.p0 * pixel_centre(u, C.su);
        double tau;
        if (ortho) {
          const float ex = a - c[0], ey = b - c[1];
          const float q0 = ex * ex;
          const float q1 = ey * ey;
          const float q = q0 + q1;
          if (!(q <= r2)) continue;
          const double ex6 = (double)a - (double)c[0], ey6 = (double)b - (double)c[1];
          const double h = (double)r * (double)r - (ex6 * ex6 + ey6 * ey6);
          tau = fmax((double)c[2] - sqrt(fmax(h, 0.0)), 0.0);
        } else {
          const float aa = a * a;
          const float bb = b * b;
          const float Aq = aa + bb;
          const float A = Aq + 1.0f;
          const float ac = a * c[0];
          const float bc = b * c[1];
          const float Dq = ac + bc;
          const float D = Dq + c[2];
          if (!(D > 0.0f)) continue;
          const float lhs = A * E;
          const float rhs = D * D;
          if (!(lhs <= rhs)) continue;
          const double a6 = a, b6 = b, x6 = c[0], y6 = c[1], z6 = c[2];
          const double A6 = a6 * a6 + b6 * b6 + 1.0;
          const double B6 = x6 * x6 + y6 * y6 + z6 * z6;
          const double D6 = a6 * x6 + b6 * y6 + z6;
          const double E6 = B6 - (double)r * (double)r;
          const double disc = fmax(D6 * D6 - A6 * E6, 0.0);
          tau = E6 / (D6 + sqrt(disc));
        }
        const float t32 = (float)tau;
        atomicMin((unsigned int*)(out + C.base + (int64_t)v * C.width + u), __float_as_uint(t32));
      }
    }
  }
}

// ----------------------------------------------------------- goal reward
// Per environment: 100/n_e for each particle inside the closed box [lo, hi]
// (binary32 comparisons of the binary32 positions), -d/n_e for each other
// particle, d = distance to the nearest point of the box in double.
// Pass 1: one workgroup per chunk (a run of at most kRewardChunk particles of
// one environment) sums its particles' distances and counts those inside,
// in a fixed order; pass 2: one thread per environment adds its chunks in
// order.  The result is bitwise reproducible.
constexpr int kRewardChunk = 4096;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_reward_chunks(const V4<R>* __restrict__ x,
                                                          const int32_t* __restrict__ chunk,  // (env, begin, end)
                                                          const float* __restrict__ boxes,
                                                          double* __restrict__ part_d,
                                                          int32_t* __restrict__ part_n) {
  __shared__ double sd[kBlock];
  __shared__ int sn[kBlock];
  const int e = chunk[3 * blockIdx.x], b = chunk[3 * blockIdx.x + 1], end = chunk[3 * blockIdx.x + 2];
  const float* lo = boxes + 6 * e;
  const float* hi = lo + 3;
  double dsum = 0.0;
  int cnt = 0;
  for (int i = b + threadIdx.x; i < end; i += kBlock) {
    const float4 p = f32of(x[i]);
    const float q[3] = {p.x, p.y, p.z};
    bool in = true;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      in = in && lo[k] <= q[k] && q[k] <= hi[k];
      const double w = fmin(fmax((double)q[k], (double)lo[k]), (double)hi[k]);
      const double g = (double)q[k] - w;
      s += g * g;
    }
    if (in)
      ++cnt;
    else
      dsum += sqrt(s);
  }
  sd[threadIdx.x] = dsum;
  sn[threadIdx.x] = cnt;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      sd[threadIdx.x] += sd[threadIdx.x + h];
      sn[threadIdx.x] += sn[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part_d[blockIdx.x] = sd[0];
    part_n[blockIdx.x] = sn[0];
  }
}

__global__ void k_reward_envs(int n_envs, const int32_t* __restrict__ env_chunk,  // n_envs + 1 chunk offsets
                              const int32_t* __restrict__ env_count, const double* __restrict__ part_d,
                              const int32_t* __restrict__ part_n, double* __restrict__ reward,
                              int64_t* __restrict__ inside) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_envs) return;
  double d = 0.0;
  long long cnt = 0;
  for (int k = env_chunk[e]; k < env_chunk[e + 1]; ++k) {
    d += part_d[k];
    cnt += part_n[k];
  }
  const int ne = env_count[e];
  reward[e] = ne > 0 ? (100.0 * (double)cnt - d) / (double)ne : 0.0;
  if (inside) inside[e] = cnt;
}

}  // namespace ggk
