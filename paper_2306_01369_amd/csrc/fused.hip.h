// One step's detection, projected-Jacobi sweeps and position update in a
// single cooperative launch: the "fused" ordering of the paper's kernel-order
// ablation (Sec. II-D: collision detection and contact impulses split into two
// loops but kept in one kernel), set against the production path, which
// splits them across kernel launches (the ordering the paper found fastest).
//
// Under the symmetric Jacobi reading every sweep reads every iterate of the
// previous sweep, so the phases inside the kernel are separated by grid-wide
// barriers (cooperative groups; the launch must be cooperative, i.e. the whole
// grid resident at once).  The cell keys and the bucket sort stay separate
// launches.  The same device functions run on the same data in the same
// order per particle as in the split path, so results agree with it up to the
// compiler's choice of where to fuse a multiply and an add (binary32: to
// rounding; the binary64 build agrees bit for bit).
//
// Hang safety: every thread of the grid reaches every barrier -- work is
// skipped on an error, barriers never are -- and a launch that is not
// cooperative is detected before the first barrier and fails the step.
#pragma once
#include <hip/hip_cooperative_groups.h>
#include "kernels.hip.h"

namespace ggk {

template <typename R>
struct FusedArgs {
  int n, K;
  V4<R>* x;
  V4<R>* v;
  const int32_t* orig;
  float inv_c;
  int n_blk;
  EnvTables env;
  const int32_t* start;
  const int32_t* sidx;
  const V4<R>* xs;
  const int32_t* os;
  const int32_t* item_start;
  const int32_t* n_items;
  const DevBody* bodies;
  int n_bodies;
  int mass_split, max_cells, max_stage, iters;
  R gx, gy, gz, dt, alpha_dt, mu, relax, zlo, zspan;
  int32_t* ncon;
  int32_t* partner;
  R* Psi;
  V4<R>* wa;   // iterate after detection and after even sweeps
  V4<R>* wb;   // after odd sweeps
  R* Px;
  R* Py;
  R* Pz;
  V4<R>* dv;
  R* imass;
  Ctl* ctl;
  DetPart* part;   // per-workgroup detection counts (summed by k_detect_stats)
  int step;
  int pair_gaps;   // store pair gaps (recorded forward)
};

template <typename R, int TB>
__global__ __launch_bounds__(TB) __attribute__((amdgpu_waves_per_eu(5))) void k_step_fused(FusedArgs<R> a) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  if (!grid.is_valid()) {  // the same for every thread: no barrier is reached
    if (blockIdx.x == 0 && threadIdx.x == 0) set_error(a.ctl, 3 /* GG_ERR_HIP */, a.step);
    return;
  }
  const int blk = xcd_block(), nblk = gridDim.x;
  // phase 1: detection (skipped after an earlier failure of this call; the
  // error word is read once per workgroup, as detection has workgroup barriers)
  __shared__ int err0;
  if (threadIdx.x == 0) err0 = __hip_atomic_load(&a.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  if (err0 == 0)
    detect_items<R, TB>(a.n, a.K, a.x, a.v, a.orig, a.inv_c, a.n_blk, a.env, a.start, a.sidx, a.xs, a.os,
                        a.item_start, a.n_items, a.bodies, a.n_bodies, a.gx, a.gy, a.gz, a.dt, a.mass_split,
                        a.max_cells, a.max_stage, a.ncon, a.partner, a.Psi, a.wa, a.imass, a.ctl, a.part, a.step,
                        blk, nblk, false, a.pair_gaps != 0);
  grid.sync();
  // nothing writes the error word after detection: every thread reads the same value
  const bool run = __hip_atomic_load(&a.ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  // phase 2: the sweeps
  for (int it = 0; it < a.iters; ++it) {
    const int mode = (it == 0 ? 1 : 0) | (it == a.iters - 1 ? 2 : 0);
    const V4<R>* w_in = (it & 1) ? a.wb : a.wa;
    V4<R>* w_out = (it & 1) ? a.wa : a.wb;
    if (run)
      for (int base = blk * TB; base < a.n; base += nblk * TB) {
        const int i = base + (int)threadIdx.x;
        if (i < a.n)
          pja_particle<R>(i, a.K, a.x, a.v, w_in, w_out, a.ncon, a.partner, a.Psi, a.Px, a.Py, a.Pz, a.Px, a.Py,
                          a.Pz, a.bodies, a.gx, a.gy, a.gz, a.dt, a.alpha_dt, a.mu, a.relax, mode, a.dv, nullptr,
                          a.imass);
      }
    grid.sync();
  }
  // phase 3: positions (every read of x by the last sweep is behind the barrier)
  if (run) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.ctl->steps_done, 1);
    for (int base = blk * TB; base < a.n; base += nblk * TB) {
      const int i = base + (int)threadIdx.x;
      if (i < a.n) integrate_particle<R>(i, a.x, a.v, a.dt, a.zlo, a.zspan);
    }
  }
}

}  // namespace ggk
