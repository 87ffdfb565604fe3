/*
 * gg.h -- C ABI of the MI355X granular contact step.
 *
 * One timestep of the method of "GranularGym: High Performance Simulation for
 * Robotic Tasks with Granular Materials" (arXiv 2306.01369), Sec. II:
 *   1. cell coordinates kappa_i = round(x_i / c) and the spatial hash of Eq. (6)
 *      h_i = XOR_a p_a (kappa_ia - q)  mod n_h;
 *   2. a table of particles per hash bucket (the role of the linked hashmap of
 *      Alg. 2, built here by a counting sort instead of compare-and-swap);
 *   3. particle-particle contacts from the particle's own cell and its 26
 *      neighbour cells, ||x_i - x_j||^2 <= (r_i + r_j)^2 (Sec. II-B, II-C);
 *   4. particle-body contacts psi = f_G(X^{-1} x) - r <= 0 through closed-form
 *      signed distance functions (Eq. (7), Sec. II-C);
 *   5. projected Jacobi sweeps over the stored contacts (Alg. 1) for the contact
 *      NCP of Eqs. (1)-(3) with the Baumgarte term alpha*psi/dt;
 *   6. symplectic Euler: velocities first, then positions (Eqs. (4)-(5)).
 *
 * Conventions shared by every call
 *   - All calls return a gg_status and never throw.  Argument checks run on the
 *     host before any device work; a failed HIP call leaves the handle in a
 *     sticky failed state (every later call returns GG_ERR_HIP).
 *   - gg_error_detail() returns a message for the last failure on this thread.
 *   - gg_mem says where a caller buffer lives: GG_MEM_HOST (pageable or pinned
 *     host memory) or GG_MEM_DEVICE (device memory on params.device).
 *   - The library copies every input into buffers it owns and copies outputs
 *     into caller memory; it never keeps or frees a caller pointer.
 *   - Work is enqueued on params.stream (a hipStream_t; NULL makes the library
 *     create its own non-blocking stream).  Calls return after the work they
 *     enqueued has finished.
 *   - Arrays of 3-vectors are dense row-major (n x 3, float32).
 *   - Units are SI (m, s, kg).
 */
#ifndef GG_H
#define GG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gg_sim gg_sim; /* opaque; owns every device buffer of one simulation */

typedef enum {
  GG_OK = 0,
  GG_ERR_INVALID = 1,     /* bad argument; nothing was changed */
  GG_ERR_OOM = 2,         /* device or host allocation failed */
  GG_ERR_HIP = 3,         /* a HIP runtime call failed; the handle is unusable */
  GG_ERR_CAPACITY = 4,    /* a particle exceeded its contact capacity; see gg_step */
  GG_ERR_NONFINITE = 5,   /* non-finite or out-of-range position/velocity */
  GG_ERR_NO_TAPE = 6,     /* gg_step_backward without a recorded forward */
  GG_ERR_UNSUPPORTED = 7  /* valid request that this build does not implement */
} gg_status;

typedef enum { GG_PLANE = 0, GG_BOX = 1, GG_CAPSULE = 2, GG_GRID = 3 } gg_shape;
typedef enum { GG_MEM_HOST = 0, GG_MEM_DEVICE = 1 } gg_mem;

/* A kinematic rigid body (Sec. II: bodies are driven by time and receive no
 * reaction).  Shapes are the closed-form SDF primitives of Sec. II-C:
 *   GG_PLANE:   f(p) = p_z (the half space below the body-frame xy plane is solid)
 *   GG_BOX:     half extents params[0..2]
 *   GG_CAPSULE: radius params[0] around the body-frame segment
 *               (0,0,-params[1]) .. (0,0,+params[1])
 *   GG_GRID:    SDF samples on a regular grid, trilinearly interpolated (the
 *               pre-computed SDF of Sec. II-C for arbitrary geometry):
 *               params[0] = index of a grid registered with gg_set_grids
 * pose = row-major [R | t] (3 x 4) mapping body to world, x_w = R p + t.
 * twist = (nu, omega): velocity of the body origin and angular velocity, both
 * in the world frame.  The pose given is the pose at the start of the next
 * step; poses are advanced by the library after every step,
 * t += dt nu, R = Exp(dt [omega]x) R, in double precision. */
typedef struct {
  int32_t env;       /* environment the body acts in (0 .. n_envs-1) */
  int32_t shape;     /* gg_shape */
  float params[4];
  float pose[12];
  float twist[6];
} gg_body;

/* A regular grid of SDF samples in a body's frame (Sec. II-C).  Knot (a, b, c),
 * 0 <= a < nx, 0 <= b < ny, 0 <= c < nz, sits at the body-frame point
 * origin + (a, b, c) / inv_spacing and holds values[offset + (c*ny + b)*nx + a].
 * The SDF at a body-frame point p is the trilinear interpolant of the knots:
 * per axis u = (p - origin) * inv_spacing, cell i = min(floor(u), n - 2),
 * t = u - i; lerps a + t (b - a) along x, then y, then z.  Points with u
 * outside [0, n - 1] on any axis are outside the geometry (no contact): the
 * grid must contain the geometry with a margin of at least the largest
 * particle radius.  The contact decision evaluates the interpolant in
 * binary32 in that order without fused multiply-add; gaps and normals use the
 * build's precision, the normal being the rotated interpolant gradient,
 * normalised. */
typedef struct {
  int32_t nx, ny, nz;    /* knots per axis, each >= 2 */
  float origin[3];       /* body-frame position of knot (0, 0, 0) */
  float inv_spacing;     /* 1 / knot spacing (> 0) */
  int64_t offset;        /* first value of this grid in the values array */
} gg_grid;

/* Flags for gg_params.flags */
#define GG_FLAG_PROFILE 1u     /* time detection and projected-Jacobi phases with HIP events */
#define GG_FLAG_DIAGNOSTICS 2u /* keep the last step's velocity change (GG_FIELD_DV) */
#define GG_FLAG_TAPE 4u        /* differentiable: keep checkpoints of every gg_step call for
                                  gg_step_backward (one environment only) */
#define GG_FLAG_GRAPH 8u       /* replay gg_step's launch sequence from a captured HIP graph:
                                  the first call with a given step count, re-sort phase and
                                  state-buffer parity captures it (the 64 most recently used
                                  captures are kept), later ones replay it; results are
                                  bitwise those of direct launches.  Ignored with
                                  GG_FLAG_PROFILE or GG_FLAG_TAPE. */

#define GG_FLAG_FUSED 16u       /* run each step's detection, projected-Jacobi sweeps and position
                                  update as one cooperative kernel launch with grid-wide
                                  barriers between the phases (the fused kernel order of the
                                  Sec. II-D ablation; the split launches are the default).
                                  Results equal the split launches' to rounding (the
                                  compiler may fuse multiply-adds differently; contact
                                  decisions are unaffected).  Not with
                                  GG_FLAG_TAPE; GG_FLAG_GRAPH is ignored; with
                                  GG_FLAG_PROFILE the detection is timed in ms_pja.  Needs a
                                  device with cooperative launches (else GG_ERR_UNSUPPORTED). */

/* Simulation parameters.  Zero selects the stated default. */
typedef struct {
  float dt;          /* timestep (> 0) */
  float alpha;       /* Baumgarte factor, Sec. II-A (>= 0) */
  float mu;          /* Coulomb friction coefficient, Eq. (3) (>= 0) */
  float gravity[3];  /* external acceleration (F_ext / m) */
  int32_t n_iters;   /* projected-Jacobi sweeps per step, Alg. 1 (>= 1) */
  float cell_size;   /* hash cell edge c; 0 -> 2 r_max (1 + 2^-10); must be >= 2 r_max */
  int64_t hash_size; /* buckets n_h per environment of Eq. (6) (the reported cell index);
                        0 -> 2 x (particles of the env), the heuristic of Sec. II-B.  The
                        internal table follows it, with at least 4 buckets per particle in
                        a single environment of 2^18 or more particles */
  float relax;       /* over-relaxation of the impulse update, 0 -> 1 */
  int32_t mass_split;/* 1: per-contact mass m/n_i (mass splitting); 0: plain masses */
  int32_t checkpoint_every;          /* backward pass: steps per checkpoint (0 -> 10) */
  int32_t max_contacts_per_particle; /* contact capacity per particle (<= 256); 0 ->
                        automatic: min(packing bound, 24 + bodies of the largest
                        environment) at first, grown on demand up to the packing
                        bound of the radius ratio (19 for equal spheres) + those
                        bodies; see gg_step */
  int32_t precision; /* 0: binary32 state and arithmetic; 1: binary64 state and arithmetic
                        (a check build: contact decisions stay the binary32 predicates on
                        the state rounded to binary32; inputs and outputs stay float) */
  float density;     /* grain density for m = rho 4/3 pi r^3; 0 -> 2500 */
  uint32_t flags;    /* GG_FLAG_* */
  int32_t reorder_every;  /* steps between re-sorts of the internal particle order along a
                             Z-order curve, each node's particles by descending contact
                             count (memory locality only; results do not depend on it);
                             0 -> 32 below 2^19 particles, else 16 (4 when the
                             largest radius exceeds 1.25x the smallest); < 0 -> never */
  int32_t tile_max_cells; /* detection tile limit in cells (item box + halo); 0 -> from the
                             node size (box + one-cell halo + one cell of drift) */
  int32_t tile_max_stage; /* detection tile limit in staged particles; 0 -> from the cells
                             and the particles per cell */
  int32_t tile_node_shift;/* detection work items follow Z-order nodes of 2^shift cells
                             (6 = 4x4x4), at most tile_threads particles each; 0 -> the
                             largest node whose particles (at the initial particles per
                             occupied cell) fit one workgroup */
  int32_t tile_threads;   /* detection workgroup size and work-item length: 64, 128 or
                             256; 0 -> 256 from 2^18 particles, else 128.
                             The tile parameters change speed only, never results. */
  float cyclic_z[2]; /* (z_lo, z_hi): when z_hi > z_lo, a particle whose updated position
                        falls below z_lo is moved up by z_hi - z_lo, velocity unchanged (the
                        cyclic vertical boundary of the paper's gear-tower benchmark, Sec. III-B);
                        contact search does not wrap.  (0, 0): off */
  int32_t pja_lanes; /* lanes per particle in a projected-Jacobi sweep: 1, 2 or 4 (each lane
                        takes every L-th contact; the sum keeps list order, so results do not
                        depend on it); 0 -> from the particle count */
  int32_t device;    /* HIP device ordinal */
  void* stream;      /* hipStream_t or NULL */
} gg_params;

/* Create a simulation of n particles split into n_envs independent
 * environments.  The state is the problem statement of Sec. II: positions and
 * velocities of n spheres (3 x n each, no rotational degrees of freedom) with
 * radii; the environments are the independent simulations run side by side
 * in Sec. III.  Particles env_offsets[e] .. env_offsets[e+1]-1 form
 * environment e (env_offsets: n_envs+1 host int64 values, first 0, last n,
 * non-decreasing; NULL means one environment).  Particles of different
 * environments never touch.  x, v: n x 3; radius: n (> 0).  where applies to
 * x, v and radius.  n may be 0.  On success *out owns a new handle.
 * Errors: GG_ERR_INVALID (bad params, offsets, radius <= 0, cell smaller than
 * 2 r_max, |x / c| >= 2^30, a contact table of more than 2^31 - 1 slots:
 * n rounded up to a multiple of 64, times the contact capacity -- the
 * explicit max_contacts_per_particle, or the automatic capacity's starting
 * value),
 * GG_ERR_NONFINITE (non-finite x or v), GG_ERR_OOM, GG_ERR_HIP. */
gg_status gg_create(const gg_params* params, int32_t n_envs, const int64_t* env_offsets, int64_t n,
                    const float* x, const float* v, const float* radius, gg_mem where, gg_sim** out);

/* Replace all bodies (n_bodies >= 0): the kinematic bodies of Sec. II, whose
 * pose in SE(3) and twist in se(3) the caller prescribes and which receive no
 * reaction; they enter the step through their SDFs (Eq. (7), Sec. II-C).
 * Each body's env must be < n_envs.  The contact capacity grows by the bodies
 * of the largest environment (see gg_create).  A successful call discards the
 * record of the last differentiable gg_step (gg_step_backward then returns
 * GG_ERR_NO_TAPE until the next gg_step).
 * Errors: GG_ERR_INVALID (unknown shape, bad env, non-positive extents,
 * non-finite pose or twist, a contact table beyond 2^31 - 1 slots; nothing is
 * changed), GG_ERR_OOM, GG_ERR_HIP. */
gg_status gg_set_bodies(gg_sim* sim, int32_t n_bodies, const gg_body* bodies, gg_mem where);

/* Register the grids that GG_GRID bodies refer to by index, replacing any
 * registered before.  grids: n_grids descriptors (host memory); values:
 * n_values floats in host or device memory (where), copied.  Each grid must
 * lie inside the values array and every value must be finite; otherwise
 * GG_ERR_INVALID and nothing changes.  gg_set_bodies checks grid indices
 * against the grids registered at that time.  A successful call discards the
 * record of the last differentiable gg_step, like gg_set_bodies. */
gg_status gg_set_grids(gg_sim* sim, int32_t n_grids, const gg_grid* grids, int64_t n_values,
                       const float* values, gg_mem where);

/* Advance n_steps timesteps (>= 0), each the step of Sec. II: cell keys and
 * the bucket table (Eq. (6), Alg. 2's role), particle-particle and
 * particle-body contact detection (Sec. II-B, II-C, Eq. (7)), n_iters
 * projected-Jacobi sweeps (Alg. 1, Eqs. (1)-(3)) and the symplectic-Euler
 * update (Eqs. (4)-(5)); then the bodies' poses advance by their twists.
 * twists: NULL keeps every body's current
 * twist, else n_steps x n_bodies x 6 floats, the twist of each body during
 * each step (where applies to twists).
 * Capacity: if a particle has more contacts than its capacity (see
 * GG_FIELD_STATS), the step is abandoned before any impulse is applied.  With
 * the automatic capacity (max_contacts_per_particle 0) the capacity then grows
 * -- to twice its value or the count found, at most the packing bound -- and
 * the call goes on from that step (a differentiable call starts again from its
 * first step, restored from its first checkpoint); contact lists do not depend
 * on the capacity, so neither does any result.  With an explicit capacity, or
 * past the bound, the state stays that of the start of that step, later steps
 * of the call are not run, and GG_ERR_CAPACITY is returned; GG_FIELD_STATS
 * reports the steps completed.  GG_ERR_NONFINITE likewise if a position leaves the hashable
 * range or becomes non-finite. */
gg_status gg_step(gg_sim* sim, int32_t n_steps, const float* twists, gg_mem where);

/* Reverse-mode gradient of the last gg_step call, for a simulation created
 * with GG_FLAG_TAPE and one environment.  This differentiates the discrete
 * step of Eqs. (2)-(5) and Alg. 1 (the impulse sweeps, the contact gaps and
 * normals of Eq. (1) and the body SDFs, the rigid-body pose update and the
 * symplectic-Euler integration) with each step's contact set held fixed, the
 * set being piecewise constant in the inputs.  The forward kept (x, v) every
 * params.checkpoint_every steps; each segment is recomputed from its
 * checkpoint before its steps are reversed, so device memory grows with
 * n_steps / checkpoint_every and one segment's recorded sweeps (12 bytes per
 * half contact per sweep, and the segment's contact tables), plus a per-call
 * workspace of 12 bytes per contact-table slot (n rounded up to 64 times the
 * contact capacity) and 28 bytes per half contact, allocated and freed by
 * each call.
 * dL_dx, dL_dv: n x 3 float32 gradients of the loss with respect to the final
 * positions and velocities, caller's particle order; NULL means zero.
 * Outputs (any may be NULL): dL_dx0, dL_dv0 (n x 3) with respect to the
 * positions and velocities at the start of the call, and dL_dtwists
 * (n_steps x n_bodies x 6, same layout as gg_step's twists) with respect to
 * each body's twist in each step.  where applies to all six arrays.
 * Errors: GG_ERR_NO_TAPE if the simulation has no tape or the last gg_step
 * failed; GG_ERR_UNSUPPORTED for more than one environment; GG_ERR_OOM if the
 * workspace cannot be allocated; GG_ERR_HIP if the recomputed contact counts
 * differ from the recorded forward.  The tape stays valid until the next
 * gg_step, gg_set_bodies or gg_set_grids call, so the call may be repeated
 * with other loss gradients. */
gg_status gg_step_backward(gg_sim* sim, const float* dL_dx, const float* dL_dv, float* dL_dx0,
                           float* dL_dv0, float* dL_dtwists, gg_mem where);

/* Fields for gg_read */
enum {
  GG_FIELD_POS = 0,        /* n x 3 float32, caller's particle order */
  GG_FIELD_VEL = 1,        /* n x 3 float32 */
  GG_FIELD_CELL_INDEX = 2, /* n int64: bucket of each particle at the last detection
                              (env bucket offset + Eq. (6) value) */
  GG_FIELD_CONTACTS = 3,   /* C x 2 int32: particle pairs (i < j) sorted by (i, j), then
                              particle-body pairs (i, body) sorted by (i, body) */
  GG_FIELD_IMPULSES = 4,   /* C x 3 float32: world-frame impulse R_c lam_c on the first
                              member of each contact, same order as GG_FIELD_CONTACTS */
  GG_FIELD_STATS = 5,      /* one gg_stats */
  GG_FIELD_DV = 6,         /* n x 3 float32: velocity change by impulses in the last
                              step (needs GG_FLAG_DIAGNOSTICS) */
  GG_FIELD_RADIUS = 7,     /* n float32 */
  GG_FIELD_BODY_POSES = 8  /* n_bodies x 12 float32: each body's pose at the start of the next
                              step, row-major [R | t] (body -> world), in gg_set_bodies order,
                              as the library advanced it (double, rounded once) */
};

typedef struct {
  int64_t steps_done;     /* steps completed by the last gg_step call */
  int64_t steps_total;    /* steps completed since creation */
  int64_t n_pp;           /* particle-particle contacts at the last detection */
  int64_t n_pb;           /* particle-body contacts at the last detection */
  int64_t candidates;     /* ordered candidate pairs tested at the last detection */
  int64_t max_contacts;   /* largest contact count of one particle at the last detection
                             (also when that detection overflowed the capacity) */
  int64_t capacity;       /* contact capacity per particle */
  int64_t last_status;    /* gg_status of the last gg_step call */
  int64_t n;              /* particles */
  int64_t n_buckets;      /* buckets of the internal cell table over all environments (per
                             environment hash_size, or 4 per particle in a single environment
                             of 2^18 or more particles if that is larger, rounded up to a
                             multiple of 64) */
  double ms_detect;       /* profiled: cell keys + sort + detection, summed over the last call */
  double ms_pja;          /* profiled: projected-Jacobi sweeps, summed */
  double ms_integrate;    /* profiled: position update (with the summing of the step's
                             detection statistics), summed */
  int64_t pja_launches;   /* profiled: projected-Jacobi launches timed */
  int64_t contacts_summed;/* contacts (pairs + body) summed over the steps of the last call */
  int64_t detect_fallback;/* detection work items (up to tile_threads particles each) that queried
                             cells one particle at a time instead of through an LDS tile, last
                             detection */
  int64_t detect_items;   /* detection work items */
  int64_t device_bytes_peak; /* largest device memory in use (whole device, hipMemGetInfo)
                                seen after this simulation's allocations, backward included */
  int32_t tile_threads;   /* detection launch shape in use (defaults resolved) */
  int32_t tile_node_shift;
  int32_t tile_max_cells;
  int32_t tile_max_stage;
  int32_t detect_workgroups; /* detection grid: workgroups resident at once on the device */
  int32_t reorder_every;
  int32_t pja_lanes;      /* lanes per particle of the sweeps (default resolved) */
  int32_t detect_queues;  /* 1: detection work items are taken from per-XCD work queues;
                             0 (GG_FLAG_FUSED): each detection workgroup takes a fixed
                             contiguous share */
} gg_stats;

/* Copy a field into dst (where says where dst lives).  If dst is NULL only
 * *written is set, to the number of bytes the field needs.  Otherwise
 * capacity_bytes must be at least that size (else GG_ERR_INVALID) and
 * *written receives the bytes copied.  Contacts and impulses describe the last
 * completed detection and projected-Jacobi solve. */
gg_status gg_read(gg_sim* sim, int32_t field, void* dst, int64_t capacity_bytes, int64_t* written,
                  gg_mem where);

/* ---- Observations of the Gym-style environment (Sec. III-A, "Bulldozing"):
 * depth images computed on the simulating device and the goal-box reward. */
typedef enum { GG_CAM_ORTHO = 0, GG_CAM_PERSPECTIVE = 1 } gg_camera_kind;

/* A depth camera.  pose = row-major [R | t] (3 x 4) mapping camera to world;
 * the camera looks along its +z axis, image columns run along +x, rows along
 * +y.  Pixel (u, v) has the binary32 centre coordinates
 * g_u = (u + 1/2) * fl32(2 / width) - 1 and g_v likewise (in [-1, 1]).
 *   GG_CAM_ORTHO:       the pixel's ray starts at camera-frame point
 *                       (params[0] g_u, params[1] g_v, 0) and runs along +z
 *                       (params[0], params[1]: half width and half height, m);
 *   GG_CAM_PERSPECTIVE: it starts at the camera origin and runs along
 *                       (params[0] g_u, params[1] g_v, 1) (the tangents of the
 *                       half angles of view).
 * A pixel's depth is the camera-frame z of the first surface its ray meets,
 * at most params[2] (far), and far when it meets none.  Drawn: the particles
 * of environment `env` (spheres) and its GG_PLANE bodies at their current
 * pose (a plane is met where the ray enters its solid side); other bodies
 * are not drawn.  Whether a ray meets a sphere is decided in binary32 without
 * fused multiply-add (camera-frame centre c = R^T (x - t) summed as the SDF
 * transform; orthographic: c_z > 0 and (o_x - c_x)^2 + (o_y - c_y)^2 <= r^2;
 * perspective: c_z > 0, E = |c|^2 - r^2 > 0 -- a sphere holding the camera is
 * skipped --, D = d.c > 0 and |d|^2 E <= D^2); depths are computed in double
 * from those binary32 values and rounded once.  Images are deterministic. */
typedef struct {
  int32_t env;            /* environment drawn (0 .. n_envs-1) */
  int32_t kind;           /* gg_camera_kind */
  int32_t width, height;  /* pixels, 1 .. 8192 each */
  float pose[12];
  float params[4];        /* p0, p1, far (each finite and > 0), unused */
} gg_camera;

/* Render n_cams (0 .. 65535) cameras of the current state into dst: the
 * cameras' images one after another, each height x width row-major
 * (pixel (u, v) at v * width + u), binary32.  capacity_bytes must be at least
 * 4 x the total pixel count.  cams is host memory; dst is host or device
 * memory as `where` says.  The state is not changed.  Returns after the images
 * are written.  Errors: GG_ERR_INVALID (bad camera, env, size or capacity;
 * nothing written), GG_ERR_OOM, GG_ERR_HIP. */
gg_status gg_render_depth(gg_sim* sim, int32_t n_cams, const gg_camera* cams, float* dst,
                          int64_t capacity_bytes, gg_mem where);

/* Goal-box reward per environment (Sec. III-A): 100 / n_e for every particle of
 * environment e inside the closed box [lo, hi] (binary32 comparisons of the
 * binary32 positions), and -d / n_e for every other, d = its distance to the
 * nearest point of the box (double).  boxes: host, n_envs x 6 (lo xyz, hi xyz,
 * finite, lo <= hi).  reward: n_envs doubles; inside: n_envs int64 particle
 * counts, or NULL; both host or device memory as `where` says.  An empty
 * environment scores 0.  Sums run in a fixed order (bitwise reproducible).
 * Errors: GG_ERR_INVALID, GG_ERR_OOM, GG_ERR_HIP. */
gg_status gg_goal_reward(gg_sim* sim, const float* boxes, double* reward, int64_t* inside, gg_mem where);

/* gg_goal_reward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, checks, kernels and results (bit for bit) as
 * gg_goal_reward, with no hipMalloc, hipFree or other allocation.  The
 * per-call workspace (a partial sum per chunk of at most 4096 particles of one
 * environment, the staged boxes and, for host outputs, the staged results)
 * lives in a 2 MiB device array of the library, one copy per GPU, held until
 * the process ends.  It needs 12 bytes per chunk and 40 bytes per environment,
 * each of its five regions rounded up to 256 bytes; a simulation beyond that
 * (about 170,000 chunks, or 50,000 environments) is rejected with
 * GG_ERR_INVALID before any device work.  Every call on a GPU shares that
 * array: calls that overlap on one GPU (from several host threads, or on
 * streams not ordered with each other) race.  Returns after the results are
 * written.  Errors: as gg_goal_reward, GG_ERR_INVALID also for a simulation
 * beyond the workspace. */
gg_status gg_goal_reward_noalloc(gg_sim* sim, const float* boxes, double* reward, int64_t* inside,
                                 gg_mem where);

/* Release every resource of the handle (NULL is ignored). */
void gg_destroy(gg_sim* sim);

/* Static description of a status code. */
const char* gg_status_string(gg_status status);

/* Message for the last failure on the calling thread ("" if none). */
const char* gg_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* GG_H */
