/*
 * fastmpm.h -- C ABI of the MI355X MLS-MPM substep library (libfastmpm.so).
 *
 * The library advances particles (Gaussian centres and interior fill points
 * of FastPhysGS, arXiv 2602.01723) through the MLS-MPM substep:
 *   Kirchhoff stress of the particle's elastic model (App. A.2, App. B.1),
 *   particle-to-grid transfer with quadratic B-spline weights, APIC affine
 *   momentum and the MLS stress term (Sec. 4.2 momentum-exchange equation;
 *   App. A.1 P2G),
 *   grid update with gravity and sticky walls (App. A.1 grid update),
 *   grid-to-particle transfer of v, C, x and F (App. A.1 G2P),
 *   plastic return mapping after the stress (App. A.2, App. B.2; Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Every call returns an int status (mpm_status); 0 is success.
 *  - Argument and configuration checks run on the host, before any device
 *    work, and return MPM_EINVAL without touching device memory.
 *  - Device pointers are caller-owned (allocate them with hipMalloc or a
 *    PyTorch CUDA tensor).  The library never frees them, and allocates no
 *    device memory of its own: a context's buffers live in the workspace the
 *    caller hands to mpm_init (size from mpm_workspace_size), MCIS takes a
 *    workspace per call, and the tape of the adjoint is caller-owned too.
 *  - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *    void*; NULL = the null stream) and is asynchronous unless stated.
 *  - One context may be used by one stream at a time; calls on a context
 *    are not thread-safe.
 *  - HIP runtime failures return MPM_EDEVICE; mpm_last_error() gives text.
 *
 * Particle arrays are structure-of-arrays, float32, component-major:
 *    x[3][N], v[3][N]          (x[c*N + p] is component c of particle p)
 *    C[9][N], F[9][N]          (row-major 3x3: entry (r,c) at plane 3*r+c)
 *    mass[N], vol0[N]          (kg, m^3: m_p and the rest volume V_p^0)
 *    log_E[N], nu[N]           (natural log of Young's modulus in Pa; Poisson ratio)
 *    mat_id[N]                 (int32 index into the material table)
 * The simulation domain is [0,1)^3 with n^3 grid nodes at i*dx, dx = 1/n.
 * A batch of scenes is stored back to back: scene b owns particles
 * [offsets[b], offsets[b+1]) and its own n^3 grid.
 */
#ifndef FASTMPM_H
#define FASTMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPM_ABI_VERSION 1

typedef struct mpm_context* mpm_ctx;

typedef enum {
  MPM_OK = 0,
  MPM_EINVAL = -1,       /* bad argument or configuration (nothing was enqueued) */
  MPM_ENOMEM = -2,       /* a caller buffer (workspace, tape), or the fixed scratch of
                            mpm_mcis_select_static, is smaller than required */
  MPM_EDEVICE = -3,      /* a HIP runtime call failed */
  MPM_ESTATE = -4,       /* call out of order (e.g. backward without a taped forward) */
  MPM_EUNSTABLE = -5,    /* device counters saw NaN/Inf or a stencil leaving the grid */
  MPM_EUNSUPPORTED = -6  /* valid request the library does not implement */
} mpm_status;

/* Elastic models (App. A.2 / B.1); J = det F, J+ = max(J, 1e-4).
 *   FCR:         tau = 2 mu (F - R) F^T + lam J (J - 1) I, R the rotation of F = R S.
 *   HENCKY:      tau = U diag(2 mu eps + lam tr(eps)) U^T, eps = log(max(sigma, 1e-4)),
 *                F = U diag(sigma) V^T with U, V rotations.
 *   NEO_HOOKEAN: tau = mu (F F^T - I) + lam log(J+) I          (P = mu (F - F^-T) + lam log J F^-T).
 *   STVK:        tau = F (2 mu E + lam tr(E) I) F^T, E = (F^T F - I) / 2 (Green-Lagrange).
 *   FLUID:       tau = lam J (J - 1) I                          (mu unused).
 *   VOLUME:      tau = kappa (J - 1 / J+) I, kappa = 2/3 mu + lam (Mie-Grueneisen form, gamma = 2).  */
enum {
  MPM_ELASTIC_FCR = 0,
  MPM_ELASTIC_HENCKY = 1,
  MPM_ELASTIC_NEO_HOOKEAN = 2,
  MPM_ELASTIC_STVK = 3,
  MPM_ELASTIC_FLUID = 4,
  MPM_ELASTIC_VOLUME = 5
};

/* Plastic return maps (App. A.2 / B.2), applied to F after the stress.
 *   NONE:            F' = F.
 *   VON_MISES:       project the log-strain deviator onto |eps_hat| = yield/(2 mu).
 *   DRUCKER_PRAGER:  tension (tr eps > 0) -> F' = U V^T; else
 *                    dgamma = |eps_hat| + (3 lam + 2 mu)/(2 mu) tr(eps) alpha,
 *                    alpha = sqrt(2/3) 2 sin(phi)/(3 - sin(phi)), zero cohesion.
 *   FLUID:           F' = cbrt(J) I (real cube root: an inverted F keeps det < 0).
 *   SIGMA:           F' = cbrt(clamp(J, 0.05, 1.2)) I.
 * VON_MISES and DRUCKER_PRAGER take an FP64 SVD of F; FLUID and SIGMA only det F.  */
enum {
  MPM_PLASTIC_NONE = 0,
  MPM_PLASTIC_VON_MISES = 1,
  MPM_PLASTIC_DRUCKER_PRAGER = 2,
  MPM_PLASTIC_FLUID = 3,
  MPM_PLASTIC_SIGMA = 4
};

typedef struct {
  int32_t elastic;       /* MPM_ELASTIC_* */
  int32_t plastic;       /* MPM_PLASTIC_* */
  float yield_stress;    /* von Mises yield stress sigma_y, Pa (> 0 for VON_MISES) */
  float friction_deg;    /* Drucker-Prager friction angle phi in degrees (0 < phi < 90) */
} mpm_material;

typedef struct {
  int32_t abi_version;   /* must be MPM_ABI_VERSION */
  int32_t grid_res;      /* n: nodes per axis, 8 <= n <= 1024 */
  int32_t bound;         /* sticky wall width in nodes (v_i = 0 if any index < bound or >= n - bound) */
  int32_t n_batch;       /* number of independent scenes, >= 1 */
  float dt;              /* substep, s (> 0) */
  float gravity[3];      /* acceleration, m/s^2, added to grid velocity as dt * g */
  int32_t sort_every;    /* re-sort particles by cell every this many substeps (0 = library default) */
  uint32_t flags;        /* 0 or MPM_FLAG_* below */
} mpm_config;

/* Deterministic forward: the particle state after any sequence of substep
 * calls is a function of the inputs alone, bit for bit (the same on every
 * run, whatever the order of the GPU's atomic operations), and a scene's
 * result in a batched context equals its result alone.  The P2G of each
 * substep adds every contribution, rounded to one fixed-point scale per
 * scene (a power of two set by the scene's largest contribution bound B_b,
 * its largest work item and its particle count), as 64-bit integers, which
 * sum exactly in any order.  The first P2G launch of a context measures B_b
 * in a launch of its own; later ones take their scales from the previous
 * launch's bounds while measuring B_b, and scatter again, from the stored
 * state, any scene whose measured scale differs (counted in
 * mpm_diag.det_rescales), so the sums are always those of the measured
 * scale.  The particles of each cell are ordered by index at every sort,
 * and the stress of a substep is taken from F as stored in float32, so a
 * run split at any call boundary (mpm_step_n, mpm_advance, mpm_store /
 * mpm_load) equals the run in one piece.  mpm_backward is deterministic
 * too: its adjoint scatter into the grid adds at one fixed-point scale per
 * scene, set by a bound of the contributions taken before the scatter.
 * Costs a conversion launch and a second stress evaluation per substep, v
 * and C stored at every substep, a bound pass per reversed substep and 64 B
 * per grid node (plus 4 B per 4^3-node block) of workspace.  A cell of more
 * than 4096 particles keeps the order of the atomics (counted in
 * mpm_diag.order_fallbacks). */
#define MPM_FLAG_DETERMINISTIC 1u

/* Block-sparse grid activity.  The three grid buffers the substeps rotate
 * through carry one flag per 4^3-node block; a substep flags the blocks it
 * adds mass to and, when it clears a buffer for the substep after next,
 * zeroes only the flagged blocks.  The grid work then follows the occupied
 * blocks rather than n^3 (the memory stays dense: n^3 float4 nodes per
 * buffer).  The default (neither flag) takes it when the grid has more than
 * 4 nodes per particle; MPM_FLAG_GRID_SPARSE asks for it, MPM_FLAG_GRID_DENSE
 * for dense clearing.  Not with MPM_FLAG_DETERMINISTIC (which clears
 * densely); the two sparse / dense flags together are invalid. */
#define MPM_FLAG_GRID_SPARSE 2u
#define MPM_FLAG_GRID_DENSE 4u

typedef struct {
  float* x;              /* [3][N] in/out */
  float* v;              /* [3][N] in/out */
  float* C;              /* [9][N] in/out (APIC affine matrix) */
  float* F;              /* [9][N] in/out (elastic deformation gradient) */
  const float* mass;     /* [N] */
  const float* vol0;     /* [N] */
  const float* log_E;    /* [N] */
  const float* nu;       /* [N], 0 <= nu < 0.5 */
  const int32_t* mat_id; /* [N], 0 <= mat_id < n_materials */
} mpm_particles;

typedef struct {
  int64_t nonfinite;      /* particle-substeps that produced a NaN/Inf x or F */
  int64_t out_of_grid;    /* particle-substeps whose stencil left the grid (skipped) */
  int64_t tile_overflow;  /* work items whose box exceeded the LDS tiles (global-memory transfers) */
  int64_t tile_escapes;   /* particles that left their item's P2G tile in one substep (global atomics) */
  int64_t substeps;       /* substeps run since mpm_init */
  int64_t cfl_violations; /* particle-substeps whose G2P velocity moves more than half a cell:
                             |v'| dt / dx > 1/2 */
  double max_cfl;         /* largest |v'| dt / dx seen since mpm_init */
  double max_wave_cfl;    /* largest c dt / dx of the particles handed in since mpm_init, with
                             c^2 = (lam + 2 mu) V0 / m the squared P-wave speed (the explicit
                             update is unstable once this is well above 1) */
  int64_t order_fallbacks; /* deterministic mode: sorts of a cell holding more than 4096
                              particles, which keep the atomics' order (0 otherwise) */
  int64_t det_rescales;    /* deterministic mode: P2G launches in which some scene's fixed-point
                              scale differed from the one predicted from the previous launch's
                              bounds, so that the scene was scattered again (0 otherwise) */
} mpm_diag;

/* Status code as text (static storage). */
const char* mpm_status_string(int status);

/* Text of the last error on this context (static per context; never NULL). */
const char* mpm_last_error(mpm_ctx ctx);

/* Bytes of device workspace a context for n_particles particles under cfg
 * needs (cell-sorted particle copies 204 B + permutation staging 128 B per
 * particle, three grids of 16 B per node, sort bins and work-item tables).
 * Host only; MPM_EINVAL for an invalid cfg or count. */
int mpm_workspace_size(const mpm_config* cfg, int64_t n_particles, size_t* bytes);

/* Create a context for n_particles particles split into cfg->n_batch scenes
 * by batch_offsets (host array of n_batch + 1 int64, offsets[0] = 0,
 * non-decreasing, offsets[n_batch] = n_particles; NULL allowed when
 * n_batch == 1).  Copies the material table (n_materials >= 1).
 * workspace: caller-owned device memory on the current HIP device, 256-byte
 * aligned, of workspace_bytes >= mpm_workspace_size bytes; the context keeps
 * its grids, sort and particle buffers there, so it must stay allocated and
 * untouched until mpm_destroy.  The library allocates no device memory.
 * MPM_EINVAL for invalid arguments or a NULL / misaligned workspace,
 * MPM_ENOMEM when workspace_bytes is too small.  On success *out holds the
 * context (Sec. 3.2 MPM state; App. A.1 grid). */
int mpm_init(const mpm_config* cfg, const mpm_material* materials, int32_t n_materials,
             int64_t n_particles, const int64_t* batch_offsets, void* workspace, size_t workspace_bytes,
             mpm_ctx* out);

/* One substep: stress -> P2G -> grid update -> G2P -> return map, updating
 * x, v, C, F in place.  Equivalent to mpm_step_n(ctx, p, 1, NULL, stream). */
int mpm_substep(mpm_ctx ctx, const mpm_particles* p, void* stream);

/* n_steps >= 0 substeps (Alg. 1 stage-1 inner loop).  tape: NULL for a
 * forward-only run, else a device buffer of mpm_tape_size() bytes that
 * receives the checkpoints mpm_backward needs (state every K substeps,
 * K = checkpoint_every >= 1). */
int mpm_step_n(mpm_ctx ctx, const mpm_particles* p, int32_t n_steps,
               void* tape, int32_t checkpoint_every, void* stream);

/* Resident stepping: the scene stays in the context between calls, in the
 * library's cell-sorted order, so a frame loop (Alg. 1 stage-1 inner loop,
 * one render frame every few substeps) moves only what the renderer reads.
 *   mpm_load(ctx, p)        copies the caller's state and parameters in
 *                           (the same arrays and rules as mpm_step_n); later
 *                           changes to p take effect only through another
 *                           mpm_load.
 *   mpm_advance(ctx, n)     n >= 0 substeps of the resident state.  The
 *                           grid of the next substep carries over between
 *                           calls, so consecutive calls run fused substeps
 *                           only; re-sorts follow sort_every across calls.
 *   mpm_store(ctx, p)       writes x, v, C, F of the resident state to p's
 *                           arrays in the caller's order (other arrays unread).
 *   mpm_export_frame(ctx, x, cov0, cov)
 *                           the frame's positions x [3][N] and Gaussian
 *                           covariances cov [6][N] = F Sigma0 F^T (Sec. 3.2;
 *                           cov0, cov as in mpm_export_covariance) in the
 *                           caller's order; x or cov may be NULL (not both),
 *                           cov0 is needed with cov.
 * mpm_advance, mpm_store and mpm_export_frame return MPM_ESTATE when no state
 * is resident: before mpm_load, and after any call that takes the context's
 * internal state from elsewhere (mpm_step_n, mpm_substep, mpm_autotune,
 * mpm_backward, mpm_graph_launch) or a failed mpm_advance.  None of the four
 * may be captured into a graph (MPM_ESTATE).  Results match mpm_step_n from
 * the same state up to FP32 rounding (the particle order at each substep
 * differs, so global atomics add in another order). */
int mpm_load(mpm_ctx ctx, const mpm_particles* p, void* stream);
int mpm_advance(mpm_ctx ctx, int32_t n_steps, void* stream);
int mpm_store(mpm_ctx ctx, const mpm_particles* p, void* stream);
int mpm_export_frame(mpm_ctx ctx, float* x, const float* cov0, float* cov, void* stream);

/* Bytes of the tape buffer for n_steps substeps checkpointed every K: the
 * checkpoints (96 B per particle each), one segment of K recomputed states
 * (K + 1 when a material has a return map) with their K grids (16 B per
 * node each) and work-item boxes, and the adjoint scratch. */
int mpm_tape_size(mpm_ctx ctx, int32_t n_steps, int32_t checkpoint_every, size_t* bytes);

/* Reverse of the n_steps substeps taped by the last mpm_step_n call with
 * the same tape: every elastic model and every return map (the von Mises and
 * Drucker-Prager maps through the SVD of F_trial, fluid and sigma through
 * det F_trial; at a yield surface the one-sided derivative of the branch the
 * forward pass took).  Inputs: the
 * adjoints of the final x, v, C, F (device [3][N], [3][N], [9][N], [9][N];
 * any may be NULL = zero).  Outputs (overwritten): g_log_E[N], g_nu[N] and,
 * when non-NULL, the adjoints of the initial state g_x0, g_v0, g_C0, g_F0.
 * p supplies the parameter arrays (its state arrays are not read). */
int mpm_backward(mpm_ctx ctx, const mpm_particles* p, const void* tape, int32_t n_steps,
                 const float* g_x, const float* g_v, const float* g_C, const float* g_F,
                 float* g_log_E, float* g_nu,
                 float* g_x0, float* g_v0, float* g_C0, float* g_F0, void* stream);

/* Grid of the most recent substep, for tests: m [B][n^3], mv and v [B][n^3][3],
 * node (ix, iy, iz) at ((ix*n)+iy)*n+iz (iz fastest).  Any pointer may be NULL. */
int mpm_grid_state(mpm_ctx ctx, float* m, float* mv, float* v, void* stream);

/* Gaussian covariances Sigma_p = F_p Sigma0_p F_p^T (Sec. 3.2) for n
 * particles: F [9][n], cov0 and cov [6][n] as (xx, xy, xz, yy, yz, zz). */
int mpm_export_covariance(mpm_ctx ctx, const float* F, const float* cov0, float* cov,
                          int64_t n, void* stream);

/* Synchronises the context's last stream and reads the device counters.
 * Returns MPM_EUNSTABLE when any particle-substep was non-finite, left the
 * grid or broke the CFL watch (cfl_violations > 0), else MPM_OK. */
int mpm_get_diagnostics(mpm_ctx ctx, mpm_diag* out);

/* Launch tuning.  chunk = particles per work item, cut from one 4^3-cell
 * block (64..8192, multiple of 64; applied at the next sort); sort_every =
 * substeps between re-sorts; tile_cap = LDS tile nodes (27..1331);
 * workgroups = width of the persistent substep kernel.  In mpm_set_tuning a
 * zero field keeps the current value; ms_per_substep is an output of
 * mpm_autotune only.  Defaults after mpm_init: chunk 768, the library's
 * re-sort interval, tile_cap 1331, 512 workgroups (at most one per possible
 * work item).  Small scenes run faster with smaller work items (mpm_autotune
 * picks 256 for 20,480 particles), at more float32 partial sums per grid
 * node when many particles share a cell. */
typedef struct {
  int32_t chunk;
  int32_t sort_every;
  int32_t tile_cap;
  int32_t workgroups;
  double ms_per_substep;
} mpm_tuning;

int mpm_set_tuning(mpm_ctx ctx, const mpm_tuning* t);
int mpm_get_tuning(mpm_ctx ctx, mpm_tuning* t);

/* Autotuner: times trial runs of trial_steps (>= 2) substeps of the given
 * particles for candidate settings (coordinate descent over chunk in
 * {256..2048}, then workgroups in {256..2048}, then sort_every in {2..64}
 * below 2 trial_steps) with HIP events on `stream`, applies the fastest and
 * returns it in *best.  Synchronous.  The trial runs work on the context's
 * internal copies: the caller's arrays are only read.  Use trial_steps equal
 * to the substeps of the calls to be tuned: each trial is such a call. */
int mpm_autotune(mpm_ctx ctx, const mpm_particles* p, int32_t trial_steps, void* stream, mpm_tuning* best);

/* Graph capture.  Between mpm_graph_begin and mpm_graph_end every call on
 * this context that takes `stream` (which must be the same non-null stream)
 * is recorded instead of run; mpm_graph_end returns an executable hipGraph
 * that mpm_graph_launch replays on the same buffers (the context and every
 * buffer must outlive it).  Used to run a whole evaluation of a batch of
 * candidates (one context with n_batch scenes): mpm_step_n with a tape,
 * mpm_position_loss_grad, mpm_backward, in one launch.  Host-side argument
 * checks still run at capture time. */
typedef struct mpm_graph_s* mpm_graph;
int mpm_graph_begin(mpm_ctx ctx, void* stream);
int mpm_graph_end(mpm_ctx ctx, void* stream, mpm_graph* out);
int mpm_graph_launch(mpm_graph g, void* stream);
int mpm_graph_destroy(mpm_graph g);

/* Cotangent of the position loss L = sum_p weight_p |x_p - x*_p|^2 used by
 * the differentiation workloads (weight_p = 1 / (3 N_scene) gives the mean
 * squared error per scene): g_x = 2 weight (x - x*), all [3][N] / [N]
 * device arrays. */
int mpm_position_loss_grad(mpm_ctx ctx, const float* x, const float* x_target, const float* weight, float* g_x,
                           void* stream);

/* BGDO (Alg. 1, Sec. 4.2, App. B.3-B.4): signals of one key frame.  `key`
 * is the key-frame state in the caller's order (reads F, log_E, nu,
 * mat_id); F_next [9][N] is F one substep later (mpm_substep from that
 * state, return map included).  For every particle, with E = exp(log_E):
 *   s      = |tau(F)|_F, the Kirchhoff stress of its elastic model; its
 *            derivative by log E equals s (tau is linear in mu, lam ~ E)
 *   delta  = |F_next - I|_F
 *   eta    = min(1, 0.1 log(1 + E))
 *   g_total[p] += eta log(1 + s) - (1 - eta) (delta - delta_target)
 * s_out, delta_out (optional, may be NULL) receive s and delta.  All
 * device arrays of N floats; g_total accumulates across key frames. */
int mpm_bgdo_accumulate(mpm_ctx ctx, const mpm_particles* key, const float* F_next, float delta_target,
                        float* g_total, float* s_out, float* delta_out, void* stream);

/* BGDO update: log_E[p] -= g_total[p] / n_keys (n_keys >= 1). */
int mpm_bgdo_apply(mpm_ctx ctx, float* log_E, const float* g_total, int32_t n_keys, void* stream);

/* Candidate generation of the interior fill (Sec. 4.1, the candidate points
 * of each instance drawn uniformly in the axis-aligned box of its convex hull
 * and kept where the hull's ray-cast occupancy exceeds a threshold, 0.6 in
 * the paper).  Context-free.  n_instances = K instances; instance k owns
 *   hull vertices   hull_vertices[3][V]     columns [hull_vertex_offsets[k], .. [k+1])
 *   hull triangles  hull_triangles[3][T]    int32 vertex indices local to the
 *                                           instance's vertex range, columns
 *                                           [hull_triangle_offsets[k], .. [k+1])
 *   raw candidates  u[3][R] (float64)       columns [raw_offsets[k], .. [k+1])
 * (hull_vertices, hull_triangles, u, candidates_out, source_out: device; the
 * three offset arrays and candidate_offsets_out: host, int64, K+1 entries,
 * offsets starting at 0).  The mesh is the caller's hull of the instance's
 * points (the paper: Quickhull); its vertices must lie in [0, 1]^3.  For
 * raw candidate j of instance k:
 *   B_k = per-axis [b_min, b_max] over the vertices the triangles use
 *   q_j = b_min + u_j (b_max - b_min), in float64, rounded to float32
 *   occ = the fraction of the six rays from q_j along +x, -x, +y, -y, +z, -z
 *         that cross the mesh an odd number of times (crossings tested in
 *         float64 without contraction, exact zeros of the 2D edge functions
 *         resolved by simulation of simplicity, so a ray through a shared
 *         edge or vertex crosses exactly one triangle of a closed mesh);
 * and q_j is kept when occ > occupancy_threshold (in [0, 1]).  An instance
 * without triangles keeps nothing.  The kept candidates are written in raw
 * order, instance by instance, to candidates_out as [3][M_in] planes of
 * stride M_in = candidate_offsets_out[K] (room for 3 R floats), with
 * candidate_offsets_out[k] the first kept candidate of instance k: the
 * layout and offsets mpm_mcis_select takes.  source_out (optional, may be
 * NULL; room for R entries) receives each kept candidate's raw index j.
 * workspace: device memory of the size mpm_ipf_workspace_size gives,
 * overwritten.  Runs on `stream` and synchronises it before returning.
 * MPM_EINVAL for bad sizes or offsets, a threshold outside [0, 1], a
 * missing workspace or output, or (found on the device) triangle indices
 * outside their instance, vertices outside [0, 1]^3 or u outside [0, 1];
 * MPM_EDEVICE for a HIP failure.  Limits: K <= 2^20, T <= 2^27, V < 2^31,
 * R < 2^30. */
int mpm_ipf_workspace_size(int32_t n_instances, int64_t n_hull_vertices, int64_t n_hull_triangles, int64_t n_raw,
                           size_t* bytes);
int mpm_ipf_candidates(int32_t n_instances, const float* hull_vertices, const int64_t* hull_vertex_offsets,
                       const int32_t* hull_triangles, const int64_t* hull_triangle_offsets, const double* u,
                       const int64_t* raw_offsets, double occupancy_threshold, void* workspace,
                       size_t workspace_bytes, float* candidates_out, int64_t* source_out,
                       int64_t* candidate_offsets_out, void* stream);

/* Interior filling by instance-aware Monte Carlo importance sampling (Sec. 4.1,
 * MCIS steps 1-5).  Context-free.  n_instances = K instances; instance k owns
 *   surface points     surface[3][S]    columns [surface_offsets[k], surface_offsets[k+1])
 *   candidate points   candidates[3][M] columns [candidate_offsets[k], candidate_offsets[k+1])
 *                      (points the caller's occupancy test kept inside the instance)
 *   uniforms           u[M] (float64, in (0, 1]), one per candidate
 *   count              n_select[k], 0 <= n_select[k] <= the instance's candidates
 * (surface, candidates, u, out_index, d_out: device; the three offset /
 * count arrays: host, int64, offsets starting at 0).  Every point must lie
 * in [0, 1]^3 (scenes are normalised to the unit cube, App. C).
 * For every candidate j of instance k, with r_s = sigma sqrt(-2 ln eps):
 *   d_j = distance to the nearest surface point of instance k (+inf when
 *         none lies within r_s: the weight is then at its floor either way)
 *   w_j = max(exp(-d_j^2 / (2 sigma^2)), eps)      (the paper: sigma 0.02, eps 1e-6)
 * and the n_select[k] candidates with the largest keys log(u_j) / w_j (the
 * exponential keys of sampling without replacement by p = w / sum w, whose
 * common factor does not change the order; equal keys by lower index) are
 * written, ascending, to out_index[o_k .. o_k + n_select[k]) with
 * o_k = n_select[0] + ... + n_select[k-1].  d_out (optional, may be NULL)
 * receives d_j.  workspace: device memory of the size
 * mpm_mcis_workspace_size gives, overwritten.  Runs on `stream` and
 * synchronises it before returning.  MPM_EINVAL for bad sizes, offsets or
 * counts, a missing workspace, or (found on the device) points outside the
 * unit cube or u outside (0, 1]; MPM_EDEVICE for a HIP failure. */
int mpm_mcis_workspace_size(int32_t n_instances, int64_t n_surface, int64_t n_candidates, double sigma, double eps,
                            size_t* bytes);
int mpm_mcis_select(int32_t n_instances, const float* surface, const int64_t* surface_offsets,
                    const float* candidates, const int64_t* candidate_offsets, const double* u,
                    const int64_t* n_select, double sigma, double eps, void* workspace, size_t workspace_bytes,
                    int64_t* out_index, double* d_out, void* stream);

/* mpm_mcis_select without allocation, for callers that cannot allocate
 * device memory (serving loops, code that may not call hipMalloc): the same
 * operation, arguments and results as mpm_mcis_select, with the workspace
 * taken from a fixed 64 MiB device array that the library holds on each GPU
 * it runs on until the process ends (no workspace arguments).  Supports at
 * most 256 instances and inputs whose layout fits the array (about 2M
 * candidates plus surface points; the search grid is coarsened to fit,
 * which leaves the result unchanged).  MPM_ENOMEM for inputs beyond that,
 * MPM_EINVAL as for mpm_mcis_select, MPM_EDEVICE if the array's device
 * address cannot be obtained.  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (other host threads, other streams)
 * race and must not be issued.  Synchronises `stream` before returning. */
int mpm_mcis_select_static(int32_t n_instances, const float* surface, const int64_t* surface_offsets,
                           const float* candidates, const int64_t* candidate_offsets, const double* u,
                           const int64_t* n_select, double sigma, double eps, int64_t* out_index, double* d_out,
                           void* stream);

/* Kernel timing with HIP events recorded on the launch stream around each
 * launch, by class: 0 fused G2P+P2G substep kernel, 1 P2G-only kernel,
 * 2 G2P-only kernel, 3 sort and permute, 4 grid clear, 5 gather from /
 * scatter to the caller's arrays, 6 adjoint G2P kernel, 7 adjoint P2G
 * kernel.  enable = 0 stops recording. */
#define MPM_PROFILE_CLASSES 8
int mpm_profile(mpm_ctx ctx, int32_t enable);

/* Synchronises, then returns the summed milliseconds and the number of
 * timed launches per class (arrays of MPM_PROFILE_CLASSES) and resets them. */
int mpm_profile_read(mpm_ctx ctx, double* ms, int64_t* launches);

/* Release the context (synchronises the device); the caller may then free
 * the workspace. */
int mpm_destroy(mpm_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* FASTMPM_H */
