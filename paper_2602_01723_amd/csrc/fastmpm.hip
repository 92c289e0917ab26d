// libfastmpm.so: host side of the C ABI declared in include/fastmpm.h.
//
// A context holds the configuration, the material table and pointers into
// the caller's workspace: cell-sorted copies of the particle state, three
// grids in rotation, the counting-sort and permutation buffers and the
// device diagnostics counters.  The library allocates no device memory.  mpm_step_n sorts the caller's
// particles by cell, runs the substeps on the sorted copies (re-sorting
// every `sort_every` substeps) and writes the state back in caller order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "fastmpm.h"
#include "mpm_adjoint.hpp"
#include "mpm_kernels.hpp"
#include "mcis_kernels.hpp"
#include "ipf_kernels.hpp"

using fmpm::kBlock;

// device counters: 0 non-finite, 1 out of grid, 2 tile overflow, 3 tile
// escapes, 4 CFL violations, 5 max (|v'| dt / dx)^2 and 6 max (c dt / dx)^2
// (float bits in the low word), 7 cells left in atomic order by the
// deterministic sort (more than fmpm::kStableMax particles), 8 deterministic
// P2G launches whose predicted scales missed for some scene
constexpr int kDiagSlots = 9;

struct mpm_context {
  mpm_config cfg{};
  int n_mat = 0;
  fmpm::Material mats[fmpm::kMaxMaterials]{};
  int64_t N = 0;
  int B = 1;
  std::vector<int64_t> offsets;
  int n = 0, nb = 0;
  int64_t nodes = 0;  // B * n^3
  int64_t bins = 0;   // sort bins
  int64_t n_bsum = 0;
  int n_chunks = 0;
  int tile_cap = fmpm::kTileCapMax;
  int sort_every = 8;

  float *xs = nullptr, *vs = nullptr, *Cs = nullptr, *Fs = nullptr, *xs2 = nullptr, *Fs2 = nullptr;
  float4 *prm = nullptr, *prm2 = nullptr;
  int *mat = nullptr, *mat2 = nullptr, *pid = nullptr, *pid2 = nullptr, *perm = nullptr;
  // rotation: read, write, cleared for the step after; each buffer is
  // followed by one flag per 4^3-node block (block-sparse clearing)
  float4* grid[3] = {nullptr, nullptr, nullptr};
  bool sparse = false;  // the rotation's launches flag blocks and clear only flagged ones
  unsigned* done_counter = nullptr;                // finished workgroups of the substep kernel
  int* item_box = nullptr;                         // [2][max_chunks][6]: per-item cell boxes, in turn
  int *chunk_start = nullptr, *chunk_batch = nullptr;            // by scene, fixed (cell keys)
  int *dchunk_start = nullptr, *dchunk_batch = nullptr, *dn_chunks = nullptr;  // by cell block, per sort
  uint32_t* nchk = nullptr;
  int* work_counter = nullptr;  // work-item queue head of the substep kernel
  int item = 768;               // particles per work item
  int64_t nblocks = 0;
  int64_t max_chunks = 0;
  int grid_blocks = 0;
  uint32_t *keys = nullptr, *slots = nullptr, *count = nullptr, *bsum = nullptr;
  // bucketed permutation (k_perm_*): destinations, positions, pass-1 buffer, counts
  int *pdest = nullptr, *ppos = nullptr, *pdop = nullptr;
  float* ptmp = nullptr;
  uint32_t *pcount = nullptr, *pbsum = nullptr;
  const int* pdest_cur = nullptr;  // destinations of the prepared permutation
  unsigned long long* diag = nullptr;
  fmpm::Material* d_mats = nullptr;
  // deterministic mode (MPM_FLAG_DETERMINISTIC): three banks of per-scene
  // bounds (4 words per scene; banks 0 and 1 alternate between the forward's
  // P2G launches, bank 2 is the adjoint's), the range factors, the 64-bit
  // fixed-point grid and the one a rescaled scene is scattered into again,
  // the second permutation buffer
  bool det = false;
  unsigned* fxb = nullptr;
  float2* fxi = nullptr;    // per-item bounds of the last measuring launch
  int* scene_item = nullptr;  // each scene's first item, then the item count (per sort)
  unsigned* gflag = nullptr;  // one flag per 4^3-node block of gfx, set by the accumulating launches
  double* fxk = nullptr;
  unsigned long long *gfx = nullptr, *gfx2 = nullptr;
  int* perm2 = nullptr;
  int fx_bank = 0;          // the bank the next forward P2G launch measures into
  bool fx_primed = false;   // the other bank holds bounds of an earlier launch
  size_t workspace_bytes = 0;  // of the caller's workspace, which holds every device buffer above

  // kernel timing (mpm_profile): event pairs recorded around launches
  bool prof_on = false;
  std::vector<hipEvent_t> prof_ev;
  std::vector<int> prof_cls;
  double prof_ms[MPM_PROFILE_CLASSES] = {0};
  int64_t prof_cnt[MPM_PROFILE_CLASSES] = {0};

  // resident stepping (mpm_load / mpm_advance / mpm_store / mpm_export_frame)
  bool resident = false;  // the internal sorted state holds the scene of the last mpm_load
  bool primed = false;    // grid[res_cur] holds the P2G of the internal state
  int res_cur = 0;        // grid rotation index
  int res_bcur = 0;       // item-box buffer the next substep kernel reads
  bool res_have_box = false;
  int res_since_sort = 0;  // substeps since the internal state was last sorted

  bool capturing = false;  // between mpm_graph_begin and mpm_graph_end
  bool prof_saved = false;
  // the last taped forward (mpm_step_n with a tape)
  const void* tape_ptr = nullptr;
  int32_t tape_n = -1;
  int32_t tape_K = 0;

  int last_grid = -1;
  int64_t substeps = 0;
  hipStream_t last_stream = nullptr;
  std::string err = "no error";
};

namespace {

const char* kStatusText[] = {"ok", "invalid argument", "out of memory", "HIP device error",
                             "call out of order", "unstable simulation", "unsupported"};

int fail(mpm_ctx ctx, int code, const std::string& what) {
  if (ctx) ctx->err = what;
  return code;
}

int hip_fail(mpm_ctx ctx, const char* what, hipError_t e) {
  return fail(ctx, MPM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                   \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), #call, e_); \
  } while (0)

#define LAUNCH_CHECK(ctx, name)                                  \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return hip_fail((ctx), (name), e_);   \
  } while (0)


constexpr int kProfPairs = 4096;

// Records a HIP event pair around the launches issued in its scope.
struct ProfScope {
  mpm_ctx c;
  hipStream_t s;
  int cls;
  int idx = -1;
  ProfScope(mpm_ctx c_, hipStream_t s_, int cls_) : c(c_), s(s_), cls(cls_) {
    if (cls >= 0 && c->prof_on && (int)c->prof_cls.size() < kProfPairs) {
      idx = (int)c->prof_cls.size();
      c->prof_cls.push_back(-1);  // slot reserved; class set when the pair is complete
      if (hipEventRecord(c->prof_ev[2 * idx], s) != hipSuccess) idx = -1;
    }
  }
  ~ProfScope() {
    if (idx >= 0 && hipEventRecord(c->prof_ev[2 * idx + 1], s) == hipSuccess) c->prof_cls[idx] = cls;
  }
};

inline unsigned blocks_for(int64_t n, int threads) { return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads); }

int fill_u32(mpm_ctx ctx, void* p, int64_t count, hipStream_t s, int cls = -1, int* counter = nullptr) {
  ProfScope ps(ctx, s, cls);
  const int64_t n4 = std::max<int64_t>(count >> 2, 4);
  fmpm::k_fill_u32<<<blocks_for(n4, 256), 256, 0, s>>>((uint32_t*)p, 0u, count, counter);
  LAUNCH_CHECK(ctx, "k_fill_u32");
  return MPM_OK;
}

fmpm::SubstepArgs make_args(mpm_ctx c) {
  fmpm::SubstepArgs a{};
  a.x = c->xs;
  a.v = c->vs;
  a.C = c->Cs;
  a.F = c->Fs;
  a.xo = c->xs;
  a.vo = c->vs;
  a.Co = c->Cs;
  a.Fo = c->Fs;
  a.prm = c->prm;
  a.mat = c->mat;
  a.N = c->N;
  a.chunk_start = c->dchunk_start;
  a.chunk_batch = c->dchunk_batch;
  a.n_chunks = c->dn_chunks;
  a.work_counter = c->work_counter;
  a.n = c->n;
  a.bound = c->cfg.bound;
  a.dt = c->cfg.dt;
  for (int k = 0; k < 3; ++k) a.g[k] = c->cfg.gravity[k];
  a.tile_cap = c->tile_cap;
  a.diag = c->diag;
  a.n_materials = c->n_mat;
  a.mats = c->d_mats;
  a.done_counter = c->done_counter;
  const double vmax = 0.5 / ((double)c->cfg.dt * (double)c->n);  // |v| dt / dx = 1/2
  a.cfl_v2 = (float)(vmax * vmax);
  a.n_scenes = c->B;
  return a;
}

// counting sort of particles by cell key; perm[j] = source index of slot j
int sort_keys(mpm_ctx c, const float* x, hipStream_t s) {
  int rc = fill_u32(c, c->count, c->bins, s);
  if (rc) return rc;
  fmpm::k_cell_keys<<<c->n_chunks, kBlock, 0, s>>>(x, c->N, c->chunk_start, c->chunk_batch, c->n, c->nb, c->keys,
                                                   c->slots, c->count);
  LAUNCH_CHECK(c, "k_cell_keys");
  fmpm::k_scan_reduce<<<(unsigned)c->n_bsum, fmpm::kScanThreads, 0, s>>>(c->count, c->bsum, c->bins);
  LAUNCH_CHECK(c, "k_scan_reduce");
  fmpm::k_scan_top<<<1, fmpm::kScanThreads, 0, s>>>(c->bsum, c->n_bsum);
  LAUNCH_CHECK(c, "k_scan_top");
  fmpm::k_scan_apply<<<(unsigned)c->n_bsum, fmpm::kScanThreads, 0, s>>>(c->count, c->bsum, c->bins);
  LAUNCH_CHECK(c, "k_scan_apply");
  fmpm::k_place<<<blocks_for(c->N, 256), 256, 0, s>>>(c->keys, c->slots, c->count, c->perm, c->N);
  LAUNCH_CHECK(c, "k_place");
  if (c->det) {  // each cell's particles by source index
    fmpm::k_stable_rank<<<blocks_for(c->N, 256), 256, 0, s>>>(c->perm, c->keys, c->count, c->bins, c->N, c->perm2,
                                                              c->diag + 7);
    LAUNCH_CHECK(c, "k_stable_rank");
    std::swap(c->perm, c->perm2);
  }
  // chunk table of the new order
  const unsigned gb = blocks_for(c->nblocks, 256);
  fmpm::k_block_chunk_count<<<gb, 256, 0, s>>>(c->count, c->nblocks, c->N, c->item, c->nchk);
  const int64_t nbs = (c->nblocks + fmpm::kScanTile - 1) / fmpm::kScanTile;
  fmpm::k_scan_reduce<<<(unsigned)nbs, fmpm::kScanThreads, 0, s>>>(c->nchk, c->bsum, c->nblocks);
  fmpm::k_scan_top<<<1, fmpm::kScanThreads, 0, s>>>(c->bsum, nbs);
  fmpm::k_scan_apply<<<(unsigned)nbs, fmpm::kScanThreads, 0, s>>>(c->nchk, c->bsum, c->nblocks);
  fmpm::k_block_chunk_write<<<gb, 256, 0, s>>>(c->count, c->nchk, c->nblocks, c->N, c->item, c->nb * c->nb * c->nb,
                                               c->dchunk_start, c->dchunk_batch, c->dn_chunks, c->scene_item);
  LAUNCH_CHECK(c, "chunk table");
  return MPM_OK;
}

// Geometry of the bucketed permutation of N elements: buckets of 2^shift
// destinations (at most 4096), counting tiles of ts sources (at most 2048).
// Pass 2 holds one bucket per workgroup in LDS, so the bucketed form serves
// N <= 2^26 (64 KB); larger N use one scatter pass.  Up to 2048 buckets
// (N <= 2^23) pass 1 is staged through LDS one 8192-source tile at a time.
struct PermGeom {
  int shift = 12, nb = 0;
  int64_t ts = 0, ntiles = 0, entries = 0;
  bool bucketed = false, staged = false;
};

PermGeom perm_geom(int64_t N) {
  PermGeom g;
  int lg = 0;
  while (((int64_t)1 << lg) < N) ++lg;
  g.shift = std::max(12, lg - 12);
  g.nb = (int)((N + ((int64_t)1 << g.shift) - 1) >> g.shift);
  g.bucketed = N > 0 && g.shift <= 14;
  g.staged = g.bucketed && g.nb <= 2048;
  g.ts = g.staged ? 8192 : std::max<int64_t>(4096, ((N + 2047) / 2048 + 255) / 256 * 256);
  g.ntiles = (N + g.ts - 1) / g.ts;
  g.entries = (int64_t)g.nb * g.ntiles;
  return g;
}

// Positions of the permutation out[dest[s]] = in[s] (dest a permutation of
// [0, N), device array that must stay unchanged until the last perm_apply).
int perm_prepare(mpm_ctx c, const int* dest, hipStream_t s) {
  c->pdest_cur = dest;
  const PermGeom g = perm_geom(c->N);
  if (!g.bucketed) return MPM_OK;
  const size_t lds = (size_t)g.nb * sizeof(uint32_t);
  fmpm::k_perm_count<<<(unsigned)g.ntiles, 256, lds, s>>>(dest, c->N, g.shift, g.ts, g.nb, g.ntiles, c->pcount);
  LAUNCH_CHECK(c, "k_perm_count");
  const int64_t nbs = (g.entries + fmpm::kScanTile - 1) / fmpm::kScanTile;
  fmpm::k_scan_reduce<<<(unsigned)nbs, fmpm::kScanThreads, 0, s>>>(c->pcount, c->pbsum, g.entries);
  fmpm::k_scan_top<<<1, fmpm::kScanThreads, 0, s>>>(c->pbsum, nbs);
  fmpm::k_scan_apply<<<(unsigned)nbs, fmpm::kScanThreads, 0, s>>>(c->pcount, c->pbsum, g.entries);
  LAUNCH_CHECK(c, "permutation scan");
  fmpm::k_perm_rank<<<(unsigned)g.ntiles, 256, lds, s>>>(dest, c->N, g.shift, g.ts, g.nb, g.ntiles, c->pcount,
                                                         c->ppos, c->pdop);
  LAUNCH_CHECK(c, "k_perm_rank");
  return MPM_OK;
}

// Apply the prepared permutation to up to 29 planes of N floats.
int perm_apply(mpm_ctx c, const fmpm::PlaneSet& ps, hipStream_t s) {
  if (c->N == 0 || ps.planes == 0) return MPM_OK;
  const PermGeom g = perm_geom(c->N);
  const unsigned gb = blocks_for(c->N, 256);
  const int groups = (ps.planes + fmpm::kPermPlanes - 1) / fmpm::kPermPlanes;  // pass-1 plane groups
  if (!g.bucketed) {
    fmpm::k_scatter_planes<<<gb, 256, 0, s>>>(ps, c->pdest_cur, c->N);
    LAUNCH_CHECK(c, "k_scatter_planes");
    return MPM_OK;
  }
  if (g.staged) {
    const size_t lds = (size_t)g.ts * 6 + (size_t)g.nb * 8;
    const dim3 grid1((unsigned)(8 * ((g.ntiles + 7) / 8)), (unsigned)groups);
    fmpm::k_perm_pass1_staged<<<grid1, 512, lds, s>>>(
        c->ptmp, ps, c->ppos, c->pcount, c->N, g.shift, (int)g.ts, g.nb, (int)g.ntiles);
  } else {
    const int64_t chunks = (c->N + fmpm::kPermChunk - 1) / fmpm::kPermChunk;
    fmpm::k_perm_pass1<<<(unsigned)(8 * ((chunks + 7) / 8)), 256, 0, s>>>(c->ptmp, ps, c->ppos, c->N);
  }
  LAUNCH_CHECK(c, "k_perm_pass1");
  fmpm::k_perm_pass2<<<(unsigned)g.nb, 1024, ((size_t)1 << g.shift) * sizeof(float), s>>>(ps, c->ptmp, c->pdop,
                                                                                          c->N, g.shift);
  LAUNCH_CHECK(c, "k_perm_pass2");
  return MPM_OK;
}

// Appends planes [0, planes) of two [*][N] blocks to a plane set (all of a
// call's planes go through one pass-1 / pass-2 launch pair).
void add_planes(fmpm::PlaneSet& ps, const float* in, float* out, int planes, int64_t N) {
  for (int k = 0; k < planes; ++k) {
    ps.in[ps.planes] = in + k * N;
    ps.out[ps.planes] = out + k * N;
    ++ps.planes;
  }
}

// The five parameter arrays of p, bound for (mass, vol0, log E, nu, mat id
// bits) planes at out[0..4].
void add_params(fmpm::PlaneSet& ps, const mpm_particles* p, float* const out[5]) {
  const float* in[5] = {p->mass, p->vol0, p->log_E, p->nu, reinterpret_cast<const float*>(p->mat_id)};
  for (int k = 0; k < 5; ++k) {
    ps.in[ps.planes] = in[k];
    ps.out[ps.planes] = out[k];
    ++ps.planes;
  }
}

// x, v, C, F: four plane blocks (3, 3, 9, 9 planes) in one set
fmpm::PlaneSet state_planes(const float* const in[4], float* const out[4], int64_t N) {
  static constexpr int kPl[4] = {3, 3, 9, 9};
  fmpm::PlaneSet ps{};
  for (int k = 0; k < 4; ++k) add_planes(ps, in[k], out[k], kPl[k], N);
  return ps;
}

// The prepared permutation applied to a [planes][N] block (planes <= 29).
int perm_block(mpm_ctx c, const float* in, float* out, int planes, hipStream_t s) {
  fmpm::PlaneSet ps{};
  add_planes(ps, in, out, planes, c->N);
  return perm_apply(c, ps, s);
}

int gather_from_caller(mpm_ctx c, const mpm_particles* p, hipStream_t s) {
  ProfScope ps(c, s, 5);
  const unsigned g = blocks_for(c->N, 256);
  const int64_t N = c->N;
  // sort the caller's particles by cell: perm = caller index of each slot
  int rc = sort_keys(c, p->x, s);
  if (rc) return rc;
  fmpm::k_invert<<<g, 256, 0, s>>>(c->perm, c->pdest, N);  // caller index -> slot
  LAUNCH_CHECK(c, "k_invert");
  rc = perm_prepare(c, c->pdest, s);
  const float* const in[4] = {p->x, p->v, p->C, p->F};
  float* const out[4] = {c->xs, c->vs, c->Cs, c->Fs};
  fmpm::PlaneSet pls = state_planes(in, out, N);
  float* const pl[5] = {c->Fs2, c->Fs2 + N, c->Fs2 + 2 * N, c->Fs2 + 3 * N, c->Fs2 + 4 * N};
  add_params(pls, p, pl);
  rc = rc ? rc : perm_apply(c, pls, s);
  if (rc) return rc;
  fmpm::k_params_planes<<<g, 256, 0, s>>>(c->prm, c->mat, c->pid, pl[0], pl[1], pl[2], pl[3], pl[4], c->perm, N,
                                          c->diag);
  LAUNCH_CHECK(c, "k_params_planes");
  return MPM_OK;
}

int resort_internal(mpm_ctx c, hipStream_t s) {
  ProfScope ps(c, s, 3);
  int rc = sort_keys(c, c->xs, s);
  if (rc) return rc;
  const unsigned g = blocks_for(c->N, 256);
  fmpm::k_gather_planes<<<g, 256, 0, s>>>(c->xs2, c->xs, c->perm, 3, c->N);
  fmpm::k_gather_planes<<<g, 256, 0, s>>>(c->Fs2, c->Fs, c->perm, 9, c->N);
  fmpm::k_gather_misc<<<g, 256, 0, s>>>(c->prm2, c->mat2, c->pid2, c->prm, c->mat, c->pid, c->perm, c->N);
  LAUNCH_CHECK(c, "resort");
  std::swap(c->xs, c->xs2);
  std::swap(c->Fs, c->Fs2);
  std::swap(c->prm, c->prm2);
  std::swap(c->mat, c->mat2);
  std::swap(c->pid, c->pid2);
  return MPM_OK;
}

int scatter_to_caller(mpm_ctx c, const mpm_particles* p, hipStream_t s) {
  ProfScope ps(c, s, 5);
  // sorted slot j -> caller index pid[j]
  int rc = perm_prepare(c, c->pid, s);
  const float* const in[4] = {c->xs, c->vs, c->Cs, c->Fs};
  float* const out[4] = {p->x, p->v, p->C, p->F};
  return rc ? rc : perm_apply(c, state_planes(in, out, c->N), s);
}

// Tape layout (floats; N particles, B n^3 grid nodes):
//   checkpoints  n_ckpt x 24 N   state at substeps 0, K, 2K, ... in caller order
//                                (x 3N, v 3N, C 9N, F 9N)
//   segment      K x 24 N        recomputed states of one segment, sorted order
//                                (K + 1 when a material has a return map)
//   adj, adjc    24 N each       state adjoint, sorted / caller order
//   gl, gn       N each          parameter gradients of a segment, sorted order
//   lnE, nu      N each          sorted copies of the parameters
//   vhb          4 B n^3         adjoint of the grid velocity
//   boxes        K x 6 items     per-item base-cell boxes of the segment's states (ints)
struct TapeLayout {
  int64_t n_ckpt, K;
  float *ckpt, *seg, *adj, *adjc, *gl, *gn, *lnE, *nu;
  float4* vhb;
  float4* grids;  // K grids (mv, m): the P2G result of each recomputed state of a segment
  int* boxes;     // K x (max_chunks + 1) x 6: item boxes of the recomputed states
  size_t bytes;
};

bool has_plastic(mpm_ctx c);

TapeLayout tape_layout(mpm_ctx c, int32_t n_steps, int32_t K, void* base) {
  TapeLayout t{};
  const int64_t N = std::max<int64_t>(c->N, 1);
  t.K = K;
  t.n_ckpt = std::max<int64_t>(1, (n_steps + K - 1) / K);
  char* p = static_cast<char*>(base);
  auto take = [&](int64_t floats) {
    char* q = p;
    p += ((floats * 4 + 255) / 256) * 256;
    return reinterpret_cast<float*>(q);
  };
  t.ckpt = take(t.n_ckpt * 24 * N);
  t.seg = take((int64_t)(K + (has_plastic(c) ? 1 : 0)) * 24 * N);
  t.adj = take(24 * N);
  t.adjc = take(24 * N);
  t.gl = take(N);
  t.gn = take(N);
  t.lnE = take(N);
  t.nu = take(N);
  t.vhb = reinterpret_cast<float4*>(take(4 * c->nodes));
  t.grids = reinterpret_cast<float4*>(take((int64_t)K * 4 * c->nodes));
  t.boxes = reinterpret_cast<int*>(take((int64_t)K * 6 * (c->max_chunks + 1)));
  t.bytes = (size_t)(p - static_cast<char*>(base));
  return t;
}

// Whether any material has a return map: the backward then also reverses
// the return maps, which needs the segment's states one substep further
// (one more tape slot) to form each F_trial from F_k and C_{k+1}.
bool has_plastic(mpm_ctx c) {
  for (int k = 0; k < c->n_mat; ++k)
    if (c->mats[k].plastic != MPM_PLASTIC_NONE) return true;
  return false;
}

int copy_f32(mpm_ctx c, float* out, const float* in, int64_t count, hipStream_t s) {
  if (count <= 0) return MPM_OK;
  fmpm::k_copy_f32<<<blocks_for(count, 256), 256, 0, s>>>(out, in, count);
  LAUNCH_CHECK(c, "k_copy_f32");
  return MPM_OK;
}

// internal state (x, v, C, F planes) -> caller-order 24-plane block
int scatter_state(mpm_ctx c, float* out24, hipStream_t s) {
  const int64_t N = c->N;
  int rc = perm_prepare(c, c->pid, s);
  const float* const in[4] = {c->xs, c->vs, c->Cs, c->Fs};
  float* const out[4] = {out24, out24 + 3 * N, out24 + 6 * N, out24 + 15 * N};
  return rc ? rc : perm_apply(c, state_planes(in, out, N), s);
}

// Workgroups of the persistent adjoint G2P (default mode): it fits three per
// CU where the forward kernels fit two, so 1.5 times the forward's count (at
// most one per work item)
unsigned adj_g2p_blocks(mpm_ctx c) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(c->max_chunks, ((int64_t)c->grid_blocks * 3 + 1) / 2));
}

// Deterministic mode: the scenes' bounds (bank) from the per-item bounds of
// the launch before, each scene flagged where its scales differ from those
// of bank prev (NULL: none is)
int fold_bounds(mpm_ctx c, unsigned* bank, const unsigned* prev, hipStream_t s) {
  fmpm::k_fx_fold<<<(unsigned)c->B, fmpm::kFoldThreads, 0, s>>>(c->fxi, c->dchunk_start, c->scene_item, bank, prev,
                                                                c->fxk);
  LAUNCH_CHECK(c, "k_fx_fold");
  return MPM_OK;
}

// One substep kernel with arguments a.  In deterministic mode a launch
// that scatters (P2G) takes this substep's bounds into bank cur and leaves
// the grid in a.grid_out through the fixed-point grid:
//  - the first such launch of a context measures the bounds in a launch of
//    its own, then accumulates at their scales;
//  - later ones accumulate at the scales of the bounds in the other bank
//    (the previous launch's) while measuring, then scatter again, from the
//    state the launch stored, every scene whose measured scales differ (a
//    P2G-only launch that returns at once when none does).
template <int MODE>
int launch_args(mpm_ctx c, fmpm::SubstepArgs a, hipStream_t s, bool rotation = false) {
  if constexpr (MODE != fmpm::kG2P) {
    if (rotation && c->sparse) {  // the rotation's buffers carry block flags
      a.clear_nodes = c->nodes;
      fmpm::k_substep<MODE, fmpm::kDetOff, true><<<c->grid_blocks, kBlock, 0, s>>>(a);
      LAUNCH_CHECK(c, "k_substep");
      return MPM_OK;
    }
  }
  if (MODE == fmpm::kG2P || !c->det) {
    fmpm::k_substep<MODE><<<c->grid_blocks, kBlock, 0, s>>>(a);  // persistent: items from the queue
    LAUNCH_CHECK(c, "k_substep");
    return MPM_OK;
  }
  if constexpr (MODE != fmpm::kG2P) {
    const int64_t B4 = 4 * (int64_t)c->B;
    unsigned* const cur = c->fxb + B4 * c->fx_bank;
    unsigned* const prev = c->fxb + B4 * (1 - c->fx_bank);
    a.fxk = c->fxk;
    a.gfx = c->gfx;
    a.fxi = c->fxi;
    a.gflag = c->gflag;
    const unsigned fx_blocks = (unsigned)((c->nblocks + 3) / 4);  // k_fx_grid_blocks: four blocks per workgroup
    if (!c->fx_primed) {
      fmpm::SubstepArgs m = a;  // reads the state, writes nothing but the bounds
      m.grid_clear = nullptr;
      m.clear_nodes = 0;
      m.box_out = nullptr;
      m.write_vc = 0;
      fmpm::k_substep<MODE, fmpm::kDetMeasure><<<c->grid_blocks, kBlock, 0, s>>>(m);
      LAUNCH_CHECK(c, "k_substep measure");
      int rc = fold_bounds(c, cur, nullptr, s);
      if (rc) return rc;
      a.fxb = cur;
      fmpm::k_substep<MODE, fmpm::kDetAccumulate><<<c->grid_blocks, kBlock, 0, s>>>(a);
      LAUNCH_CHECK(c, "k_substep accumulate");
      fmpm::k_fx_grid_blocks<<<fx_blocks, 256, 0, s>>>(c->gfx, nullptr, a.grid_out, c->gflag, c->nblocks, c->nb, c->n,
                                                       cur, c->fxk);
      LAUNCH_CHECK(c, "k_fx_grid_blocks");
    } else {
      a.fxb = prev;
      if (MODE == fmpm::kFused) a.write_vc = 1;  // a scatter again reads v and C
      fmpm::k_substep<MODE, fmpm::kDetPredict><<<c->grid_blocks, kBlock, 0, s>>>(a);
      LAUNCH_CHECK(c, "k_substep predict");
      int rc = fold_bounds(c, cur, prev, s);
      if (rc) return rc;
      fmpm::SubstepArgs r = a;  // the P2G of the stored state, at the measured scales, into gfx2
      if (MODE == fmpm::kFused) {
        r.x = a.xo;
        r.v = a.vo;
        r.C = a.Co;
        r.F = a.Fo;
      }
      r.grid_in = nullptr;
      r.grid_clear = nullptr;
      r.clear_nodes = 0;
      r.box_in = nullptr;
      r.box_out = nullptr;
      r.write_vc = 0;
      r.fxb = cur;
      r.gfx = c->gfx2;
      fmpm::k_substep<fmpm::kP2G, fmpm::kDetRedo><<<c->grid_blocks, kBlock, 0, s>>>(r);
      LAUNCH_CHECK(c, "k_substep rescale");
      fmpm::k_fx_grid_blocks<<<fx_blocks, 256, 0, s>>>(c->gfx, c->gfx2, a.grid_out, c->gflag, c->nblocks, c->nb, c->n,
                                                       cur, c->fxk);
      LAUNCH_CHECK(c, "k_fx_grid_blocks");
    }
    c->fx_bank ^= 1;
    c->fx_primed = true;
  }
  return MPM_OK;
}

template <int MODE>
int launch_substep(mpm_ctx c, const float4* gin, float4* gout, int write_vc, hipStream_t s,
                   float4* gclear = nullptr, const int* box_in = nullptr, int* box_out = nullptr) {
  fmpm::SubstepArgs a = make_args(c);
  a.grid_in = gin;
  a.grid_out = gout;
  a.write_vc = write_vc;
  a.grid_clear = gclear;
  a.clear_nodes = gclear ? c->nodes : 0;
  a.box_in = box_in;
  a.box_out = box_out;
  ProfScope ps(c, s, MODE == fmpm::kFused ? 0 : (MODE == fmpm::kP2G ? 1 : 2));
  return launch_args<MODE>(c, a, s, true);
}

int check_particles(mpm_ctx ctx, const mpm_particles* p) {
  if (!p) return fail(ctx, MPM_EINVAL, "particles is NULL");
  if (ctx->N == 0) return MPM_OK;
  if (!p->x || !p->v || !p->C || !p->F || !p->mass || !p->vol0 || !p->log_E || !p->nu || !p->mat_id)
    return fail(ctx, MPM_EINVAL, "a particle array is NULL");
  return MPM_OK;
}

// Sizes derived from the configuration (shared by mpm_workspace_size and mpm_init).
struct Geometry {
  bool det = false, sparse = false;
  int n = 0, nb = 0, B = 1;
  int64_t N = 0, nodes = 0, bins = 0, n_bsum = 0, nblocks = 0, max_chunks = 0, chunk_cap = 0;
};

// Host-side checks of the configuration and the batch offsets (off receives
// them); MPM_EINVAL on any violation.
int check_config(const mpm_config* cfg, int64_t n_particles, const int64_t* batch_offsets, std::vector<int64_t>* off,
                 Geometry* g) {
  if (!cfg) return MPM_EINVAL;
  if (cfg->abi_version != MPM_ABI_VERSION) return MPM_EINVAL;
  if (cfg->grid_res < 8 || cfg->grid_res > 1024) return MPM_EINVAL;
  if (cfg->bound < 0 || 2 * cfg->bound + 3 > cfg->grid_res) return MPM_EINVAL;
  if (cfg->n_batch < 1) return MPM_EINVAL;
  if (!(cfg->dt > 0.0f) || !std::isfinite(cfg->dt)) return MPM_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(cfg->gravity[k])) return MPM_EINVAL;
  const uint32_t known = MPM_FLAG_DETERMINISTIC | MPM_FLAG_GRID_SPARSE | MPM_FLAG_GRID_DENSE;
  if (cfg->sort_every < 0 || (cfg->flags & ~known) != 0) return MPM_EINVAL;
  if ((cfg->flags & MPM_FLAG_GRID_SPARSE) && (cfg->flags & (MPM_FLAG_GRID_DENSE | MPM_FLAG_DETERMINISTIC)))
    return MPM_EINVAL;
  if (n_particles < 0 || n_particles > (int64_t)0x7fffff00) return MPM_EINVAL;
  if (off) {
    if (batch_offsets) {
      off->assign(batch_offsets, batch_offsets + cfg->n_batch + 1);
    } else {
      if (cfg->n_batch != 1) return MPM_EINVAL;
      *off = {0, n_particles};
    }
    if ((*off)[0] != 0 || off->back() != n_particles) return MPM_EINVAL;
    for (int b = 0; b < cfg->n_batch; ++b)
      if ((*off)[b + 1] < (*off)[b]) return MPM_EINVAL;
  }
  g->det = (cfg->flags & MPM_FLAG_DETERMINISTIC) != 0;
  g->B = cfg->n_batch;
  g->n = cfg->grid_res;
  g->nb = (g->n + 3) / 4;
  g->N = n_particles;
  g->bins = (int64_t)cfg->n_batch * g->nb * g->nb * g->nb * 64;
  if (g->bins >= ((int64_t)1 << 32)) return MPM_EINVAL;
  g->n_bsum = (g->bins + fmpm::kScanTile - 1) / fmpm::kScanTile;
  g->nodes = (int64_t)cfg->n_batch * g->n * g->n * g->n;
  g->nblocks = (int64_t)cfg->n_batch * g->nb * g->nb * g->nb;
  // block-sparse clearing: asked for, or by default where the grid has
  // more than 4 nodes per particle (the deterministic mode stays dense)
  g->sparse = (cfg->flags & MPM_FLAG_GRID_SPARSE) ||
              (!(cfg->flags & (MPM_FLAG_GRID_DENSE | MPM_FLAG_DETERMINISTIC)) && g->nodes > 4 * n_particles);
  g->max_chunks = (n_particles + 63) / 64 + std::min<int64_t>(n_particles, g->nblocks) + 1;  // items >= 64
  g->chunk_cap = (n_particles + kBlock - 1) / kBlock + cfg->n_batch;  // per-scene chunks of kBlock
  return MPM_OK;
}

// Points the context's device buffers into the workspace at base (or, with
// base NULL, only measures); returns the bytes used.  Every buffer starts
// on a 256-byte boundary.
size_t carve(mpm_ctx c, const Geometry& g, char* base) {
  size_t off = 0;
  auto take = [&](auto& ptr, int64_t count) {
    using T = std::remove_pointer_t<std::remove_reference_t<decltype(ptr)>>;
    const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    if (base) ptr = reinterpret_cast<T*>(base + off);
    off += (bytes + 255) & ~(size_t)255;
  };
  const int64_t N = std::max<int64_t>(g.N, 1);
  take(c->xs, 3 * N);
  take(c->vs, 3 * N);
  take(c->Cs, 9 * N);
  take(c->Fs, 9 * N);
  take(c->xs2, 3 * N);
  take(c->Fs2, 9 * N);
  take(c->prm, N);
  take(c->prm2, N);
  take(c->mat, N);
  take(c->mat2, N);
  take(c->pid, N);
  take(c->pid2, N);
  take(c->perm, N);
  take(c->keys, N);
  take(c->slots, N);
  for (int k = 0; k < 3; ++k) take(c->grid[k], g.nodes + (g.nblocks + 3) / 4);  // nodes, then block flags
  take(c->done_counter, 1);
  take(c->item_box, 2 * 6 * (g.max_chunks + 1));
  take(c->count, g.bins);
  take(c->bsum, g.n_bsum);
  take(c->chunk_start, g.chunk_cap + 1);
  take(c->chunk_batch, g.chunk_cap);
  take(c->diag, kDiagSlots);
  take(c->dchunk_start, g.max_chunks + 1);
  take(c->dchunk_batch, g.max_chunks + 1);
  take(c->dn_chunks, 1);
  take(c->nchk, g.nblocks);
  take(c->work_counter, 1);
  take(c->d_mats, fmpm::kMaxMaterials);
  if (g.det) {
    take(c->gfx, 4 * g.nodes);
    take(c->gfx2, 4 * g.nodes);
    take(c->fxb, 12 * (int64_t)g.B);
    take(c->fxi, g.max_chunks + 1);
    take(c->scene_item, (int64_t)g.B + 1);
    take(c->gflag, g.nblocks);
    take(c->fxk, g.B);
    take(c->perm2, N);
  }
  const PermGeom pg = perm_geom(N);
  take(c->pdest, N);
  if (pg.bucketed) {
    take(c->ppos, N);
    take(c->pdop, N);
    take(c->ptmp, (int64_t)fmpm::PlaneSet::kMax * N);
    take(c->pcount, pg.entries);
    take(c->pbsum, (pg.entries + fmpm::kScanTile - 1) / fmpm::kScanTile);
  }
  return off;
}

}  // namespace

extern "C" {

const char* mpm_status_string(int status) {
  if (status > 0 || status < -6) return "unknown status";
  return kStatusText[-status];
}

const char* mpm_last_error(mpm_ctx ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

int mpm_workspace_size(const mpm_config* cfg, int64_t n_particles, size_t* bytes) {
  if (!bytes) return MPM_EINVAL;
  Geometry g;
  const int rc = check_config(cfg, n_particles, nullptr, nullptr, &g);
  if (rc) return rc;
  mpm_context tmp;
  *bytes = carve(&tmp, g, nullptr);
  return MPM_OK;
}

int mpm_init(const mpm_config* cfg, const mpm_material* materials, int32_t n_materials, int64_t n_particles,
             const int64_t* batch_offsets, void* workspace, size_t workspace_bytes, mpm_ctx* out) {
  if (!out) return MPM_EINVAL;
  *out = nullptr;
  if (!cfg || !materials) return MPM_EINVAL;
  std::vector<int64_t> off;
  Geometry g;
  int rc = check_config(cfg, n_particles, batch_offsets, &off, &g);
  if (rc) return rc;
  if (n_materials < 1 || n_materials > fmpm::kMaxMaterials) return MPM_EINVAL;
  fmpm::Material mats[fmpm::kMaxMaterials]{};
  for (int k = 0; k < n_materials; ++k) {
    const mpm_material& m = materials[k];
    if (m.elastic < MPM_ELASTIC_FCR || m.elastic > MPM_ELASTIC_VOLUME) return MPM_EINVAL;
    if (m.plastic < MPM_PLASTIC_NONE || m.plastic > MPM_PLASTIC_SIGMA) return MPM_EINVAL;
    if (m.plastic == MPM_PLASTIC_VON_MISES && !(m.yield_stress > 0.0f)) return MPM_EINVAL;
    if (m.plastic == MPM_PLASTIC_DRUCKER_PRAGER && !(m.friction_deg > 0.0f && m.friction_deg < 90.0f))
      return MPM_EINVAL;
    mats[k].elastic = m.elastic;
    mats[k].plastic = m.plastic;
    mats[k].yield_stress = m.yield_stress;
    const double sp = std::sin((double)m.friction_deg * M_PI / 180.0);
    mats[k].dp_alpha = (float)(std::sqrt(2.0 / 3.0) * 2.0 * sp / (3.0 - sp));
  }
  if (!workspace || ((uintptr_t)workspace & 255u)) return MPM_EINVAL;
  mpm_context probe;
  const size_t need = carve(&probe, g, nullptr);
  if (workspace_bytes < need) return MPM_ENOMEM;

  mpm_ctx c = new mpm_context();
  c->cfg = *cfg;
  c->n_mat = n_materials;
  std::memcpy(c->mats, mats, sizeof(mats));
  c->N = n_particles;
  c->B = cfg->n_batch;
  c->offsets = off;
  c->n = g.n;
  c->nb = g.nb;
  c->nodes = g.nodes;
  c->bins = g.bins;
  c->n_bsum = g.n_bsum;
  if (cfg->sort_every > 0) c->sort_every = cfg->sort_every;
  c->det = g.det;
  c->sparse = g.sparse;

  std::vector<int> cs, cb;
  for (int b = 0; b < c->B; ++b)
    for (int64_t s = off[b]; s < off[b + 1]; s += kBlock) {
      cs.push_back((int)s);
      cb.push_back(b);
    }
  cs.push_back((int)n_particles);
  c->n_chunks = (int)cb.size();
  c->nblocks = g.nblocks;
  c->max_chunks = g.max_chunks;
  c->grid_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(c->max_chunks, 256 * 2));
  c->workspace_bytes = carve(c, g, static_cast<char*>(workspace));

  hipError_t e = hipMemcpy(c->chunk_start, cs.data(), cs.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess && !cb.empty())
    e = hipMemcpy(c->chunk_batch, cb.data(), cb.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(c->diag, 0, kDiagSlots * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemset(c->dn_chunks, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemset(c->done_counter, 0, sizeof(unsigned));
  if (e == hipSuccess) e = hipMemset(c->work_counter, 0, sizeof(int));
  if (e == hipSuccess) e = hipMemcpy(c->d_mats, c->mats, sizeof(c->mats), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_particles > 0) {
    fmpm::k_iota<<<blocks_for(n_particles, 256), 256>>>(c->pid, n_particles);
    e = hipGetLastError();
  }
  for (int k = 0; k < 3 && e == hipSuccess; ++k)  // empty grids, no block flagged
    e = hipMemset(c->grid[k], 0, (size_t)(c->nodes + (g.nblocks + 3) / 4) * sizeof(float4));
  if (e == hipSuccess && c->det) {  // N_b / 2^13 (the range factor's floor); the fixed-point grid at zero
    std::vector<double> k(c->B);
    for (int b = 0; b < c->B; ++b) k[b] = (double)(off[b + 1] - off[b]) / 8192.0;
    e = hipMemcpy(c->fxk, k.data(), k.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(c->gfx, 0, (size_t)c->nodes * 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->gfx2, 0, (size_t)c->nodes * 4 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(c->gflag, 0, (size_t)c->nblocks * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(c->fxb, 0, (size_t)c->B * 12 * sizeof(unsigned));
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    delete c;
    return MPM_EDEVICE;
  }
  *out = c;
  return MPM_OK;
}

}  // extern "C"

namespace {
// The substep loop of mpm_step_n; with write_back = false the caller's
// arrays are only read (the autotuner times trial runs this way).
int run_steps(mpm_ctx ctx, const mpm_particles* p, int32_t n_steps, void* tape, int32_t checkpoint_every,
              void* stream, bool write_back) {
  int rc = MPM_OK;
  if (n_steps < 0) return fail(ctx, MPM_EINVAL, "n_steps < 0");
  if (tape && checkpoint_every < 1) return fail(ctx, MPM_EINVAL, "checkpoint_every < 1 with a tape");
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  ctx->resident = ctx->primed = false;  // the internal state is taken from the caller's arrays
  TapeLayout tl{};
  const int64_t N = ctx->N;
  if (tape) {
    tl = tape_layout(ctx, n_steps, checkpoint_every, tape);
    ctx->tape_ptr = tape;
    ctx->tape_n = n_steps;
    ctx->tape_K = checkpoint_every;
    if (N > 0) {  // checkpoint 0: the caller's state as given
      rc = copy_f32(ctx, tl.ckpt, p->x, 3 * N, s);
      rc = rc ? rc : copy_f32(ctx, tl.ckpt + 3 * N, p->v, 3 * N, s);
      rc = rc ? rc : copy_f32(ctx, tl.ckpt + 6 * N, p->C, 9 * N, s);
      rc = rc ? rc : copy_f32(ctx, tl.ckpt + 15 * N, p->F, 9 * N, s);
      if (rc) return rc;
    }
  } else {
    ctx->tape_ptr = nullptr;
    ctx->tape_n = -1;
  }
  if (n_steps == 0 || ctx->N == 0) {
    ctx->substeps += n_steps;
    return MPM_OK;
  }
  rc = gather_from_caller(ctx, p, s);
  if (rc) return rc;
  // three grids in rotation: substep kernel k reads grid k % 3, writes
  // grid (k + 1) % 3 (zeroed by kernel k - 1) and zeroes grid (k + 2) % 3;
  // each kernel leaves the work-queue head at zero for the next
  // per-item cell boxes in turn: each kernel hands the next one the box of
  // its particles' new cells, so only the first kernel after a sort reads x
  // for it
  int* boxes[2] = {ctx->item_box, ctx->item_box + 6 * (ctx->max_chunks + 1)};
  int bcur = 0;
  rc = fill_u32(ctx, ctx->grid[0], 4 * ctx->nodes, s, 4, ctx->work_counter);
  if (rc) return rc;
  rc = launch_substep<fmpm::kP2G>(ctx, nullptr, ctx->grid[0], 0, s, n_steps > 1 ? ctx->grid[1] : nullptr, nullptr,
                                  boxes[0]);
  if (rc) return rc;
  bool have_box = true;
  int cur = 0;
  for (int st = 0; st < n_steps; ++st) {
    if (st == n_steps - 1) {
      rc = launch_substep<fmpm::kG2P>(ctx, ctx->grid[cur], nullptr, 1, s, nullptr, have_box ? boxes[bcur] : nullptr);
      if (rc) return rc;
    } else {
      const int nxt = (cur + 1) % 3, clr = (cur + 2) % 3;
      const bool ckpt = tape && (st + 1) % checkpoint_every == 0;
      rc = launch_substep<fmpm::kFused>(ctx, ctx->grid[cur], ctx->grid[nxt], ckpt ? 1 : 0, s,
                                        st + 2 < n_steps ? ctx->grid[clr] : nullptr,
                                        have_box ? boxes[bcur] : nullptr, boxes[1 - bcur]);
      if (rc) return rc;
      bcur = 1 - bcur;
      have_box = true;
      cur = nxt;
      if (ckpt) {
        rc = scatter_state(ctx, tl.ckpt + ((st + 1) / checkpoint_every) * 24 * N, s);
        if (rc) return rc;
      }
      if (ctx->sort_every > 0 && (st + 1) % ctx->sort_every == 0) {
        rc = resort_internal(ctx, s);
        if (rc) return rc;
        have_box = false;  // new items: the next kernel reads x for its boxes
      }
    }
  }
  ctx->last_grid = cur;
  ctx->substeps += n_steps;
  return write_back ? scatter_to_caller(ctx, p, s) : MPM_OK;
}
}  // namespace

extern "C" {

int mpm_step_n(mpm_ctx ctx, const mpm_particles* p, int32_t n_steps, void* tape, int32_t checkpoint_every,
               void* stream) {
  if (!ctx) return MPM_EINVAL;
  int rc = check_particles(ctx, p);
  if (rc) return rc;
  return run_steps(ctx, p, n_steps, tape, checkpoint_every, stream, true);
}

int mpm_substep(mpm_ctx ctx, const mpm_particles* p, void* stream) {
  return mpm_step_n(ctx, p, 1, nullptr, 0, stream);
}

int mpm_load(mpm_ctx ctx, const mpm_particles* p, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (ctx->capturing) return fail(ctx, MPM_ESTATE, "resident stepping is not captured into graphs");
  int rc = check_particles(ctx, p);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  ctx->resident = ctx->primed = false;
  if (ctx->N > 0) {
    rc = gather_from_caller(ctx, p, s);
    if (rc) return rc;
  }
  ctx->resident = true;
  ctx->res_since_sort = 0;
  return MPM_OK;
}

int mpm_advance(mpm_ctx ctx, int32_t n_steps, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (n_steps < 0) return fail(ctx, MPM_EINVAL, "n_steps < 0");
  if (ctx->capturing) return fail(ctx, MPM_ESTATE, "resident stepping is not captured into graphs");
  if (!ctx->resident) return fail(ctx, MPM_ESTATE, "no resident state: mpm_load first");
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  if (n_steps == 0 || ctx->N == 0) {
    ctx->substeps += n_steps;
    return MPM_OK;
  }
  int* boxes[2] = {ctx->item_box, ctx->item_box + 6 * (ctx->max_chunks + 1)};
  int rc = MPM_OK;
  if (!ctx->primed) {
    // P2G of the loaded state into grid 0 (zeroed here); grid 1 is zeroed
    // for the first fused kernel
    rc = fill_u32(ctx, ctx->grid[0], 4 * ctx->nodes, s, 4, ctx->work_counter);
    rc = rc ? rc : launch_substep<fmpm::kP2G>(ctx, nullptr, ctx->grid[0], 0, s, ctx->grid[1], nullptr, boxes[0]);
    if (rc) {
      ctx->resident = false;
      return rc;
    }
    ctx->res_cur = 0;
    ctx->res_bcur = 0;
    ctx->res_have_box = true;
    ctx->primed = true;
  }
  // fused substeps only: kernel k reads grid k % 3, writes grid (k + 1) % 3
  // and zeroes grid (k + 2) % 3, and the rotation carries over to the next
  // call.  The last kernel of the call also writes v and C, so the internal
  // state is whole between calls.  A re-sort that falls due is done before
  // the next kernel (the grid does not depend on the particle order).
  int prev = ctx->res_cur;
  for (int st = 0; st < n_steps; ++st) {
    if (ctx->sort_every > 0 && ctx->res_since_sort >= ctx->sort_every) {
      rc = resort_internal(ctx, s);
      if (rc) break;
      ctx->res_since_sort = 0;
      ctx->res_have_box = false;
    }
    const int cur = ctx->res_cur, nxt = (cur + 1) % 3, clr = (cur + 2) % 3;
    rc = launch_substep<fmpm::kFused>(ctx, ctx->grid[cur], ctx->grid[nxt], st == n_steps - 1 ? 1 : 0, s,
                                      ctx->grid[clr], ctx->res_have_box ? boxes[ctx->res_bcur] : nullptr,
                                      boxes[1 - ctx->res_bcur]);
    if (rc) break;
    ctx->res_bcur = 1 - ctx->res_bcur;
    ctx->res_have_box = true;
    prev = cur;
    ctx->res_cur = nxt;
    ++ctx->res_since_sort;
  }
  if (rc) {
    ctx->resident = ctx->primed = false;
    return rc;
  }
  ctx->last_grid = prev;
  ctx->substeps += n_steps;
  return MPM_OK;
}

int mpm_store(mpm_ctx ctx, const mpm_particles* p, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (ctx->capturing) return fail(ctx, MPM_ESTATE, "resident stepping is not captured into graphs");
  if (!p) return fail(ctx, MPM_EINVAL, "particles is NULL");
  if (!ctx->resident) return fail(ctx, MPM_ESTATE, "no resident state: mpm_load first");
  if (ctx->N == 0) return MPM_OK;
  if (!p->x || !p->v || !p->C || !p->F) return fail(ctx, MPM_EINVAL, "a state array is NULL");
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  return scatter_to_caller(ctx, p, s);
}

int mpm_export_frame(mpm_ctx ctx, float* x, const float* cov0, float* cov, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (ctx->capturing) return fail(ctx, MPM_ESTATE, "resident stepping is not captured into graphs");
  if (!ctx->resident) return fail(ctx, MPM_ESTATE, "no resident state: mpm_load first");
  if (!x && !cov) return fail(ctx, MPM_EINVAL, "x and cov are both NULL");
  if (cov && !cov0) return fail(ctx, MPM_EINVAL, "cov without cov0");
  const int64_t N = ctx->N;
  if (N == 0) return MPM_OK;
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  ProfScope ps(ctx, s, 5);
  // x, and F into the re-sort buffer, to caller order in one permutation;
  // then the covariances elementwise in caller order
  int rc = perm_prepare(ctx, ctx->pid, s);
  fmpm::PlaneSet pl{};
  if (x) add_planes(pl, ctx->xs, x, 3, N);
  if (cov) add_planes(pl, ctx->Fs, ctx->Fs2, 9, N);
  rc = rc ? rc : perm_apply(ctx, pl, s);
  if (rc) return rc;
  if (cov) {
    fmpm::k_covariance<<<blocks_for(N, 256), 256, 0, s>>>(ctx->Fs2, cov0, cov, N);
    LAUNCH_CHECK(ctx, "k_covariance");
  }
  return MPM_OK;
}

int mpm_tape_size(mpm_ctx ctx, int32_t n_steps, int32_t checkpoint_every, size_t* bytes) {
  if (!ctx || !bytes || n_steps < 0 || checkpoint_every < 1) return MPM_EINVAL;
  *bytes = tape_layout(ctx, n_steps, checkpoint_every, nullptr).bytes;
  return MPM_OK;
}

int mpm_backward(mpm_ctx ctx, const mpm_particles* p, const void* tape, int32_t n_steps, const float* g_x,
                 const float* g_v, const float* g_C, const float* g_F, float* g_log_E, float* g_nu, float* g_x0,
                 float* g_v0, float* g_C0, float* g_F0, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (!p || !tape || !g_log_E || !g_nu) return fail(ctx, MPM_EINVAL, "NULL argument");
  if (ctx->N > 0 && (!p->mass || !p->vol0 || !p->log_E || !p->nu || !p->mat_id))
    return fail(ctx, MPM_EINVAL, "a parameter array is NULL");
  if (tape != ctx->tape_ptr || n_steps != ctx->tape_n)
    return fail(ctx, MPM_ESTATE, "tape does not hold the last taped mpm_step_n of this length");
  hipStream_t s = (hipStream_t)stream;
  ctx->last_stream = s;
  ctx->resident = ctx->primed = false;  // the recompute overwrites the internal state
  const int64_t N = ctx->N;
  const int K = ctx->tape_K;
  TapeLayout tl = tape_layout(ctx, n_steps, K, const_cast<void*>(tape));
  if (N == 0) return MPM_OK;
  int rc = fill_u32(ctx, g_log_E, N, s);
  rc = rc ? rc : fill_u32(ctx, g_nu, N, s);
  // caller-order adjoint of the final state
  const float* gin[4] = {g_x, g_v, g_C, g_F};
  const int64_t off[4] = {0, 3 * N, 6 * N, 15 * N};
  const int64_t cnt[4] = {3 * N, 3 * N, 9 * N, 9 * N};
  for (int k = 0; k < 4 && !rc; ++k)
    rc = gin[k] ? copy_f32(ctx, tl.adjc + off[k], gin[k], cnt[k], s) : fill_u32(ctx, tl.adjc + off[k], cnt[k], s);
  if (rc) return rc;
  const unsigned gp = blocks_for(N, 256);
  for (int64_t seg = tl.n_ckpt - 1; seg >= 0 && n_steps > 0; --seg) {
    const int k0 = (int)(seg * K);
    const int L = std::min(K, n_steps - k0);
    if (L <= 0) continue;
    const float* ck = tl.ckpt + seg * 24 * N;
    // (1) sort the checkpoint, gather state and parameters into sorted order
    rc = sort_keys(ctx, ck, s);
    if (rc) return rc;
    auto slot = [&](int j) { return tl.seg + (int64_t)j * 24 * N; };
    fmpm::k_invert<<<gp, 256, 0, s>>>(ctx->perm, ctx->pdest, N);  // caller index -> slot
    LAUNCH_CHECK(ctx, "k_invert");
    rc = perm_prepare(ctx, ctx->pdest, s);
    fmpm::PlaneSet pk{};
    add_planes(pk, ck, slot(0), 24, N);
    float* const pl[5] = {ctx->Fs2, ctx->Fs2 + N, tl.lnE, tl.nu, ctx->Fs2 + 2 * N};
    add_params(pk, p, pl);
    rc = rc ? rc : perm_apply(ctx, pk, s);
    if (rc) return rc;
    fmpm::k_params_planes<<<gp, 256, 0, s>>>(ctx->prm, ctx->mat, ctx->pid, pl[0], pl[1], pl[2], pl[3], pl[4],
                                              ctx->perm, N, ctx->diag);
    LAUNCH_CHECK(ctx, "backward gather");
    // (2) recompute the segment: slot j holds the state of substep k0 + j
    // and grid slot j its P2G (the grid the forward pass read at that
    // substep); the fused kernel reads slot j and grid j, writes slot j + 1
    // and grid j + 1
    auto args_for = [&](int j_in, int j_out) {
      fmpm::SubstepArgs a = make_args(ctx);
      float* si = slot(j_in);
      float* so = slot(j_out);
      a.x = si;
      a.v = si + 3 * N;
      a.C = si + 6 * N;
      a.F = si + 15 * N;
      a.xo = so;
      a.vo = so + 3 * N;
      a.Co = so + 6 * N;
      a.Fo = so + 15 * N;
      return a;
    };
    auto gslot = [&](int j) { return tl.grids + (int64_t)j * ctx->nodes; };
    rc = fill_u32(ctx, gslot(0), 4 * ctx->nodes, s, -1, ctx->work_counter);
    if (rc) return rc;
    // each kernel also records the item boxes of the state it produces,
    // which the next kernel and the two adjoint kernels of that state reuse
    auto bslot = [&](int j) { return tl.boxes + (int64_t)j * 6 * (ctx->max_chunks + 1); };
    // each launch also zeroes the grid slot the launch after it writes
    // (slot 0 is filled above); the kernels reset the item queue themselves
    {
      fmpm::SubstepArgs a = args_for(0, 0);
      a.grid_out = gslot(0);
      a.box_out = bslot(0);
      if (L > 1) {
        a.grid_clear = gslot(1);
        a.clear_nodes = ctx->nodes;
      }
      rc = launch_args<fmpm::kP2G>(ctx, a, s);
      if (rc) return rc;
    }
    for (int j = 0; j + 1 < L; ++j) {
      fmpm::SubstepArgs a = args_for(j, j + 1);
      a.grid_in = gslot(j);
      a.grid_out = gslot(j + 1);
      a.box_in = bslot(j);
      a.box_out = bslot(j + 1);
      a.write_vc = 1;
      if (j + 2 < L) {
        a.grid_clear = gslot(j + 2);
        a.clear_nodes = ctx->nodes;
      }
      rc = launch_args<fmpm::kFused>(ctx, a, s);
      if (rc) return rc;
    }
    // with return maps: the state after the segment's last substep as well
    // (slot L), whose C forms that substep's F_trial
    const bool plastic = has_plastic(ctx);
    if (plastic) {
      fmpm::SubstepArgs a = args_for(L - 1, L);
      a.grid_in = gslot(L - 1);
      a.box_in = bslot(L - 1);
      rc = launch_args<fmpm::kG2P>(ctx, a, s);
      if (rc) return rc;
    }
    // (3) adjoint of the segment's final state, in sorted order, through
    // the permutation (1) prepared (caller index -> slot; the recompute
    // leaves it in place)
    rc = perm_block(ctx, tl.adjc, tl.adj, 24, s);
    rc = rc ? rc : fill_u32(ctx, tl.gl, N, s);
    rc = rc ? rc : fill_u32(ctx, tl.gn, N, s);
    if (rc) return rc;
    // (4) reverse the substeps of the segment
    for (int j = L - 1; j >= 0; --j) {
      const float* st = slot(j);
      rc = fill_u32(ctx, tl.vhb, 4 * ctx->nodes, s, -1, ctx->work_counter);
      if (rc) return rc;
      fmpm::AdjArgs b{};
      b.x = st;
      b.v = st + 3 * N;
      b.C = st + 6 * N;
      b.F = st + 15 * N;
      b.prm = ctx->prm;
      b.lnE = tl.lnE;
      b.nu = tl.nu;
      b.N = N;
      b.chunk_start = ctx->chunk_start;
      b.chunk_batch = ctx->chunk_batch;
      b.grid = gslot(j);
      b.vhb = tl.vhb;
      b.ax = tl.adj;
      b.av = tl.adj + 3 * N;
      b.aC = tl.adj + 6 * N;
      b.aF = tl.adj + 15 * N;
      b.g_lnE = tl.gl;
      b.g_nu = tl.gn;
      b.mat = ctx->mat;
      b.mats = ctx->d_mats;
      b.n_materials = ctx->n_mat;
      b.n = ctx->n;
      b.bound = ctx->cfg.bound;
      b.dt = ctx->cfg.dt;
      for (int k = 0; k < 3; ++k) b.g[k] = ctx->cfg.gravity[k];
      fmpm::AdjItems items{ctx->dchunk_start, ctx->dchunk_batch, ctx->dn_chunks, ctx->work_counter, ctx->tile_cap,
                           bslot(j)};
      if (plastic) {  // adjoint of F_{j+1} -> adjoint of F_trial
        fmpm::k_adj_return_map<<<gp, 256, 0, s>>>(b.x, b.F, slot(j + 1) + 6 * N, ctx->prm, ctx->mat, ctx->d_mats,
                                                   ctx->n_mat, tl.lnE, tl.nu, ctx->cfg.dt, ctx->n, b.aF, tl.gl,
                                                   tl.gn, N);
        LAUNCH_CHECK(ctx, "k_adj_return_map");
      }
      if (ctx->det) {  // exact sums of the grid-velocity adjoint at one scale per scene
        ProfScope pa(ctx, s, 6);
        unsigned* const bank = ctx->fxb + 8 * (int64_t)ctx->B;  // the adjoint's bound bank
        b.fxb = bank;
        b.fxi = ctx->fxi;
        b.gflag = ctx->gflag;
        b.fxk = ctx->fxk;
        b.gfx = ctx->gfx;
        fmpm::k_adj_bound<<<(unsigned)std::max<int64_t>(ctx->max_chunks, 1), 256, 0, s>>>(b, items);
        LAUNCH_CHECK(ctx, "k_adj_bound");
        rc = fold_bounds(ctx, bank, nullptr, s);
        if (rc) return rc;
        fmpm::k_adj_g2p<true><<<ctx->grid_blocks, kBlock, 0, s>>>(b, items);
        LAUNCH_CHECK(ctx, "k_adj_g2p");
        fmpm::k_fx_grid_blocks<<<(unsigned)((ctx->nblocks + 3) / 4), 256, 0, s>>>(
            ctx->gfx, nullptr, tl.vhb, ctx->gflag, ctx->nblocks, ctx->nb, ctx->n, bank, ctx->fxk);
      } else {
        ProfScope pa(ctx, s, 6);
        fmpm::k_adj_g2p<<<adj_g2p_blocks(ctx), kBlock, 0, s>>>(b, items);
      }
      LAUNCH_CHECK(ctx, "k_adj_g2p");
      rc = fill_u32(ctx, ctx->work_counter, 1, s);  // the item queue again, for k_adj_p2g
      if (rc) return rc;
      {
        ProfScope pa(ctx, s, 7);
        fmpm::k_adj_p2g<<<ctx->grid_blocks, kBlock, 0, s>>>(b, items);
      }
      LAUNCH_CHECK(ctx, "k_adj_p2g");
    }
    // (5) back to caller order (slot j -> caller index pid[j]); the
    // parameter gradients go through the sort's free key and slot buffers
    {
      float* gl_c = reinterpret_cast<float*>(ctx->keys);
      float* gn_c = reinterpret_cast<float*>(ctx->slots);
      rc = perm_prepare(ctx, ctx->pid, s);
      fmpm::PlaneSet pg{};
      add_planes(pg, tl.adj, tl.adjc, 24, N);
      add_planes(pg, tl.gl, gl_c, 1, N);
      add_planes(pg, tl.gn, gn_c, 1, N);
      rc = rc ? rc : perm_apply(ctx, pg, s);
      if (rc) return rc;
      fmpm::k_add2<<<gp, 256, 0, s>>>(g_log_E, gl_c, g_nu, gn_c, N);
      LAUNCH_CHECK(ctx, "adjoint to caller order");
    }
  }
  float* gout[4] = {g_x0, g_v0, g_C0, g_F0};
  for (int k = 0; k < 4 && !rc; ++k)
    if (gout[k]) rc = copy_f32(ctx, gout[k], tl.adjc + off[k], cnt[k], s);
  return rc;
}

int mpm_grid_state(mpm_ctx ctx, float* m, float* mv, float* v, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (ctx->last_grid < 0) return fail(ctx, MPM_ESTATE, "no substep has run");
  hipStream_t s = (hipStream_t)stream;
  fmpm::SubstepArgs a = make_args(ctx);
  fmpm::k_grid_export<<<blocks_for(ctx->nodes, 256), 256, 0, s>>>(ctx->grid[ctx->last_grid], ctx->nodes, a, m, mv, v);
  LAUNCH_CHECK(ctx, "k_grid_export");
  return MPM_OK;
}

int mpm_export_covariance(mpm_ctx ctx, const float* F, const float* cov0, float* cov, int64_t n, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (n < 0) return fail(ctx, MPM_EINVAL, "n < 0");
  if (n == 0) return MPM_OK;
  if (!F || !cov0 || !cov) return fail(ctx, MPM_EINVAL, "NULL array");
  fmpm::k_covariance<<<blocks_for(n, 256), 256, 0, (hipStream_t)stream>>>(F, cov0, cov, n);
  LAUNCH_CHECK(ctx, "k_covariance");
  return MPM_OK;
}

int mpm_get_diagnostics(mpm_ctx ctx, mpm_diag* out) {
  if (!ctx || !out) return MPM_EINVAL;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  unsigned long long h[kDiagSlots];
  HIP_TRY(ctx, hipMemcpy(h, ctx->diag, sizeof(h), hipMemcpyDeviceToHost));
  out->nonfinite = (int64_t)h[0];
  out->out_of_grid = (int64_t)h[1];
  out->tile_overflow = (int64_t)h[2];
  out->tile_escapes = (int64_t)h[3];
  out->substeps = ctx->substeps;
  out->cfl_violations = (int64_t)h[4];
  const double scale = (double)ctx->cfg.dt * (double)ctx->n;  // dt / dx
  float v2, c2;
  const uint32_t b5 = (uint32_t)h[5], b6 = (uint32_t)h[6];
  std::memcpy(&v2, &b5, 4);
  std::memcpy(&c2, &b6, 4);
  out->max_cfl = std::sqrt((double)v2) * scale;
  out->max_wave_cfl = std::sqrt((double)c2) * scale;
  out->order_fallbacks = (int64_t)h[7];
  out->det_rescales = (int64_t)h[8];
  return (h[0] || h[1] || h[4]) ? MPM_EUNSTABLE : MPM_OK;
}

int mpm_set_tuning(mpm_ctx ctx, const mpm_tuning* t) {
  if (!ctx || !t) return MPM_EINVAL;
  if (t->chunk != 0 && (t->chunk < 64 || t->chunk > 8192 || t->chunk % 64 != 0)) return fail(ctx, MPM_EINVAL, "chunk");
  if (t->sort_every < 0) return fail(ctx, MPM_EINVAL, "sort_every < 0");
  if (t->tile_cap != 0 && (t->tile_cap < 27 || t->tile_cap > fmpm::kTileCapMax)) return fail(ctx, MPM_EINVAL, "tile_cap");
  if (t->workgroups != 0 && (t->workgroups < 1 || t->workgroups > 65536)) return fail(ctx, MPM_EINVAL, "workgroups");
  if (t->sort_every > 0) ctx->sort_every = t->sort_every;
  if (t->tile_cap > 0) ctx->tile_cap = t->tile_cap;
  if (t->chunk > 0) ctx->item = t->chunk;  // takes effect at the next sort
  if (t->workgroups > 0) ctx->grid_blocks = t->workgroups;
  return MPM_OK;
}

int mpm_get_tuning(mpm_ctx ctx, mpm_tuning* t) {
  if (!ctx || !t) return MPM_EINVAL;
  t->chunk = ctx->item;
  t->sort_every = ctx->sort_every;
  t->tile_cap = ctx->tile_cap;
  t->workgroups = ctx->grid_blocks;
  t->ms_per_substep = 0.0;
  return MPM_OK;
}

int mpm_autotune(mpm_ctx ctx, const mpm_particles* p, int32_t trial_steps, void* stream, mpm_tuning* best) {
  if (!ctx || !best) return MPM_EINVAL;
  int rc = check_particles(ctx, p);
  if (rc) return rc;
  if (trial_steps < 2) return fail(ctx, MPM_EINVAL, "trial_steps < 2");
  hipStream_t s = (hipStream_t)stream;
  mpm_tuning cur{};
  mpm_get_tuning(ctx, &cur);
  if (ctx->N == 0) {
    *best = cur;
    return MPM_OK;
  }
  hipEvent_t e0, e1;
  HIP_TRY(ctx, hipEventCreate(&e0));
  HIP_TRY(ctx, hipEventCreate(&e1));
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  const int64_t saved_substeps = ctx->substeps;
  // time one setting: a warm-up run, then the timed run (both on internal copies)
  auto trial = [&](const mpm_tuning& t, double* ms) -> int {
    int r = mpm_set_tuning(ctx, &t);
    r = r ? r : run_steps(ctx, p, trial_steps, nullptr, 0, stream, false);
    if (r) return r;
    if (hipEventRecord(e0, s) != hipSuccess) return MPM_EDEVICE;
    r = run_steps(ctx, p, trial_steps, nullptr, 0, stream, false);
    if (r) return r;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return MPM_EDEVICE;
    float f = 0.f;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return MPM_EDEVICE;
    *ms = f / trial_steps;
    return MPM_OK;
  };
  mpm_tuning bt = cur;
  double bms = 0.0;
  rc = trial(bt, &bms);
  // coordinate descent: work-item size, then workgroups, then sort interval
  const int chunks[] = {256, 512, 768, 1024, 1536, 2048};
  const int wgs[] = {256, 512, 768, 1024, 2048};
  const int sorts[] = {2, 4, 8, 16, 32, 64};
  for (int c : chunks) {
    if (rc) break;
    mpm_tuning t = bt;
    t.chunk = c;
    double ms;
    rc = trial(t, &ms);
    if (!rc && ms < bms) { bt = t; bms = ms; }
  }
  for (int w : wgs) {
    if (rc) break;
    mpm_tuning t = bt;
    t.workgroups = w;
    double ms;
    rc = trial(t, &ms);
    if (!rc && ms < bms) { bt = t; bms = ms; }
  }
  for (int so : sorts) {
    if (rc) break;
    if (so >= 2 * trial_steps) break;  // one interval beyond the trial: no re-sort inside a call
    mpm_tuning t = bt;
    t.sort_every = so;
    double ms;
    rc = trial(t, &ms);
    if (!rc && ms < bms) { bt = t; bms = ms; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->prof_on = prof;
  ctx->substeps = saved_substeps;
  if (rc) {
    mpm_set_tuning(ctx, &cur);
    return rc;
  }
  bt.ms_per_substep = bms;
  mpm_set_tuning(ctx, &bt);
  *best = bt;
  return MPM_OK;
}

struct mpm_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  mpm_ctx ctx = nullptr;
};

int mpm_graph_begin(mpm_ctx ctx, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (!stream) return fail(ctx, MPM_EINVAL, "capture needs a non-null stream");
  if (ctx->capturing) return fail(ctx, MPM_ESTATE, "already capturing");
  ctx->prof_saved = ctx->prof_on;
  ctx->prof_on = false;  // no event records inside a graph
  HIP_TRY(ctx, hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  return MPM_OK;
}

int mpm_graph_end(mpm_ctx ctx, void* stream, mpm_graph* out) {
  if (!ctx || !out) return MPM_EINVAL;
  *out = nullptr;
  if (!ctx->capturing) return fail(ctx, MPM_ESTATE, "not capturing");
  ctx->capturing = false;
  ctx->prof_on = ctx->prof_saved;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture((hipStream_t)stream, &graph);
  if (e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_fail(ctx, "hipStreamEndCapture", e);
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ctx, "hipGraphInstantiate", e);
  }
  mpm_graph g = new mpm_graph_s();
  g->graph = graph;
  g->exec = exec;
  g->ctx = ctx;
  *out = g;
  return MPM_OK;
}

int mpm_position_loss_grad(mpm_ctx ctx, const float* x, const float* x_target, const float* weight, float* g_x,
                           void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (ctx->N == 0) return MPM_OK;
  if (!x || !x_target || !weight || !g_x) return fail(ctx, MPM_EINVAL, "NULL array");
  fmpm::k_position_loss_grad<<<blocks_for(ctx->N, 256), 256, 0, (hipStream_t)stream>>>(x, x_target, weight, g_x,
                                                                                       ctx->N);
  LAUNCH_CHECK(ctx, "k_position_loss_grad");
  return MPM_OK;
}

int mpm_bgdo_accumulate(mpm_ctx ctx, const mpm_particles* key, const float* F_next, float delta_target,
                        float* g_total, float* s_out, float* delta_out, void* stream) {
  if (!ctx || !key) return MPM_EINVAL;
  if (!std::isfinite(delta_target)) return fail(ctx, MPM_EINVAL, "delta_target");
  if (ctx->N == 0) return MPM_OK;
  if (!key->F || !key->log_E || !key->nu || !key->mat_id || !F_next || !g_total)
    return fail(ctx, MPM_EINVAL, "NULL array");
  fmpm::k_bgdo_accumulate<<<blocks_for(ctx->N, 256), 256, 0, (hipStream_t)stream>>>(
      key->F, F_next, key->log_E, key->nu, key->mat_id, ctx->d_mats, ctx->n_mat, delta_target, g_total, s_out,
      delta_out, ctx->N);
  LAUNCH_CHECK(ctx, "k_bgdo_accumulate");
  return MPM_OK;
}

int mpm_bgdo_apply(mpm_ctx ctx, float* log_E, const float* g_total, int32_t n_keys, void* stream) {
  if (!ctx) return MPM_EINVAL;
  if (n_keys < 1) return fail(ctx, MPM_EINVAL, "n_keys < 1");
  if (ctx->N == 0) return MPM_OK;
  if (!log_E || !g_total) return fail(ctx, MPM_EINVAL, "NULL array");
  fmpm::k_bgdo_apply<<<blocks_for(ctx->N, 256), 256, 0, (hipStream_t)stream>>>(log_E, g_total, 1.0f / (float)n_keys,
                                                                               ctx->N);
  LAUNCH_CHECK(ctx, "k_bgdo_apply");
  return MPM_OK;
}

int mpm_graph_launch(mpm_graph g, void* stream) {
  if (!g) return MPM_EINVAL;
  g->ctx->resident = g->ctx->primed = false;  // a replay rewrites the internal state
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? MPM_OK : MPM_EDEVICE;
}

int mpm_graph_destroy(mpm_graph g) {
  if (!g) return MPM_EINVAL;
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return MPM_OK;
}

int mpm_profile(mpm_ctx ctx, int32_t enable) {
  if (!ctx) return MPM_EINVAL;
  if (enable && ctx->prof_ev.empty()) {
    ctx->prof_ev.resize(2 * kProfPairs);
    for (auto& e : ctx->prof_ev) HIP_TRY(ctx, hipEventCreate(&e));
  }
  ctx->prof_on = enable != 0;
  return MPM_OK;
}

int mpm_profile_read(mpm_ctx ctx, double* ms, int64_t* launches) {
  if (!ctx || !ms || !launches) return MPM_EINVAL;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->last_stream));
  for (size_t i = 0; i < ctx->prof_cls.size(); ++i) {
    if (ctx->prof_cls[i] < 0) continue;
    float t = 0.f;
    HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->prof_ev[2 * i], ctx->prof_ev[2 * i + 1]));
    ctx->prof_ms[ctx->prof_cls[i]] += t;
    ctx->prof_cnt[ctx->prof_cls[i]] += 1;
  }
  ctx->prof_cls.clear();
  for (int k = 0; k < MPM_PROFILE_CLASSES; ++k) {
    ms[k] = ctx->prof_ms[k];
    launches[k] = ctx->prof_cnt[k];
    ctx->prof_ms[k] = 0.0;
    ctx->prof_cnt[k] = 0;
  }
  return MPM_OK;
}

int mpm_destroy(mpm_ctx ctx) {
  if (!ctx) return MPM_EINVAL;
  (void)hipDeviceSynchronize();
  for (auto& e : ctx->prof_ev) (void)hipEventDestroy(e);
  delete ctx;
  return MPM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// MCIS interior filling (context-free; the caller supplies the workspace)
// ---------------------------------------------------------------------------
namespace {

struct McisLayout {
  fmpm::McisGrid g;
  int64_t fine_cells = 0, coarse_cells = 0;  // over all instances
  size_t so = 0, co = 0, out_off = 0, prefix = 0, rank = 0, start = 0, bsum_start = 0, coarse = 0, skey = 0,
         sslot = 0, sorted = 0, cstart = 0, ckey = 0, cslot = 0, corder = 0, okey = 0, eq = 0, sel = 0, bsum_m = 0,
         hist = 0, bad = 0, total = 0;
};

constexpr int64_t kMcisMaxCells = (int64_t)1 << 27;  // per cell array (0.5 GB of uint32)

// Workspace layout for K instances, S surface points, M candidates; the
// fine grid is the finest (most rings per search radius, at most
// kMcisRings) within the cell budget and, when max_bytes is nonzero, within
// max_bytes of workspace.  The search result does not depend on the rings.
int mcis_layout(int32_t K, int64_t S, int64_t M, double sigma, double eps, McisLayout& L, size_t max_bytes = 0);

int mcis_layout_rings(int32_t K, int64_t S, int64_t M, double rs, int rings, McisLayout& L) {
  L.g.hc = rs * (1.0 + 1e-9);
  L.g.r2 = rs * rs;
  L.g.gc = (int)std::max(1.0, std::ceil(1.0 / L.g.hc));
  L.coarse_cells = (int64_t)K * L.g.gc * L.g.gc * L.g.gc;
  L.g.rings = rings;
  L.g.hf = rs * (1.0 + 1e-9) / rings;
  L.g.gf = (int)std::max(1.0, std::ceil(1.0 / L.g.hf));
  L.fine_cells = (int64_t)K * L.g.gf * L.g.gf * L.g.gf;
  if (L.fine_cells >= kMcisMaxCells || L.coarse_cells >= kMcisMaxCells) return MPM_EINVAL;  // sigma too small
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const int64_t nb_start = (L.fine_cells + 2 + fmpm::kScanTile - 1) / fmpm::kScanTile;
  const int64_t nb_m = (M + fmpm::kScanTile - 1) / fmpm::kScanTile;
  L.so = take(8 * (size_t)(K + 1));
  L.co = take(8 * (size_t)(K + 1));
  L.out_off = take(8 * (size_t)K);
  L.prefix = take(8 * (size_t)K);
  L.rank = take(8 * (size_t)K);
  L.start = take(4 * (size_t)(L.fine_cells + 1));
  L.bsum_start = take(4 * (size_t)std::max<int64_t>(nb_start, 1));
  L.coarse = take(4 * (size_t)L.coarse_cells);
  L.skey = take(4 * (size_t)std::max<int64_t>(S, 1));
  L.sslot = take(4 * (size_t)std::max<int64_t>(S, 1));
  L.sorted = take(16 * (size_t)std::max<int64_t>(S, 1));
  L.cstart = take(4 * (size_t)(L.fine_cells + 2));  // one more bin for out-of-domain candidates
  L.ckey = take(4 * (size_t)std::max<int64_t>(M, 1));
  L.cslot = take(4 * (size_t)std::max<int64_t>(M, 1));
  L.corder = take(4 * (size_t)std::max<int64_t>(M, 1));
  L.okey = take(8 * (size_t)std::max<int64_t>(M, 1));
  L.eq = take(4 * (size_t)std::max<int64_t>(M, 1));
  L.sel = take(4 * (size_t)std::max<int64_t>(M, 1));
  L.bsum_m = take(4 * (size_t)std::max<int64_t>(nb_m, 1));
  L.hist = take(4 * 256 * (size_t)K);
  L.bad = take(8);
  L.total = off;
  return MPM_OK;
}

int mcis_layout(int32_t K, int64_t S, int64_t M, double sigma, double eps, McisLayout& L, size_t max_bytes) {
  if (K < 1 || S < 0 || M < 0 || M >= ((int64_t)1 << 32) || S >= ((int64_t)1 << 32)) return MPM_EINVAL;
  if (!(sigma > 0.0) || !(eps > 0.0 && eps < 1.0) || !std::isfinite(sigma)) return MPM_EINVAL;
  const double rs = sigma * std::sqrt(-2.0 * std::log(eps)) * (1.0 + 1e-9);
  int rc = MPM_EINVAL;
  for (int rings = fmpm::kMcisRings; rings >= 1; --rings) {
    rc = mcis_layout_rings(K, S, M, rs, rings, L);
    if (rc == MPM_OK && (max_bytes == 0 || L.total <= max_bytes)) return MPM_OK;
  }
  return max_bytes && rc == MPM_OK ? MPM_ENOMEM : MPM_EINVAL;
}

#define MCIS_TRY(call)                                  \
  do {                                                  \
    if ((call) != hipSuccess) {                         \
      (void)hipGetLastError();                          \
      return MPM_EDEVICE;                               \
    }                                                   \
  } while (0)

int mcis_fill(void* p, int64_t count, hipStream_t s) {
  if (count <= 0) return MPM_OK;
  const int64_t n4 = std::max<int64_t>(count >> 2, 4);
  fmpm::k_fill_u32<<<blocks_for(n4, 256), 256, 0, s>>>((uint32_t*)p, 0u, count, nullptr);
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EDEVICE;
}

int mcis_scan(uint32_t* data, uint32_t* bsum, int64_t n, hipStream_t s) {
  const int64_t nb = (n + fmpm::kScanTile - 1) / fmpm::kScanTile;
  fmpm::k_scan_reduce<<<(unsigned)nb, fmpm::kScanThreads, 0, s>>>(data, bsum, n);
  fmpm::k_scan_top<<<1, fmpm::kScanThreads, 0, s>>>(bsum, nb);
  fmpm::k_scan_apply<<<(unsigned)nb, fmpm::kScanThreads, 0, s>>>(data, bsum, n);
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EDEVICE;
}

}  // namespace

int mpm_mcis_workspace_size(int32_t n_instances, int64_t n_surface, int64_t n_candidates, double sigma, double eps,
                            size_t* bytes) {
  if (!bytes) return MPM_EINVAL;
  McisLayout L;
  const int rc = mcis_layout(n_instances, n_surface, n_candidates, sigma, eps, L);
  if (rc) return rc;
  *bytes = L.total;
  return MPM_OK;
}

namespace {

// MCIS steps 1-5 on `workspace` (layout L); out_off, prefix, rank are host
// arrays of K int64 (see mcis_prepare).
int mcis_run(int32_t K, const float* surface, const int64_t* surface_offsets, const float* candidates,
             const int64_t* candidate_offsets, const double* u, double sigma, double eps, const McisLayout& L,
             void* workspace, const int64_t* out_off, const int64_t* prefix, const int64_t* rank, int64_t* out_index,
             double* d_out, hipStream_t s);

// Host checks of the per-instance counts; fills each instance's output
// offset and the start of its radix select (prefix, rank).
int mcis_prepare(int32_t K, const int64_t* surface_offsets, const int64_t* candidate_offsets, const int64_t* n_select,
                 int64_t* out_off, int64_t* prefix, int64_t* rank) {
  int64_t total_sel = 0;
  for (int k = 0; k < K; ++k) {
    const int64_t ns = surface_offsets[k + 1] - surface_offsets[k], nc = candidate_offsets[k + 1] - candidate_offsets[k];
    if (ns < 0 || nc < 0 || n_select[k] < 0 || n_select[k] > nc) return MPM_EINVAL;
    out_off[k] = total_sel;
    total_sel += n_select[k];
    if (n_select[k] == 0) {  // nothing: a threshold above every key
      prefix[k] = (int64_t)~0ull;
      rank[k] = 0;
    } else if (n_select[k] == nc) {  // everything: every valid key is above 0
      prefix[k] = 0;
      rank[k] = 0;
    } else {
      prefix[k] = 0;
      rank[k] = n_select[k];
    }
  }
  return MPM_OK;
}

int mcis_run(int32_t K, const float* surface, const int64_t* surface_offsets, const float* candidates,
             const int64_t* candidate_offsets, const double* u, double sigma, double eps, const McisLayout& L,
             void* workspace, const int64_t* out_off, const int64_t* prefix, const int64_t* rank, int64_t* out_index,
             double* d_out, hipStream_t s) {
  const int64_t S = surface_offsets[K], M = candidate_offsets[K];
  int rc = MPM_OK;
  char* w = static_cast<char*>(workspace);
  auto at = [&](size_t o) { return static_cast<void*>(w + o); };
  int64_t* d_so = (int64_t*)at(L.so);
  int64_t* d_co = (int64_t*)at(L.co);
  int64_t* d_out_off = (int64_t*)at(L.out_off);
  uint64_t* d_prefix = (uint64_t*)at(L.prefix);
  int64_t* d_rank = (int64_t*)at(L.rank);
  uint32_t* d_start = (uint32_t*)at(L.start);
  uint32_t* d_coarse = (uint32_t*)at(L.coarse);
  uint32_t* d_skey = (uint32_t*)at(L.skey);
  uint32_t* d_sslot = (uint32_t*)at(L.sslot);
  float4* d_sorted = (float4*)at(L.sorted);
  uint64_t* d_okey = (uint64_t*)at(L.okey);
  uint32_t* d_eq = (uint32_t*)at(L.eq);
  uint32_t* d_sel = (uint32_t*)at(L.sel);
  uint32_t* d_hist = (uint32_t*)at(L.hist);
  unsigned long long* d_bad = (unsigned long long*)at(L.bad);
  uint32_t* d_cstart = (uint32_t*)at(L.cstart);
  uint32_t* d_corder = (uint32_t*)at(L.corder);

  MCIS_TRY(hipMemcpyAsync(d_so, surface_offsets, 8 * (size_t)(K + 1), hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_co, candidate_offsets, 8 * (size_t)(K + 1), hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_out_off, out_off, 8 * (size_t)K, hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_prefix, prefix, 8 * (size_t)K, hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_rank, rank, 8 * (size_t)K, hipMemcpyHostToDevice, s));
  if ((rc = mcis_fill(d_start, L.fine_cells + 1, s)) || (rc = mcis_fill(d_cstart, L.fine_cells + 2, s)) ||
      (rc = mcis_fill(d_coarse, L.coarse_cells, s)) ||
      (rc = mcis_fill(d_hist, 256 * (int64_t)K, s)) || (rc = mcis_fill(d_bad, 2, s)))
    return rc;
  // surface points into fine-cell order
  if (S > 0) {
    fmpm::k_mcis_bin_surface<<<blocks_for(S, 256), 256, 0, s>>>(surface, S, d_so, K, L.g, d_start, d_coarse, d_skey,
                                                                d_sslot, d_bad);
    MCIS_TRY(hipGetLastError());
  }
  if ((rc = mcis_scan(d_start, (uint32_t*)at(L.bsum_start), L.fine_cells + 1, s))) return rc;
  if (S > 0) {
    fmpm::k_mcis_place_surface<<<blocks_for(S, 256), 256, 0, s>>>(surface, S, d_skey, d_sslot, d_start, d_sorted);
    MCIS_TRY(hipGetLastError());
  }
  // candidates into fine-cell order
  fmpm::k_mcis_bin_candidates<<<blocks_for(M, 256), 256, 0, s>>>(candidates, M, d_co, K, L.g, d_cstart,
                                                                 (uint32_t*)at(L.ckey), (uint32_t*)at(L.cslot));
  MCIS_TRY(hipGetLastError());
  if ((rc = mcis_scan(d_cstart, (uint32_t*)at(L.bsum_start), L.fine_cells + 2, s))) return rc;
  fmpm::k_mcis_place_candidates<<<blocks_for(M, 256), 256, 0, s>>>(M, (uint32_t*)at(L.ckey), (uint32_t*)at(L.cslot),
                                                                   d_cstart, d_corder);
  MCIS_TRY(hipGetLastError());
  // steps 1, 2 and the keys
  fmpm::k_mcis_keys<<<blocks_for(M, 256), 256, 0, s>>>(candidates, M, d_co, K, u, L.g, sigma, eps, d_coarse, d_start,
                                                       d_sorted, d_corder, d_okey, d_out, d_bad);
  MCIS_TRY(hipGetLastError());
  // radix select of each instance's n-th largest key, 8 digits of 8 bits
  const unsigned hist_blocks = (unsigned)std::min<int64_t>((M + fmpm::kMcisChunk - 1) / fmpm::kMcisChunk, 2048);
  for (int shift = 56; shift >= 0; shift -= 8) {
    fmpm::k_mcis_hist<<<hist_blocks, 256, 0, s>>>(d_okey, M, d_co, K, d_prefix, d_rank, shift, d_hist);
    fmpm::k_mcis_pick<<<blocks_for(K, 64), 64, 0, s>>>(K, shift, d_hist, d_prefix, d_rank);
    MCIS_TRY(hipGetLastError());
  }
  // ties by index, then ordered compaction
  fmpm::k_mcis_eq<<<blocks_for(M, 256), 256, 0, s>>>(d_okey, M, d_co, K, d_prefix, d_eq);
  MCIS_TRY(hipGetLastError());
  if ((rc = mcis_scan(d_eq, (uint32_t*)at(L.bsum_m), M, s))) return rc;
  fmpm::k_mcis_sel<<<blocks_for(M, 256), 256, 0, s>>>(d_okey, M, d_co, K, d_prefix, d_rank, d_eq, d_sel);
  MCIS_TRY(hipGetLastError());
  if ((rc = mcis_scan(d_sel, (uint32_t*)at(L.bsum_m), M, s))) return rc;
  fmpm::k_mcis_write<<<blocks_for(M, 256), 256, 0, s>>>(d_okey, M, d_co, K, d_prefix, d_rank, d_eq, d_sel, d_out_off,
                                                        out_index);
  MCIS_TRY(hipGetLastError());
  unsigned long long bad = 0;
  MCIS_TRY(hipMemcpyAsync(&bad, d_bad, 8, hipMemcpyDeviceToHost, s));
  MCIS_TRY(hipStreamSynchronize(s));
  return bad ? MPM_EINVAL : MPM_OK;
}

}  // namespace

int mpm_mcis_select(int32_t n_instances, const float* surface, const int64_t* surface_offsets,
                    const float* candidates, const int64_t* candidate_offsets, const double* u,
                    const int64_t* n_select, double sigma, double eps, void* workspace, size_t workspace_bytes,
                    int64_t* out_index, double* d_out, void* stream) {
  const int K = n_instances;
  if (K < 1 || !surface_offsets || !candidate_offsets || !n_select) return MPM_EINVAL;
  const int64_t S = surface_offsets[K], M = candidate_offsets[K];
  if (surface_offsets[0] != 0 || candidate_offsets[0] != 0) return MPM_EINVAL;
  std::vector<int64_t> out_off(K), prefix(K), rank(K);
  int rc = mcis_prepare(K, surface_offsets, candidate_offsets, n_select, out_off.data(), prefix.data(), rank.data());
  if (rc) return rc;
  McisLayout L;
  rc = mcis_layout(K, S, M, sigma, eps, L);
  if (rc) return rc;
  if (M == 0) return MPM_OK;
  if (!candidates || !u || !out_index || (S > 0 && !surface)) return MPM_EINVAL;
  if (!workspace || workspace_bytes < L.total) return MPM_EINVAL;
  return mcis_run(K, surface, surface_offsets, candidates, candidate_offsets, u, sigma, eps, L, workspace,
                  out_off.data(), prefix.data(), rank.data(), out_index, d_out, (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Candidate generation for the interior fill (context-free; the caller
// supplies the workspace)
// ---------------------------------------------------------------------------
namespace {

struct IpfLayout {
  int64_t cells = 0, refs = 0;  // capacities
  size_t ro = 0, hv_off = 0, ht_off = 0, box = 0, grid = 0, tri = 0, count = 0, cursor = 0, refs_at = 0,
         per_grid = 0, bsum = 0, qbuf = 0, ccount = 0, ccursor = 0, order = 0, par = 0, flag = 0, offsets = 0,
         bad = 0, total = 0;
};

constexpr int kIpfMaxSide = 1024;  // cells per side of a triangle grid

// Cells per side of instance grids with T_k triangles: the smallest g with
// 2 g^2 >= T_k (at most kIpfMaxSide), so g^2 <= T_k + 2.
int ipf_side(int64_t tk) {
  int64_t g = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt(0.5 * (double)tk)));
  while (g > 1 && 2 * (g - 1) * (g - 1) >= tk) --g;
  while (2 * g * g < tk) ++g;
  return (int)std::min<int64_t>(g, kIpfMaxSide);
}

// References a grid may hold before its side is halved.
int64_t ipf_ref_budget(int64_t tk) { return 8 * tk + 64; }

int ipf_layout(int32_t K, int64_t V, int64_t T, int64_t R, IpfLayout& L) {
  if (K < 1 || K > (1 << 20) || V < 0 || T < 0 || R < 0 || V >= ((int64_t)1 << 31) || T > ((int64_t)1 << 27) ||
      R >= ((int64_t)1 << 30))
    return MPM_EINVAL;
  L.cells = 3 * (T + 2 * (int64_t)K);        // sum over grids of g^2 <= T_k + 2
  L.refs = 24 * T + 192 * (int64_t)K;        // sum over grids of the budget
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += (bytes + 255) & ~(size_t)255;
    return at;
  };
  const int64_t nb = (std::max(L.cells, R) + 1 + fmpm::kScanTile - 1) / fmpm::kScanTile;
  L.ro = take(8 * (size_t)(K + 1));
  L.hv_off = take(8 * (size_t)(K + 1));
  L.ht_off = take(8 * (size_t)(K + 1));
  L.box = take(4 * 6 * (size_t)K);
  L.grid = take(sizeof(fmpm::IpfGrid) * 3 * (size_t)K);
  L.tri = take(sizeof(fmpm::IpfTri) * (size_t)std::max<int64_t>(T, 1));
  L.count = take(4 * (size_t)(L.cells + 1));
  L.cursor = take(4 * (size_t)L.cells);
  L.refs_at = take(4 * (size_t)L.refs);
  L.per_grid = take(8 * 3 * (size_t)K);
  L.bsum = take(4 * (size_t)std::max<int64_t>(nb, 1));
  L.qbuf = take(16 * (size_t)std::max<int64_t>(R, 1));
  L.ccount = take(4 * (size_t)(L.cells + 1));
  L.ccursor = take(4 * (size_t)L.cells);
  L.order = take(4 * 3 * (size_t)std::max<int64_t>(R, 1));
  L.par = take(3 * (size_t)std::max<int64_t>(R, 1));
  L.flag = take(4 * (size_t)(R + 1));
  L.offsets = take(4 * (size_t)(K + 1));
  L.bad = take(8);
  L.total = off;
  return MPM_OK;
}

bool ipf_offsets_ok(const int64_t* off, int K, int64_t total) {
  if (off[0] != 0 || off[K] != total) return false;
  for (int k = 0; k < K; ++k)
    if (off[k + 1] < off[k]) return false;
  return true;
}

// u32 fill on the device (the kernels' counters and flags start at zero)
int ipf_fill(void* p, int64_t count, uint32_t v, hipStream_t s) {
  if (count <= 0) return MPM_OK;
  const int64_t n4 = std::max<int64_t>(count >> 2, 4);
  fmpm::k_fill_u32<<<blocks_for(n4, 256), 256, 0, s>>>((uint32_t*)p, v, count, nullptr);
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EDEVICE;
}

}  // namespace

int mpm_ipf_workspace_size(int32_t n_instances, int64_t n_hull_vertices, int64_t n_hull_triangles, int64_t n_raw,
                           size_t* bytes) {
  if (!bytes) return MPM_EINVAL;
  IpfLayout L;
  const int rc = ipf_layout(n_instances, n_hull_vertices, n_hull_triangles, n_raw, L);
  if (rc) return rc;
  *bytes = L.total;
  return MPM_OK;
}

int mpm_ipf_candidates(int32_t n_instances, const float* hull_vertices, const int64_t* hull_vertex_offsets,
                       const int32_t* hull_triangles, const int64_t* hull_triangle_offsets, const double* u,
                       const int64_t* raw_offsets, double occupancy_threshold, void* workspace,
                       size_t workspace_bytes, float* candidates_out, int64_t* source_out,
                       int64_t* candidate_offsets_out, void* stream) {
  const int K = n_instances;
  if (K < 1 || !hull_vertex_offsets || !hull_triangle_offsets || !raw_offsets || !candidate_offsets_out)
    return MPM_EINVAL;
  const int64_t V = hull_vertex_offsets[K], T = hull_triangle_offsets[K], R = raw_offsets[K];
  IpfLayout L;
  int rc = ipf_layout(K, V, T, R, L);
  if (rc) return rc;
  if (!ipf_offsets_ok(hull_vertex_offsets, K, V) || !ipf_offsets_ok(hull_triangle_offsets, K, T) ||
      !ipf_offsets_ok(raw_offsets, K, R))
    return MPM_EINVAL;
  if (!(occupancy_threshold >= 0.0 && occupancy_threshold <= 1.0)) return MPM_EINVAL;
  for (int k = 0; k <= K; ++k) candidate_offsets_out[k] = 0;
  if (R == 0 || T == 0) return MPM_OK;  // no candidates, or no hull: nothing is kept
  if (!hull_vertices || !hull_triangles || !u || !candidates_out) return MPM_EINVAL;
  if (!workspace || workspace_bytes < L.total) return MPM_EINVAL;
  const hipStream_t s = (hipStream_t)stream;
  char* w = static_cast<char*>(workspace);
  auto at = [&](size_t o) { return static_cast<void*>(w + o); };
  int64_t* d_ro = (int64_t*)at(L.ro);
  int64_t* d_hv_off = (int64_t*)at(L.hv_off);
  int64_t* d_ht_off = (int64_t*)at(L.ht_off);
  uint32_t* d_box = (uint32_t*)at(L.box);
  fmpm::IpfGrid* d_grid = (fmpm::IpfGrid*)at(L.grid);
  fmpm::IpfTri* d_tri = (fmpm::IpfTri*)at(L.tri);
  uint32_t* d_count = (uint32_t*)at(L.count);
  uint32_t* d_cursor = (uint32_t*)at(L.cursor);
  uint32_t* d_refs = (uint32_t*)at(L.refs_at);
  unsigned long long* d_per_grid = (unsigned long long*)at(L.per_grid);
  uint32_t* d_bsum = (uint32_t*)at(L.bsum);
  float4* d_qbuf = (float4*)at(L.qbuf);
  uint32_t* d_ccount = (uint32_t*)at(L.ccount);
  uint32_t* d_ccursor = (uint32_t*)at(L.ccursor);
  uint32_t* d_order = (uint32_t*)at(L.order);
  uint8_t* d_par = (uint8_t*)at(L.par);
  uint32_t* d_flag = (uint32_t*)at(L.flag);
  uint32_t* d_offsets = (uint32_t*)at(L.offsets);
  unsigned long long* d_bad = (unsigned long long*)at(L.bad);

  MCIS_TRY(hipMemcpyAsync(d_ro, raw_offsets, 8 * (size_t)(K + 1), hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_hv_off, hull_vertex_offsets, 8 * (size_t)(K + 1), hipMemcpyHostToDevice, s));
  MCIS_TRY(hipMemcpyAsync(d_ht_off, hull_triangle_offsets, 8 * (size_t)(K + 1), hipMemcpyHostToDevice, s));
  // boxes: min at +inf, max at 0 (as float bits)
  fmpm::k_ipf_box_init<<<blocks_for(6 * (int64_t)K, 256), 256, 0, s>>>(d_box, K);
  MCIS_TRY(hipGetLastError());
  if ((rc = ipf_fill(d_bad, 2, 0u, s))) return rc;
  fmpm::k_ipf_tris<<<blocks_for(T, 256), 256, 0, s>>>(hull_vertices, V, hull_triangles, T, d_hv_off, d_ht_off, K,
                                                      d_tri, d_box, d_bad);
  MCIS_TRY(hipGetLastError());
  // triangle grids: halve the side of any grid whose references exceed its
  // budget, until every grid fits (a side of 1 always does)
  std::vector<int> side(3 * (size_t)K);
  for (int k = 0; k < K; ++k)
    side[3 * k] = side[3 * k + 1] = side[3 * k + 2] =
        ipf_side(hull_triangle_offsets[k + 1] - hull_triangle_offsets[k]);
  std::vector<fmpm::IpfGrid> grid(3 * (size_t)K);
  std::vector<unsigned long long> per_grid(3 * (size_t)K);
  int64_t cells = 0;
  for (;;) {
    cells = 0;
    for (int i = 0; i < 3 * K; ++i) {
      grid[i].g = side[i];
      grid[i].base = (uint32_t)cells;
      cells += (int64_t)side[i] * side[i];
    }
    MCIS_TRY(hipMemcpyAsync(d_grid, grid.data(), sizeof(fmpm::IpfGrid) * 3 * (size_t)K, hipMemcpyHostToDevice, s));
    if ((rc = ipf_fill(d_count, cells + 1, 0u, s)) || (rc = ipf_fill(d_per_grid, 6 * (int64_t)K, 0u, s))) return rc;
    fmpm::k_ipf_bin<false><<<blocks_for(T, 256), 256, 0, s>>>(d_tri, T, d_ht_off, K, d_box, d_grid, d_count,
                                                                   d_per_grid, nullptr, nullptr, nullptr);
    MCIS_TRY(hipGetLastError());
    MCIS_TRY(hipMemcpyAsync(per_grid.data(), d_per_grid, 8 * 3 * (size_t)K, hipMemcpyDeviceToHost, s));
    MCIS_TRY(hipStreamSynchronize(s));
    bool fits = true;
    for (int i = 0; i < 3 * K; ++i) {
      const int64_t tk = hull_triangle_offsets[i / 3 + 1] - hull_triangle_offsets[i / 3];
      if ((int64_t)per_grid[i] > ipf_ref_budget(tk) && side[i] > 1) {
        side[i] = std::max(1, side[i] / 2);
        fits = false;
      }
    }
    if (fits) break;
  }
  if ((rc = mcis_scan(d_count, d_bsum, cells + 1, s))) return rc;
  if ((rc = ipf_fill(d_cursor, cells, 0u, s))) return rc;
  fmpm::k_ipf_bin<true><<<blocks_for(T, 256), 256, 0, s>>>(d_tri, T, d_ht_off, K, d_box, d_grid, nullptr,
                                                                nullptr, d_count, d_cursor, d_refs);
  MCIS_TRY(hipGetLastError());
  // raw candidates into column order per axis, ray parities column by
  // column, then the occupancy of every raw candidate
  if ((rc = ipf_fill(d_ccount, cells + 1, 0u, s)) || (rc = ipf_fill(d_ccursor, cells, 0u, s))) return rc;
  fmpm::k_ipf_points<<<blocks_for(R, 256), 256, 0, s>>>(u, R, d_ro, K, d_box, d_grid, d_qbuf, d_ccount, d_bad);
  MCIS_TRY(hipGetLastError());
  if ((rc = mcis_scan(d_ccount, d_bsum, cells + 1, s))) return rc;
  fmpm::k_ipf_columns<<<blocks_for(R, 256), 256, 0, s>>>(d_qbuf, R, d_box, d_grid, d_ccount, d_ccursor, d_order);
  MCIS_TRY(hipGetLastError());
  fmpm::k_ipf_rays<<<blocks_for(3 * R, 256), 256, 0, s>>>(d_qbuf, R, d_box, d_grid, d_count, d_refs, d_tri,
                                                          d_order, d_ccount + cells, d_par);
  MCIS_TRY(hipGetLastError());
  if ((rc = ipf_fill(d_flag + R, 1, 0u, s))) return rc;
  fmpm::k_ipf_flags<<<blocks_for(R, 256), 256, 0, s>>>(d_qbuf, R, d_par, occupancy_threshold, d_flag);
  MCIS_TRY(hipGetLastError());
  if ((rc = mcis_scan(d_flag, d_bsum, R + 1, s))) return rc;
  fmpm::k_ipf_offsets<<<blocks_for(K + 1, 64), 64, 0, s>>>(d_flag, d_ro, K, d_offsets);
  MCIS_TRY(hipGetLastError());
  std::vector<uint32_t> offs(K + 1);
  unsigned long long bad = 0;
  MCIS_TRY(hipMemcpyAsync(offs.data(), d_offsets, 4 * (size_t)(K + 1), hipMemcpyDeviceToHost, s));
  MCIS_TRY(hipMemcpyAsync(&bad, d_bad, 8, hipMemcpyDeviceToHost, s));
  MCIS_TRY(hipStreamSynchronize(s));
  if (bad) return MPM_EINVAL;
  const int64_t M_in = offs[K];
  if (M_in > 0) {
    fmpm::k_ipf_write<<<blocks_for(R, 256), 256, 0, s>>>(d_qbuf, R, d_flag, M_in, candidates_out, source_out);
    MCIS_TRY(hipGetLastError());
    MCIS_TRY(hipStreamSynchronize(s));
  }
  for (int k = 0; k <= K; ++k) candidate_offsets_out[k] = offs[k];
  return MPM_OK;
}

// ---------------------------------------------------------------------------
// MCIS without allocation (mpm_mcis_select_static): the workspace is a
// file-scope device array of fixed size.  Its host-side name is only a
// stand-in; the device address comes from hipGetSymbolAddress, looked up
// once per device on the first call there, and is what the kernels get.
// ---------------------------------------------------------------------------
constexpr size_t kMcisStaticBytes = (size_t)64 << 20;  // per device
constexpr int kMcisStaticMaxInstances = 256;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kMcisStaticBytes];

namespace {

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
int static_scratch(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return MPM_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MPM_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MPM_OK;
}

}  // namespace

int mpm_mcis_select_static(int32_t n_instances, const float* surface, const int64_t* surface_offsets,
                           const float* candidates, const int64_t* candidate_offsets, const double* u,
                           const int64_t* n_select, double sigma, double eps, int64_t* out_index, double* d_out,
                           void* stream) {
  const int K = n_instances;
  if (K < 1 || K > kMcisStaticMaxInstances || !surface_offsets || !candidate_offsets || !n_select)
    return MPM_EINVAL;
  const int64_t S = surface_offsets[K], M = candidate_offsets[K];
  if (surface_offsets[0] != 0 || candidate_offsets[0] != 0) return MPM_EINVAL;
  int64_t out_off[kMcisStaticMaxInstances], prefix[kMcisStaticMaxInstances], rank[kMcisStaticMaxInstances];
  int rc = mcis_prepare(K, surface_offsets, candidate_offsets, n_select, out_off, prefix, rank);
  if (rc) return rc;
  McisLayout L;
  rc = mcis_layout(K, S, M, sigma, eps, L, kMcisStaticBytes);  // MPM_ENOMEM beyond the fixed scratch
  if (rc) return rc;
  if (M == 0) return MPM_OK;
  if (!candidates || !u || !out_index || (S > 0 && !surface)) return MPM_EINVAL;
  void* ws = nullptr;
  rc = static_scratch(&ws);
  if (rc) return rc;
  return mcis_run(K, surface, surface_offsets, candidates, candidate_offsets, u, sigma, eps, L, ws, out_off, prefix,
                  rank, out_index, d_out, (hipStream_t)stream);
}
