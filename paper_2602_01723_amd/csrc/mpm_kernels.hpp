// HIP kernels of the MLS-MPM substep (included once, by fastmpm.hip) for gfx950 (wave64, LDS, FP32 atomics,
// FP64 SVD).  See fastmpm.h for the operation and its citations.
//
// Layout
//   particles (sorted, internal)  SoA planes: x[3][N], v[3][N], C[9][N], F[9][N]
//                                  prm[N] = float4(mass, vol0, mu, lam), mat[N], pid[N]
//   grid                           float4 (mv.x, mv.y, mv.z, m) per node, scene-major,
//                                  node (ix, iy, iz) of scene b at ((b*n+ix)*n+iy)*n+iz
//   chunks                         workgroup c owns particles [chunk_start[c], chunk_start[c+1]),
//                                  all of scene chunk_batch[c]
//
// One substep = stress -> P2G -> grid update -> G2P -> return map.  The
// pipeline fuses G2P of substep s, the return map, the stress and P2G of
// substep s+1 into one kernel (k_substep<kFused>): v and C never leave
// registers.  The grid update is folded into the G2P tile load.  P2G
// accumulates in an LDS tile (64-bit fixed point, integer atomics) covering
// the chunk's stencil box with staggered per-lane node order (lanes of one
// cell hit different nodes), then flushes the tile with one global FP32
// atomic per node and channel.
// Chunks whose box exceeds the LDS tile fall back to global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_math.hpp"

namespace fmpm {

constexpr int kPadX = 3;            // P2G tile x-stride padding (nodes), spreads LDS banks
constexpr int kBlock = 256;         // threads per workgroup = particles per chunk
constexpr int kTileCapMax = 1331;   // LDS tile nodes (11^3): P2G 4 x 64 bits + G2P 3 floats per node
constexpr int kMaxMaterials = 16;

enum { kP2G = 0, kFused = 1, kG2P = 2 };

struct SubstepArgs {
  // particle state read by the kernel (plane stride N) ...
  float* x;
  float* v;
  float* C;
  float* F;
  // ... and where it writes the new state (the same arrays, or other ones)
  float* xo;
  float* vo;
  float* Co;
  float* Fo;
  const float4* prm;
  const int* mat;
  int64_t N;  // plane stride
  const int* chunk_start;  // [n_chunks + 1]
  const int* chunk_batch;  // [n_chunks]
  const int* n_chunks;     // device scalar: number of work items
  int* work_counter;       // device scalar, zero at launch
  const float4* grid_in;
  float4* grid_out;
  int n;
  int bound;
  float dt;
  float g[3];
  int tile_cap;
  int write_vc;  // fused mode: also store v and C
  unsigned long long* diag;
  int n_materials;
  const Material* mats;  // device table [n_materials]
  // a grid buffer this launch neither reads nor writes, zeroed for the
  // launch after next (NULL: none), and the node count of a grid buffer
  float4* grid_clear;
  int64_t clear_nodes;
  // workgroups finished; the last one resets it and the queue head, so the
  // next launch needs no counter reset (NULL: the caller resets the queue)
  unsigned* done_counter;
  // per-item base-cell boxes [item][lo xyz, hi xyz]: box_in, when set, is the
  // box of the particles' current cells (skips the box pass); box_out, when
  // set, receives a box containing the cells after this substep
  const int* box_in;
  int* box_out;
  // CFL watch: G2P velocities with |v'|^2 above cfl_v2 (|v'| dt / dx > 1/2)
  // are counted in diag[4]; the largest |v'|^2 goes to diag[5]
  float cfl_v2;
  int n_scenes;  // scenes (grids) of the context
  // deterministic mode (k_substep<MODE, kDet...>).  A bound bank holds, per
  // scene b, [4 b + 0 / 1] the largest P2G contribution bound (momentum,
  // mass; float bits) and [4 b + 2] the particle count of the largest work
  // item, [4 b + 3] whether the scales of these bounds differ from the
  // ones predicted (k_fx_fold forms the bank from fxi).  fxb: the bank the
  // fixed-point scales are taken from; fxi: a measuring or predicting
  // launch's largest bounds per work item; fxk[b] = N_b / 2^13; gfx the
  // 64-bit fixed-point grid [node][4] the launch adds into
  unsigned* fxb;
  float2* fxi;
  const double* fxk;
  unsigned long long* gfx;
  // deterministic accumulation: one flag per 4^3-node block of gfx (the
  // layout of the sparse grid's flags), set for every block the launch adds
  // into, so the conversion visits only those blocks
  unsigned* gflag;
};

// Deterministic mode.  The P2G of a substep runs twice: a measuring launch
// computes every particle's contribution bound and keeps each scene's
// largest, B_b; the accumulating launch then uses one fixed-point scale per
// scene and channel, s_b = fx_scale(K_b B_b), for every contribution, in
// the LDS tiles and in a 64-bit integer grid, so each node's sum is exact
// and independent of the order of the additions and of how the particles
// are grouped into items.  K_b = max(the largest item's particle count,
// N_b / 2^13) keeps a tile node sum (at most one contribution per particle
// of the item, each below 2^49 / K_b) below 2^49 and a grid node sum below
// 2^62.  Items, and so K_b, are the same whether a scene runs alone or in a
// batch.
//
// After the first substep the measuring launch is replaced by a prediction:
// the fused launch takes its scales from the previous substep's bounds and
// raises this substep's bounds as it goes (kDetPredict).  Only a scene whose
// scale, fx_scale(K_b B_b), differs from the predicted one is scattered
// again, from the state the launch stored, at the measured scale into a
// second fixed-point grid (kDetRedo), and the conversion takes that grid for
// it.  Either way every node sum is the one the measured scale gives.
constexpr int kDetOff = 0, kDetMeasure = 1, kDetAccumulate = 2, kDetPredict = 3, kDetRedo = 4;

// K_b of scene b (deterministic mode)
__device__ __forceinline__ double fx_range(const unsigned* fxb, const double* fxk, int b) {
  return fmax((double)fxb[4 * b + 2], fxk[b]);
}

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ float wave_maxf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ unsigned wave_sum_u(unsigned v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Raises the float maximum kept as bits in *slot (non-negative values
// compare as unsigned integers).  The atomic is skipped when the value read
// is already as large: one address taken by every wave would otherwise
// serialise them.
__device__ __forceinline__ void raise_max(unsigned* slot, float v) {
  const unsigned b = __float_as_uint(v);
  if (v > 0.0f && b > __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMax(slot, b);
}

// The CFL watch of one wave: adds its count of violations to diag[4] and
// raises diag[5] (float bits, non-negative) to its largest |v|^2.
__device__ __forceinline__ void cfl_flush(unsigned long long* diag, float v2max, unsigned count) {
  const float m = wave_maxf(v2max);
  const unsigned c = wave_sum_u(count);
  if ((threadIdx.x & 63) == 0) {
    if (c) atomicAdd(&diag[4], (unsigned long long)c);
    raise_max(reinterpret_cast<unsigned*>(&diag[5]), m);
  }
}

// 64-bit fixed point of the P2G tile.  fx_bits(v, s) = bits of
// fma(v, s, 1.5*2^52): for |v s| < 2^51 that double lies in [2^52, 2^53),
// where one unit is one ulp, so its bits are 0x4338000000000000 + round(v s)
// as a 64-bit integer.  The constant has its low 51 bits zero, so a sum of
// such words, taken modulo 2^51 and sign-extended from bit 50, is the exact
// sum of the rounded values whenever that sum's magnitude is below 2^50.
constexpr float kFxMargin = 16.0f;  // headroom of later particles over the first sub-chunk's largest

__device__ __forceinline__ unsigned long long fx_bits(float v, double s) {
  return (unsigned long long)__double_as_longlong(fma((double)v, s, 6755399441055744.0));
}

__device__ __forceinline__ long long fx_value(unsigned long long u) { return (long long)(u << 13) >> 13; }

// Power-of-two scale s with x s < 2^49 (x >= 0; 1 for x = 0).
__device__ __forceinline__ double fx_scale(double x) {
  if (!(x > 0.0)) return 1.0;
  int e;
  (void)frexp(x, &e);  // x < 2^e
  e = min(max(49 - e, -900), 900);
  return ldexp(1.0, e);
}

// Deterministic mode: whether scene b's scales from the measured bank cur
// differ from those predicted from bank prev (either channel)
__device__ __forceinline__ bool fx_mismatch(const unsigned* cur, const unsigned* prev, const double* fxk, int b) {
  const double kc = fx_range(cur, fxk, b), kp = fx_range(prev, fxk, b);
  return fx_scale(kc * (double)__uint_as_float(cur[4 * b])) != fx_scale(kp * (double)__uint_as_float(prev[4 * b])) ||
         fx_scale(kc * (double)__uint_as_float(cur[4 * b + 1])) !=
             fx_scale(kp * (double)__uint_as_float(prev[4 * b + 1]));
}

// Box of base cells over the workgroup's valid particles, plus the maxima
// of NF non-negative floats.  out[0..2] = min, out[3..5] = max (empty ->
// min > max); fmax_io[k] in: this lane's value, out: the workgroup maximum.
// red: LDS scratch of (6 + NF) * waves ints.
template <int NF = 0>
__device__ __forceinline__ void block_box(bool valid, const int* b, int* red, int* out, float* fmax_io = nullptr) {
  constexpr int NV = 6 + NF;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int v[NV];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = valid ? b[k] : 0x3fffffff;
    v[k + 3] = valid ? -b[k] : 0x3fffffff;
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) v[6 + k] = -__float_as_int(fmax_io[k]);  // order of non-negative floats
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_min(v[k]);
  __syncthreads();  // red may still be read by an earlier call
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
  int r[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) r[k] = red[k];
  for (int w = 1; w < kBlock / 64; ++w)
#pragma unroll
    for (int k = 0; k < NV; ++k) r[k] = min(r[k], red[w * NV + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    out[k] = r[k];
    out[k + 3] = -r[k + 3];
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) fmax_io[k] = __int_as_float(-r[6 + k]);
}

// Base cell and fraction of one coordinate.  base = floor(x n - 0.5) is
// computed exactly (x n of a float32 x is exact in double).  Valid only if
// the whole 3-node stencil lies inside [0, n).
__device__ __forceinline__ bool cell_of(float xc, int n, int& base, float& f) {
  const double t = (double)xc * (double)n - 0.5;
  if (!(t >= 0.0 && t < (double)(n - 2))) {
    base = 0;
    f = 1.0f;
    return false;
  }
  base = (int)floor(t);
  f = (float)((double)xc * (double)n - (double)base);
  return true;
}

__device__ __forceinline__ void bspline_w(float f, float* w) {
  const float a = 1.5f - f, b = f - 1.0f, c = f - 0.5f;
  w[0] = 0.5f * a * a;
  w[1] = 0.75f - b * b;
  w[2] = 0.5f * c * c;
}

// vs = sum_o w_o v_o and M[c][b] = sum_o w_o v_o[c] o_b over the 27 nodes o
// of a stencil, w_o = wx[ox] wy[oy] wz[oz].  The weight is a product of
// per-axis factors, so the sums go axis by axis: z per (ox, oy) row, then y
// per ox plane, then x.  fetch(ox, oy, oz, v) loads node o's velocity.
template <class Fetch>
__device__ __forceinline__ void g2p_moments(const float* wx, const float* wy, const float* wz, Fetch fetch,
                                            float* vs, float (*M)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    vs[c] = 0.f;
    M[c][0] = M[c][1] = M[c][2] = 0.f;
  }
#pragma unroll
  for (int ox = 0; ox < 3; ++ox) {
    float s0[3] = {0.f, 0.f, 0.f}, sy[3] = {0.f, 0.f, 0.f}, sz1[3] = {0.f, 0.f, 0.f};  // per ox plane
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      float r0[3] = {0.f, 0.f, 0.f}, r1[3] = {0.f, 0.f, 0.f};  // sum_z wz v, sum_z oz wz v
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        float vi[3];
        fetch(ox, oy, oz, vi);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          r0[c] = fmaf(wz[oz], vi[c], r0[c]);
          if (oz) r1[c] = fmaf((float)oz * wz[oz], vi[c], r1[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s0[c] = fmaf(wy[oy], r0[c], s0[c]);
        if (oy) sy[c] = fmaf((float)oy * wy[oy], r0[c], sy[c]);
        sz1[c] = fmaf(wy[oy], r1[c], sz1[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vs[c] = fmaf(wx[ox], s0[c], vs[c]);
      if (ox) M[c][0] = fmaf((float)ox * wx[ox], s0[c], M[c][0]);
      M[c][1] = fmaf(wx[ox], sy[c], M[c][1]);
      M[c][2] = fmaf(wx[ox], sz1[c], M[c][2]);
    }
  }
}

// Grid velocity from accumulated (mv, m): normalise, gravity, sticky walls.
__device__ __forceinline__ void grid_velocity(const float4 g, int ix, int iy, int iz, const SubstepArgs& a,
                                              float* vo) {
  const int n = a.n, bd = a.bound;
  const bool wall = ix < bd || iy < bd || iz < bd || ix >= n - bd || iy >= n - bd || iz >= n - bd;
  if (!(g.w > 0.0f) || wall) {
    vo[0] = vo[1] = vo[2] = 0.0f;
    return;
  }
  vo[0] = g.x / g.w + a.dt * a.g[0];
  vo[1] = g.y / g.w + a.dt * a.g[1];
  vo[2] = g.z / g.w + a.dt * a.g[2];
}

__device__ __forceinline__ int rot3(int s, int k) {  // (k + s) mod 3 for s, k in [0, 3)
  const int r = k + s;
  return r >= 3 ? r - 3 : r;
}

__device__ __forceinline__ float sel3(const float* w, int r) { return r == 0 ? w[0] : (r == 1 ? w[1] : w[2]); }

__device__ __forceinline__ void count_event(unsigned long long* diag, int slot, bool flag) {
  const unsigned long long m = __ballot(flag);
  if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(&diag[slot], (unsigned long long)__popcll(m));
}

// --------------------------------------------------------------------------
// The substep kernel.  A work item is a contiguous run of particles of one
// 4^3-cell block (the table is rebuilt after every sort); workgroups take
// items from a device counter.  Per item:
//   1. box of the particles' base cells;
//   2. G2P tile (box + 2 nodes) loaded from the grid being read, with the
//      grid update applied on the way in; P2G tile (box grown by one cell,
//      since a particle moves less than a cell per substep) zeroed;
//   3. sub-chunks of kBlock particles, one per thread: G2P gather from the
//      tile, F update, return map (FP64 SVD), stress of the new F and the
//      P2G scatter into the tile with 64-bit fixed-point LDS atomics in a
//      staggered node order (one barrier, after the first sub-chunk's
//      stress, fixes the item's fixed-point scales); a particle outside the
//      P2G box, or beyond the fixed-point range, scatters to global memory;
//   4. flush: one global FP32 atomic per touched node and channel.
// Items whose box exceeds the LDS tiles use global memory throughout.
// --------------------------------------------------------------------------
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// Workgroup min of lo[3] and max of hi[3] into box[6].
__device__ __forceinline__ void block_minmax(const int* lo, const int* hi, int* red, int* box) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int v[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = wave_min(lo[k]);
    v[k + 3] = wave_max(hi[k]);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) red[wave * 6 + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 6; ++k) box[k] = red[k];
  for (int w = 1; w < kBlock / 64; ++w)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      box[k] = min(box[k], red[w * 6 + k]);
      box[k + 3] = max(box[k + 3], red[w * 6 + k + 3]);
    }
}

// SPARSE: block-sparse activity of the rotation's grid buffers.  Each
// buffer is followed in memory (at clear_nodes nodes) by one uint32 flag per
// 4^3-node block, (n + 3) / 4 blocks per axis and scene.  The launch flags
// every block it adds to in grid_out and zeroes only the flagged blocks of
// grid_clear (resetting their flags), so its grid work follows the occupied
// blocks instead of the whole n^3.  Flags only ever over-cover the blocks
// that hold mass.
template <int MODE, int DET = kDetOff, bool SPARSE = false>
__global__ __launch_bounds__(kBlock, 2) void k_substep(SubstepArgs a) {
  constexpr bool kMeasure = DET == kDetMeasure, kPredict = DET == kDetPredict, kRedo = DET == kDetRedo;
  constexpr bool kAccum = DET == kDetAccumulate || kPredict || kRedo;  // adds into the fixed-point grid
  constexpr bool kRaise = kMeasure || kPredict;                        // records the bounds in fxi
  constexpr bool kQuiet = kMeasure || kRedo;  // repeats work another launch counts: no diagnostics
  // deterministic modes take the stress of the stored (float32) F, as a
  // P2G-only launch from stored state does, so that a run split at any call
  // boundary equals the run in one piece
  constexpr bool kStressFromStored = (DET != kDetOff) && (MODE == kFused);
  __shared__ unsigned long long ptile[4 * kTileCapMax];  // P2G fixed-point accumulators: mv.x, mv.y, mv.z, m
  __shared__ float gtile[3 * kTileCapMax];               // G2P node velocities
  __shared__ int red[8 * (kBlock / 64)];
  __shared__ float fred[2 * (kBlock / 64)];
  __shared__ float imax_s[2 * (kBlock / 64)];
  __shared__ int item_s;
  __shared__ int nbox_s[6];  // the item's box after this substep

  const int n = a.n;
  const int64_t N = a.N;
  const float inv_dx = (float)n, dx = 1.0f / (float)n;
  const int cap = a.tile_cap;
  const int n_items = *a.n_chunks;
  if (kRedo) {  // nothing to do unless a scene's measured scale differs from its predicted one
    bool any = false;  // the fold's flags, a wave's lanes over the scenes
    for (int b = (int)(threadIdx.x & 63); b < a.n_scenes; b += 64) any |= a.fxb[4 * b + 3] != 0u;
    if (!__any(any)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.diag[8], 1ull);
  }

  const int nbn = (n + 3) >> 2;  // 4^3-node blocks per axis
  // block flags of the buffer this launch adds into: the rotation's grid
  // buffer (SPARSE) or the fixed-point grid (deterministic accumulation)
  unsigned* const flag_out = SPARSE ? (a.grid_out ? reinterpret_cast<unsigned*>(a.grid_out + a.clear_nodes) : nullptr)
                                    : (kAccum ? a.gflag : nullptr);
  if (SPARSE && a.grid_clear) {
    // this workgroup's slice of the block flags: a thread zeroes the 64
    // nodes of a flagged block (rows of 4 nodes along z) and resets its flag
    // (32-bit block arithmetic: block indices stay below 2^31)
    unsigned* const fc = reinterpret_cast<unsigned*>(a.grid_clear + a.clear_nodes);
    const int per_scene = nbn * nbn * nbn;
    const int nflags = a.n_scenes * per_scene;
    const int per = (nflags + (int)gridDim.x - 1) / (int)gridDim.x;
    const int c0 = (int)blockIdx.x * per, c1 = min(nflags, c0 + per);
    for (int blk = c0 + (int)threadIdx.x; blk < c1; blk += kBlock) {
      if (!fc[blk]) continue;
      const int sc = blk / per_scene, rb = blk - sc * per_scene;
      const int bx = rb / (nbn * nbn), by = (rb / nbn) % nbn, bz = rb % nbn;
      for (int r = 0; r < 16; ++r) {
        const int ix = 4 * bx + (r >> 2), iy = 4 * by + (r & 3);
        if (ix >= n || iy >= n) continue;
        float4* row = a.grid_clear + ((((int64_t)sc * n + ix) * n + iy) * n + 4 * bz);
        for (int k = 0; k < 4 && 4 * bz + k < n; ++k) row[k] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      fc[blk] = 0u;
    }
  } else if (a.grid_clear) {  // this workgroup's slice of the buffer to clear
    const int64_t per = (a.clear_nodes + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * per, c1 = min(a.clear_nodes, c0 + per);
    for (int64_t t = c0 + threadIdx.x; t < c1; t += kBlock) a.grid_clear[t] = make_float4(0.f, 0.f, 0.f, 0.f);
  }

  float v2max = 0.0f;  // CFL watch over this lane's particles
  unsigned cfl_count = 0;
  for (;;) {
    __syncthreads();  // tiles and item_s are reused
    if (threadIdx.x == 0) item_s = atomicAdd(a.work_counter, 1);
    __syncthreads();
    const int item = item_s;
    if (item >= n_items) break;
    const int start = a.chunk_start[item], end = a.chunk_start[item + 1];
    const int64_t gbase = (int64_t)a.chunk_batch[item] * n * n * n;
    if (kRedo && a.fxb[4 * a.chunk_batch[item] + 3] == 0u) continue;  // its scale held

    // 1. box of base cells: from the previous substep, or a pass over x
    int box[6];
    if (a.box_in) {
#pragma unroll
      for (int k = 0; k < 6; ++k) box[k] = a.box_in[6 * item + k];
    } else {
      int lo[3] = {0x3fffffff, 0x3fffffff, 0x3fffffff}, hi[3] = {-0x3fffffff, -0x3fffffff, -0x3fffffff};
      for (int i = start + (int)threadIdx.x; i < end; i += kBlock) {
        int b[3];
        float f[3];
        bool in = true;
  #pragma unroll
        for (int k = 0; k < 3; ++k) in &= cell_of(a.x[k * N + i], n, b[k], f[k]);
        if (in) {
  #pragma unroll
          for (int k = 0; k < 3; ++k) {
            lo[k] = min(lo[k], b[k]);
            hi[k] = max(hi[k], b[k]);
          }
        }
      }
      block_minmax(lo, hi, red, box);
    }
    // the next box starts as this one; particles that change cell widen it
    if (threadIdx.x == 0) {
#pragma unroll
      for (int k = 0; k < 6; ++k) nbox_s[k] = box[k];
    }
    const bool empty = box[0] > box[3];
    // G2P tile: nodes box.lo .. box.hi + 2
    const int gx = box[3] - box[0] + 3, gy = box[4] - box[1] + 3, gz = box[5] - box[2] + 3;
    const int GT = empty ? 0 : gx * gy * gz;
    // P2G tile: base cells in [plo, phi] (the box grown by one cell where the
    // particles have moved, clamped to the grid), nodes plo .. phi + 2
    const int grow = (MODE == kP2G) ? 0 : 1;
    int plo[3], phi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      plo[k] = max(box[k] - grow, 0);
      phi[k] = min(box[k + 3] + grow, n - 3);
    }
    const int px = phi[0] - plo[0] + 3, py = phi[1] - plo[1] + 3, pz = phi[2] - plo[2] + 3;
    // x stride padded by kPadX nodes: with the plain py*pz stride the nodes a
    // wave scatters to fall on few LDS banks (x-neighbours share a bank)
    const int SX = py * pz + kPadX;
    const int PT = empty ? 0 : (px - 1) * SX + (py - 1) * pz + pz;
    const bool lds_g = (MODE != kP2G) && !empty && GT <= cap;
    const bool lds_p = !kMeasure && (MODE != kG2P) && !empty && PT <= cap;
    if (!kQuiet && threadIdx.x == 0 && !empty && (((MODE != kP2G) && !lds_g) || ((MODE != kG2P) && !lds_p)))
      atomicAdd(&a.diag[2], 1ull);

    // 2. tiles
    if (lds_g) {
      for (int t = threadIdx.x; t < GT; t += kBlock) {
        const int tk = t % gz, tq = t / gz;
        const int tj = tq % gy, ti = tq / gy;
        const int ix = box[0] + ti, iy = box[1] + tj, iz = box[2] + tk;
        float vv[3];
        grid_velocity(a.grid_in[gbase + ((int64_t)ix * n + iy) * n + iz], ix, iy, iz, a, vv);
        gtile[t] = vv[0];
        gtile[kTileCapMax + t] = vv[1];
        gtile[2 * kTileCapMax + t] = vv[2];
      }
    }
    if (lds_p) {
      for (int t = threadIdx.x; t < PT; t += kBlock) {
        ptile[t] = 0ull;
        ptile[kTileCapMax + t] = 0ull;
        ptile[2 * kTileCapMax + t] = 0ull;
        ptile[3 * kTileCapMax + t] = 0ull;
      }
    }
    __syncthreads();

    // 3. particles.  The P2G tile holds 64-bit fixed point: a contribution
    // val enters as the bits of fma(val, s, 1.5*2^52), whose low 51 bits are
    // round(val*s) in two's complement (the constant's low 51 bits are 0),
    // so integer LDS adds (ds_add_u64, about twice the rate of ds_add_f64)
    // sum the rounded values exactly modulo 2^51.  The scales s (momentum,
    // mass; powers of two) are set per item from the first sub-chunk's
    // largest contribution so that every node sum stays below 2^49; a later
    // particle whose contribution exceeds kFxMargin times that maximum
    // scatters to global memory instead.
    double s_mom = 1.0, s_mass = 1.0;
    float meas_mom = 0.0f, meas_mass = 0.0f;  // kRaise: this lane's largest bounds in the item
    float lim_mom = 0.0f, lim_mass = 0.0f;
    const int scene = a.chunk_batch[item];
    if (kAccum) {  // the scene's scales from the measured (or, predicting, the previous) bounds
      lim_mom = __uint_as_float(a.fxb[4 * scene]);
      lim_mass = __uint_as_float(a.fxb[4 * scene + 1]);
      const double K = fx_range(a.fxb, a.fxk, scene);
      s_mom = fx_scale(K * (double)lim_mom);
      s_mass = fx_scale(K * (double)lim_mass);
      // predicting, every finite contribution enters the tile: if this
      // substep's bounds give the same scales, they keep every sum in range
      // (as for the measured bounds); if not, the scene is scattered again
      if (kPredict) lim_mom = lim_mass = INFINITY;
    }
    for (int sub = start; sub < end; sub += kBlock) {
      const int i = sub + (int)threadIdx.x;
      const bool scale_pass = !kAccum && (MODE != kG2P) && lds_p && sub == start;
      if (i >= end && !scale_pass) break;  // the scale pass needs every thread at its barrier
      // P2G contribution of this thread's particle: w (q + Ad o) for node offset o
      bool scat = false;
      float q[3], Ad[9], f1[3], mass = 0.0f;
      int b1[3];
      if (i < end) {
        float xp[3], vp[3] = {0.f, 0.f, 0.f};
        float Cp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        double Fd[9];
#pragma unroll
        for (int k = 0; k < 3; ++k) xp[k] = a.x[k * N + i];
#pragma unroll
        for (int k = 0; k < 9; ++k) Fd[k] = (double)a.F[k * N + i];
        const float4 prm = a.prm[i];
        int mid = a.mat[i];
        if (MODE == kP2G) {
#pragma unroll
          for (int k = 0; k < 3; ++k) vp[k] = a.v[k * N + i];
#pragma unroll
          for (int k = 0; k < 9; ++k) Cp[k] = a.C[k * N + i];
        }
        mid = (mid >= 0 && mid < a.n_materials) ? mid : 0;
        const Material mat = a.mats[mid];
        const double mu = (double)prm.z, lam = (double)prm.w;
        double tau[9];
        bool ok = true;
        int b0p = -1;  // base cell before this substep, 10 bits per axis (grid_res <= 1024)

        // -------------------------------------------------------- G2P
        if (MODE != kP2G) {
          int b0[3];
          float f0[3];
          bool in_grid = true;
#pragma unroll
          for (int k = 0; k < 3; ++k) in_grid &= cell_of(xp[k], n, b0[k], f0[k]);
          ok = in_grid;
          if (in_grid) b0p = b0[0] | (b0[1] << 10) | (b0[2] << 20);
          if (!in_grid && !kQuiet) {
            atomicAdd(&a.diag[1], 1ull);
            if (a.xo != a.x) {  // skipped: carry the state over unchanged
#pragma unroll
              for (int k = 0; k < 3; ++k) a.xo[k * N + i] = xp[k];
#pragma unroll
              for (int k = 0; k < 9; ++k) a.Fo[k * N + i] = (float)Fd[k];
              if (a.write_vc) {
#pragma unroll
                for (int k = 0; k < 3; ++k) a.vo[k * N + i] = a.v[k * N + i];
#pragma unroll
                for (int k = 0; k < 9; ++k) a.Co[k * N + i] = a.C[k * N + i];
              }
            }
          }
          if (ok) {
            float wx[3], wy[3], wz[3];
            bspline_w(f0[0], wx);
            bspline_w(f0[1], wy);
            bspline_w(f0[2], wz);
            // vs = sum w v and M[c][b] = sum w v_c o_b, summed axis by axis
            // (the weight is a product of per-axis factors): z sums per
            // (ox, oy) row, then y per ox plane, then x.  The same sums as
            // g2p_moments, written out here: through the helper's fetch
            // callback this kernel needed 12 more registers and dropped to one
            // wave per SIMD.
            float vs[3] = {0.f, 0.f, 0.f};
            float M[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
            if (lds_g) {
              const int sz = gy * gz;
              const int a0 = ((b0[0] - box[0]) * gy + (b0[1] - box[1])) * gz + (b0[2] - box[2]);
#pragma unroll
              for (int ox = 0; ox < 3; ++ox) {
                float s0[3] = {0.f, 0.f, 0.f}, sy[3] = {0.f, 0.f, 0.f}, sz1[3] = {0.f, 0.f, 0.f};  // per ox plane
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                  const int row = a0 + ox * sz + oy * gz;
                  float r0[3] = {0.f, 0.f, 0.f}, r1[3] = {0.f, 0.f, 0.f};  // sum_z wz v, sum_z oz wz v
#pragma unroll
                  for (int oz = 0; oz < 3; ++oz) {
                    const float vi[3] = {gtile[row + oz], gtile[kTileCapMax + row + oz],
                                         gtile[2 * kTileCapMax + row + oz]};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                      r0[c] = fmaf(wz[oz], vi[c], r0[c]);
                      if (oz) r1[c] = fmaf((float)oz * wz[oz], vi[c], r1[c]);
                    }
                  }
#pragma unroll
                  for (int c = 0; c < 3; ++c) {
                    s0[c] = fmaf(wy[oy], r0[c], s0[c]);
                    if (oy) sy[c] = fmaf((float)oy * wy[oy], r0[c], sy[c]);
                    sz1[c] = fmaf(wy[oy], r1[c], sz1[c]);
                  }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  vs[c] = fmaf(wx[ox], s0[c], vs[c]);
                  if (ox) M[c][0] = fmaf((float)ox * wx[ox], s0[c], M[c][0]);
                  M[c][1] = fmaf(wx[ox], sy[c], M[c][1]);
                  M[c][2] = fmaf(wx[ox], sz1[c], M[c][2]);
                }
              }
            } else {
              // the item's box exceeds the LDS tile (rare): node by node from
              // the grid, in a loop kept rolled (code size)
#pragma unroll 1
              for (int o = 0; o < 27; ++o) {
                const int ox = o / 9, oy = (o / 3) % 3, oz = o % 3;
                const int ix = b0[0] + ox, iy = b0[1] + oy, iz = b0[2] + oz;
                float vi[3];
                grid_velocity(a.grid_in[gbase + ((int64_t)ix * n + iy) * n + iz], ix, iy, iz, a, vi);
                const float w = sel3(wx, ox) * sel3(wy, oy) * sel3(wz, oz);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                  const float wv = w * vi[c];
                  vs[c] += wv;
                  M[c][0] = fmaf((float)ox, wv, M[c][0]);
                  M[c][1] = fmaf((float)oy, wv, M[c][1]);
                  M[c][2] = fmaf((float)oz, wv, M[c][2]);
                }
              }
            }
            // C' = 4/dx^2 sum w v (x_i - x_p)^T = 4/dx (M - v f^T)
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int c = 0; c < 3; ++c) Cp[3 * r + c] = 4.0f * inv_dx * (M[r][c] - vs[r] * f0[c]);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              vp[k] = vs[k];
              xp[k] = xp[k] + a.dt * vs[k];
            }
            const float v2 = vs[0] * vs[0] + vs[1] * vs[1] + vs[2] * vs[2];
            if (!kQuiet) {
              v2max = fmaxf(v2max, v2);
              cfl_count += (v2 > a.cfl_v2) ? 1u : 0u;
            }
            // F_trial = (I + dt C') F, in double
            double Ftr[9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                double acc = Fd[3 * r + c];
#pragma unroll
                for (int k = 0; k < 3; ++k) acc += (double)a.dt * (double)Cp[3 * r + k] * Fd[3 * k + c];
                Ftr[3 * r + c] = acc;
              }
            update_and_stress(mat, mu, lam, Ftr, true, MODE == kFused && !kStressFromStored, Fd, tau);
            float Ff[9];
            bool fin = true;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
              Ff[k] = (float)Fd[k];
              fin &= isfinite(Ff[k]);
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) fin &= isfinite(xp[k]);
            if (!fin) {
              if (!kQuiet) atomicAdd(&a.diag[0], 1ull);
              ok = false;
            }
            if (!kMeasure) {
#pragma unroll
              for (int k = 0; k < 3; ++k) a.xo[k * N + i] = xp[k];
#pragma unroll
              for (int k = 0; k < 9; ++k) a.Fo[k * N + i] = Ff[k];
            }
            if (!kMeasure && (MODE == kG2P || a.write_vc)) {
#pragma unroll
              for (int k = 0; k < 3; ++k) a.vo[k * N + i] = vp[k];
#pragma unroll
              for (int k = 0; k < 9; ++k) a.Co[k * N + i] = Cp[k];
            }
          }
        }

        // -------------------------------------------------------- P2G contribution
        if (MODE != kG2P) {
          bool in_grid = true;
#pragma unroll
          for (int k = 0; k < 3; ++k) in_grid &= cell_of(xp[k], n, b1[k], f1[k]);
          if (MODE == kP2G && !in_grid && !kQuiet) atomicAdd(&a.diag[1], 1ull);
          // a particle that changed cell may widen the item's next box
          if (MODE == kFused && a.box_out && in_grid && (b1[0] | (b1[1] << 10) | (b1[2] << 20)) != b0p) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              atomicMin(&nbox_s[k], b1[k]);
              atomicMax(&nbox_s[k + 3], b1[k]);
            }
          }
          if (ok && in_grid) {
            // A = m C - 4/dx^2 dt V0 tau, folded with dx for the node offsets
            mass = prm.x;
            if (MODE == kP2G || kStressFromStored) {
              double Fs[9];
#pragma unroll
              for (int k = 0; k < 9; ++k) Fs[k] = kStressFromStored ? (double)(float)Fd[k] : Fd[k];
              update_and_stress(mat, mu, lam, Fs, false, true, Fd, tau);
            }
            const float ks = 4.0f * inv_dx * inv_dx * a.dt * prm.y;
#pragma unroll
            for (int k = 0; k < 9; ++k) Ad[k] = (mass * Cp[k] - ks * (float)tau[k]) * dx;
            // contribution to node o: w (m v + A (o - f) dx) = w (q + Ad o)
            bool fin = isfinite(mass);
#pragma unroll
            for (int r = 0; r < 3; ++r) {
              q[r] = mass * vp[r] - (Ad[3 * r] * f1[0] + Ad[3 * r + 1] * f1[1] + Ad[3 * r + 2] * f1[2]);
              fin &= isfinite(q[r]);
            }
#pragma unroll
            for (int k = 0; k < 9; ++k) fin &= isfinite(Ad[k]);
            if (fin) {
              scat = true;
            } else if (!kQuiet) {  // never let a bad particle reach the grid
              atomicAdd(&a.diag[0], 1ull);
            }
          }
        }
      }
      if (MODE == kG2P) continue;

      // bound of |w (q + Ad o)| over the 27 nodes (w <= 0.75^3) and of w m
      float bnd_mom = 0.0f, bnd_mass = 0.0f;
      if (scat) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
          bnd_mom = fmaxf(bnd_mom, fabsf(q[r]) + 2.0f * (fabsf(Ad[3 * r]) + fabsf(Ad[3 * r + 1]) + fabsf(Ad[3 * r + 2])));
        bnd_mom *= 0.421875f;
        bnd_mass = 0.421875f * fabsf(mass);
      }
      // a bound that overflows float32 keeps its particle out of the tile and out of the scale
      const bool fx_ok = bnd_mom <= 3.0e38f && bnd_mass <= 3.0e38f;
      if (kRaise && scat && fx_ok) {  // the lane's largest bounds
        meas_mom = fmaxf(meas_mom, bnd_mom);
        meas_mass = fmaxf(meas_mass, bnd_mass);
      }
      if (kMeasure) continue;  // nothing is scattered
      if (scale_pass) {
        float m2[2] = {wave_maxf(fx_ok ? bnd_mom : 0.0f), wave_maxf(fx_ok ? bnd_mass : 0.0f)};
        if ((threadIdx.x & 63) == 0) {
          fred[2 * (threadIdx.x >> 6)] = m2[0];
          fred[2 * (threadIdx.x >> 6) + 1] = m2[1];
        }
        __syncthreads();
        for (int w = 0; w < kBlock / 64; ++w) {
          m2[0] = fmaxf(m2[0], fred[2 * w]);
          m2[1] = fmaxf(m2[1], fred[2 * w + 1]);
        }
        const double cnt = (double)(end - start) * (double)kFxMargin;
        lim_mom = kFxMargin * m2[0];
        lim_mass = kFxMargin * m2[1];
        s_mom = fx_scale(cnt * (double)m2[0]);
        s_mass = fx_scale(cnt * (double)m2[1]);
      }
      if (!scat) continue;

      const bool in_tile = lds_p && b1[0] >= plo[0] && b1[0] <= phi[0] && b1[1] >= plo[1] && b1[1] <= phi[1] &&
                           b1[2] >= plo[2] && b1[2] <= phi[2] && fx_ok && bnd_mom <= lim_mom &&
                           bnd_mass <= lim_mass;
      if (lds_p && !in_tile && !kQuiet) atomicAdd(&a.diag[3], 1ull);
      float w[3][3];
      bspline_w(f1[0], w[0]);
      bspline_w(f1[1], w[1]);
      bspline_w(f1[2], w[2]);
      // staggered node order: lane group g visits offset (k + g_axis) mod 3 at step k
      const int g = (threadIdx.x & 63) % 27;
      const int gs[3] = {g / 9, (g / 3) % 3, g % 3};
      int r[3][3];
      float wr[3][3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          r[ax][k] = rot3(gs[ax], k);
          wr[ax][k] = sel3(w[ax], r[ax][k]);
        }
      const int sz = SX;
      const int a1 = (b1[0] - plo[0]) * SX + (b1[1] - plo[1]) * pz + (b1[2] - plo[2]);
      if (in_tile) {
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const float ox = (float)r[0][kx];
          float vx[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) vx[c] = q[c] + Ad[3 * c] * ox;
#pragma unroll
          for (int ky = 0; ky < 3; ++ky) {
            const float oy = (float)r[1][ky];
            const float wxy = wr[0][kx] * wr[1][ky];
            float vy[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) vy[c] = vx[c] + Ad[3 * c + 1] * oy;
            const int row = a1 + r[0][kx] * sz + r[1][ky] * pz;
#pragma unroll
            for (int kz = 0; kz < 3; ++kz) {
              const float oz = (float)r[2][kz];
              const float wgt = wxy * wr[2][kz];
              const int t = row + r[2][kz];
#pragma unroll
              for (int c = 0; c < 3; ++c)
                atomicAdd(&ptile[c * kTileCapMax + t], fx_bits(wgt * (vy[c] + Ad[3 * c + 2] * oz), s_mom));
              atomicAdd(&ptile[3 * kTileCapMax + t], fx_bits(wgt * mass, s_mass));
            }
          }
        }
      } else {
        // outside the item's P2G tile or its fixed-point range (rare): FP32
        // global atomics node by node, in a loop kept rolled (code size);
        // with SPARSE each node's block is flagged first
#pragma unroll 1
        for (int o = 0; o < 27; ++o) {
          const int ox = o / 9, oy = (o / 3) % 3, oz = o % 3;
          const float wgt = sel3(w[0], ox) * sel3(w[1], oy) * sel3(w[2], oz);
          const int ix = b1[0] + ox, iy = b1[1] + oy, iz = b1[2] + oz;
          const int64_t node = gbase + ((int64_t)ix * n + iy) * n + iz;
          if ((SPARSE || kAccum) && flag_out)
            flag_out[(int64_t)scene * nbn * nbn * nbn + ((int64_t)(ix >> 2) * nbn + (iy >> 2)) * nbn + (iz >> 2)] = 1u;
          if (kAccum) {  // the scene's fixed point, added exactly
            unsigned long long* gq = a.gfx + 4 * node;
#pragma unroll
            for (int c = 0; c < 3; ++c)
              atomicAdd(gq + c, (unsigned long long)fx_value(fx_bits(
                                    wgt * (q[c] + Ad[3 * c] * (float)ox + Ad[3 * c + 1] * (float)oy +
                                           Ad[3 * c + 2] * (float)oz), s_mom)));
            atomicAdd(gq + 3, (unsigned long long)fx_value(fx_bits(wgt * mass, s_mass)));
          } else {
            float* gp = (float*)&a.grid_out[node];
#pragma unroll
            for (int c = 0; c < 3; ++c)
              atomicAdd(gp + c, wgt * (q[c] + Ad[3 * c] * (float)ox + Ad[3 * c + 1] * (float)oy + Ad[3 * c + 2] * (float)oz));
            atomicAdd(gp + 3, wgt * mass);
          }
        }
      }
    }

    if (kRaise) {  // the waves' largest bounds
      const float m0 = wave_maxf(meas_mom), m1 = wave_maxf(meas_mass);
      if ((threadIdx.x & 63) == 0) {
        imax_s[2 * (threadIdx.x >> 6)] = m0;
        imax_s[2 * (threadIdx.x >> 6) + 1] = m1;
      }
    }
    __syncthreads();  // the tile, the next box and the waves' bounds are complete
    if (kRaise && threadIdx.x == 0) {  // the item's largest bounds: a plain store per item
      float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w) {
        m0 = fmaxf(m0, imax_s[2 * w]);
        m1 = fmaxf(m1, imax_s[2 * w + 1]);
      }
      a.fxi[item] = make_float2(m0, m1);
    }
    if (a.box_out && threadIdx.x < 6) a.box_out[6 * item + threadIdx.x] = nbox_s[threadIdx.x];

    // 4. flush (with SPARSE, after flagging the node blocks the tile covers)
    if ((SPARSE || kAccum) && lds_p && flag_out) {
      const int bx0 = plo[0] >> 2, by0 = plo[1] >> 2, bz0 = plo[2] >> 2;
      const int nx = ((phi[0] + 2) >> 2) - bx0 + 1, ny = ((phi[1] + 2) >> 2) - by0 + 1,
                nz = ((phi[2] + 2) >> 2) - bz0 + 1;
      const int64_t sbase = (int64_t)scene * nbn * nbn * nbn;
      for (int t = threadIdx.x; t < nx * ny * nz; t += kBlock) {
        const int bx = bx0 + t / (ny * nz), by = by0 + (t / nz) % ny, bz = bz0 + t % nz;
        flag_out[sbase + ((int64_t)bx * nbn + by) * nbn + bz] = 1u;
      }
    }
    if (lds_p) {
      const double is_mom = 1.0 / s_mom, is_mass = 1.0 / s_mass;
      for (int t = threadIdx.x; t < PT; t += kBlock) {
        const long long im = fx_value(ptile[3 * kTileCapMax + t]);
        if (im == 0) continue;
        const int ti = t / SX, tr = t - ti * SX;
        const int tj = tr / pz, tk = tr - tj * pz;
        if (tj >= py) continue;  // padding
        const int64_t node = gbase + ((int64_t)(plo[0] + ti) * n + (plo[1] + tj)) * n + (plo[2] + tk);
        if (kAccum) {  // integer sums at the scene's scale: exact, in any order
          unsigned long long* gq = a.gfx + 4 * node;
          atomicAdd(gq + 0, (unsigned long long)fx_value(ptile[t]));
          atomicAdd(gq + 1, (unsigned long long)fx_value(ptile[kTileCapMax + t]));
          atomicAdd(gq + 2, (unsigned long long)fx_value(ptile[2 * kTileCapMax + t]));
          atomicAdd(gq + 3, (unsigned long long)im);
        } else {
          float* gp = (float*)&a.grid_out[node];
          atomicAdd(gp + 0, (float)((double)fx_value(ptile[t]) * is_mom));
          atomicAdd(gp + 1, (float)((double)fx_value(ptile[kTileCapMax + t]) * is_mom));
          atomicAdd(gp + 2, (float)((double)fx_value(ptile[2 * kTileCapMax + t]) * is_mom));
          atomicAdd(gp + 3, (float)((double)im * is_mass));
        }
      }
    }
  }
  if (MODE != kP2G && !kQuiet) cfl_flush(a.diag, v2max, cfl_count);
  // the queue is drained: the last workgroup out resets the counters
  if (a.done_counter && threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(a.done_counter, 1u) == gridDim.x - 1) {
      atomicExch(a.work_counter, 0);
      atomicExch(a.done_counter, 0u);
    }
  }
}


// --------------------------------------------------------------------------
// Fill, sort (counting sort by cell key), gather / scatter
// --------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n, int* counter) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (counter && i == 0) *counter = 0;
  const int64_t n4 = n >> 2;
  if (i < n4) reinterpret_cast<uint4*>(p)[i] = make_uint4(v, v, v, v);
  const int64_t t = (n4 << 2) + i;
  if (i < (n & 3)) p[t] = v;
}

// Deterministic mode: each scene's bounds from the per-item bounds of a
// measuring or predicting launch (or of k_adj_bound): bank[4 b + 0 / 1] =
// the largest of fxi[item].x / .y over scene b's items (scene_item[b] ..
// scene_item[b + 1] - 1), bank[4 b + 2] = the particle count of its largest
// item (zero for a scene without items), and bank[4 b + 3] = 1 where prev
// is set (the bank the launch's scales were predicted from) and the scales
// of these bounds differ from it, else 0.  One workgroup of kFoldThreads
// per scene.
constexpr int kFoldThreads = 1024;
__global__ __launch_bounds__(kFoldThreads) void k_fx_fold(const float2* fxi, const int* chunk_start,
                                                          const int* scene_item, unsigned* bank,
                                                          const unsigned* prev, const double* fxk) {
  __shared__ float r0[kFoldThreads / 64], r1[kFoldThreads / 64];
  __shared__ int rc[kFoldThreads / 64];
  const int b = blockIdx.x;
  const int lo = scene_item[b], hi = scene_item[b + 1];
  float m0 = 0.0f, m1 = 0.0f;
  int cnt = 0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += kFoldThreads) {
    const float2 v = fxi[i];
    m0 = fmaxf(m0, v.x);
    m1 = fmaxf(m1, v.y);
    cnt = max(cnt, chunk_start[i + 1] - chunk_start[i]);
  }
  m0 = wave_maxf(m0);
  m1 = wave_maxf(m1);
  cnt = -wave_min(-cnt);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    r0[w] = m0;
    r1[w] = m1;
    rc[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kFoldThreads / 64; ++k) {
      m0 = fmaxf(m0, r0[k]);
      m1 = fmaxf(m1, r1[k]);
      cnt = max(cnt, rc[k]);
    }
    reinterpret_cast<uint4*>(bank)[b] = make_uint4(__float_as_uint(m0), __float_as_uint(m1), (unsigned)cnt, 0u);
    if (prev && fx_mismatch(bank, prev, fxk, b)) bank[4 * b + 3] = 1u;
  }
}

// Deterministic mode: node t (of scene b) of the 64-bit fixed-point grid
// [node][4] -> grid (mv, m) as float4 at the scene's scales (the same
// fx_scale of the same bounds as the accumulating launch: bank fxb), and
// the fixed-point node zeroed for the next accumulation.  With gfx2 set, a
// scene flagged by k_fx_fold (its measured scales differ from the predicted
// ones) was scattered again into gfx2: its node is taken from gfx2, and
// both grids' nodes are zeroed.  The float grid is zero where nothing was
// added (it was cleared before the launch), so untouched nodes are only read.
__device__ __forceinline__ void fx_convert_node(unsigned long long* gfx, unsigned long long* gfx2, float4* grid,
                                                int64_t t, int b, const unsigned* fxb, const double* fxk) {
  ulonglong2* g = reinterpret_cast<ulonglong2*>(gfx + 4 * t);
  ulonglong2 a = g[0], c = g[1];
  if (gfx2 && fxb[4 * b + 3]) {  // the sums at the measured scale are in gfx2
    if ((a.x | a.y | c.x | c.y) != 0ull) {
      g[0] = make_ulonglong2(0ull, 0ull);
      g[1] = make_ulonglong2(0ull, 0ull);
    }
    g = reinterpret_cast<ulonglong2*>(gfx2 + 4 * t);
    a = g[0];
    c = g[1];
  }
  if ((a.x | a.y | c.x | c.y) == 0ull) return;
  const double K = fx_range(fxb, fxk, b);
  const double is_mom = 1.0 / fx_scale(K * (double)__uint_as_float(fxb[4 * b]));
  const double is_mass = 1.0 / fx_scale(K * (double)__uint_as_float(fxb[4 * b + 1]));
  grid[t] = make_float4((float)((double)(long long)a.x * is_mom), (float)((double)(long long)a.y * is_mom),
                        (float)((double)(long long)c.x * is_mom), (float)((double)(long long)c.y * is_mass));
  g[0] = make_ulonglong2(0ull, 0ull);
  g[1] = make_ulonglong2(0ull, 0ull);
}

// The conversion over the flagged 4^3-node blocks only (the accumulating
// launches and the deterministic adjoint scatter flag every block they add
// into), one wave per block, resetting its flag.  nflags = scenes * nbn^3,
// nbn = (n + 3) / 4.
__global__ void k_fx_grid_blocks(unsigned long long* gfx, unsigned long long* gfx2, float4* grid, unsigned* flags,
                                 int64_t nflags, int nbn, int n, const unsigned* fxb, const double* fxk) {
  const int64_t blk = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (blk >= nflags) return;  // whole waves
  if (!flags[blk]) return;    // wave-uniform
  const int per = nbn * nbn * nbn;
  const int b = (int)(blk / per), rb = (int)(blk - (int64_t)b * per);
  const int bx = rb / (nbn * nbn), by = (rb / nbn) % nbn, bz = rb % nbn;
  const int l = threadIdx.x & 63;
  const int ix = 4 * bx + (l >> 4), iy = 4 * by + ((l >> 2) & 3), iz = 4 * bz + (l & 3);
  if (ix < n && iy < n && iz < n) fx_convert_node(gfx, gfx2, grid, (((int64_t)b * n + ix) * n + iy) * n + iz, b, fxb, fxk);
  if (l == 0) flags[blk] = 0u;  // after the wave's read of the flag
}

// Deterministic mode: order the particles of each cell by source index
// (the counting sort's slots come from atomics, in no fixed order).
// perm: sorted slot -> source index; start: exclusive scan of the cell
// counts.  A cell of more than kStableMax particles keeps its order and is
// counted in *fallbacks.
constexpr int kStableMax = 4096;
__global__ void k_stable_rank(const int* perm, const uint32_t* keys, const uint32_t* start, int64_t bins, int64_t N,
                              int* perm_out, unsigned long long* fallbacks) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int me = perm[j];
  const uint32_t key = keys[me];
  const int64_t s0 = start[key], s1 = (int64_t)key + 1 < bins ? (int64_t)start[key + 1] : N;
  if (s1 - s0 > kStableMax) {
    perm_out[j] = me;
    if (j == s0) atomicAdd(fallbacks, 1ull);
    return;
  }
  int64_t r = 0;
  for (int64_t q = s0; q < s1; ++q) r += perm[q] < me;
  perm_out[s0 + r] = me;
}

// key = scene * bins_per_scene + block(4^3 cells, linear) * 64 + morton(cell in block)
__device__ __forceinline__ uint32_t spread2(uint32_t v) {  // 2 bits -> positions 0, 3
  return (v & 1u) | ((v & 2u) << 2);
}

__global__ void k_cell_keys(const float* x, int64_t N, const int* chunk_start, const int* chunk_batch, int n, int nb,
                            uint32_t* key, uint32_t* slot, uint32_t* count) {
  const int chunk = blockIdx.x;
  const int i = chunk_start[chunk] + (int)threadIdx.x;
  const bool live = i < chunk_start[chunk + 1];
  uint32_t k = 0xffffffffu;
  if (live) {
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double t = (double)x[a * N + i] * (double)n - 0.5;
      c[a] = (t >= 0.0) ? (t < (double)(n - 1) ? (int)floor(t) : n - 1) : 0;  // NaN -> 0
    }
    const uint32_t blk = ((uint32_t)(c[0] >> 2) * nb + (uint32_t)(c[1] >> 2)) * nb + (uint32_t)(c[2] >> 2);
    const uint32_t mort = spread2(c[0] & 3) << 2 | spread2(c[1] & 3) << 1 | spread2(c[2] & 3);
    k = (uint32_t)chunk_batch[chunk] * (uint32_t)(nb * nb * nb * 64) + blk * 64u + mort;
  }
  // runs of equal keys in consecutive lanes take one atomic per run (the
  // input is mostly in cell order already)
  const int lane = threadIdx.x & 63;
  const uint32_t prev = __shfl_up(k, 1);
  const bool head = live && (lane == 0 || prev != k);
  const unsigned long long heads = __ballot(head);
  const unsigned long long livem = __ballot(live);
  const unsigned long long below = (lane == 63) ? ~0ull : ((1ull << (lane + 1)) - 1);
  const int my_head = 63 - __clzll(heads & below);                                  // head of my run
  const unsigned long long after = (lane == 63) ? 0ull : (heads & ~below);          // heads above me
  const int next = after ? (__ffsll((long long)after) - 1) : (64 - __clzll(livem));  // end of my run
  uint32_t base = 0;
  if (head) base = atomicAdd(&count[k], (uint32_t)(next - lane));
  base = __shfl(base, my_head);
  if (live) {
    key[i] = k;
    slot[i] = base + (uint32_t)(lane - my_head);
  }
}

// exclusive scan over K uint32 in three passes (tiles of 4096 = 1024 threads x 4)
constexpr int kScanThreads = 1024;
constexpr int kScanTile = 4 * kScanThreads;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t s = v;  // inclusive wave scan
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(s, o);
    if (lane >= o) s += t;
  }
  if (lane == 63) sh[wave] = s;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int nw = blockDim.x >> 6;
    uint32_t w = (lane < nw) ? sh[lane] : 0u;
    uint32_t ws = w;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(ws, o);
      if (lane >= o) ws += t;
    }
    if (lane < nw) sh[64 + lane] = ws - w;
    if (lane == nw - 1) sh[128] = ws;
  }
  __syncthreads();
  total = sh[128];
  const uint32_t r = s - v + sh[64 + wave];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* in, uint32_t* bsum, int64_t K) {
  __shared__ uint32_t sh[160];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (base + k < K) s += in[base + k];
  uint32_t total;
  block_exclusive_scan(s, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t* bsum, int64_t nblk) {
  __shared__ uint32_t sh[160];
  uint32_t carry = 0;
  for (int64_t t0 = 0; t0 < nblk; t0 += kScanTile) {
    const int64_t base = t0 + 4 * threadIdx.x;
    uint32_t v[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = (base + k < nblk) ? bsum[base + k] : 0u;
      s += v[k];
    }
    uint32_t total;
    uint32_t e = block_exclusive_scan(s, sh, total) + carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (base + k < nblk) bsum[base + k] = e;
      e += v[k];
    }
    carry += total;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t* data, const uint32_t* bsum, int64_t K) {
  __shared__ uint32_t sh[160];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  uint32_t v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = (base + k < K) ? data[base + k] : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t e = block_exclusive_scan(s, sh, total) + bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < K) data[base + k] = e;
    e += v[k];
  }
}

__global__ void k_place(const uint32_t* key, const uint32_t* slot, const uint32_t* off, int* perm, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) perm[off[key[i]] + slot[i]] = (int)i;
}

// Work-item table after a sort: each 4^3-cell block's particles (a
// contiguous range of the sorted order) are cut into items of at most
// `item` particles.
// off = exclusive bin offsets (64 bins per block), nchk[b] = chunks of block b.
__global__ void k_block_chunk_count(const uint32_t* off, int64_t nblocks, int64_t N, int item, uint32_t* nchk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const uint32_t lo = off[b * 64];
  const uint32_t hi = (b + 1 < nblocks) ? off[(b + 1) * 64] : (uint32_t)N;
  nchk[b] = (hi - lo + item - 1) / item;
}

// base = exclusive scan of nchk (same array, scanned in place beforehand).
// scene_item (optional, [scenes + 1]) receives each scene's first item and,
// last, the item count: items come in scene order.
__global__ void k_block_chunk_write(const uint32_t* off, const uint32_t* base, int64_t nblocks, int64_t N, int item,
                                    int blocks_per_scene, int* chunk_start, int* chunk_batch, int* n_chunks,
                                    int* scene_item) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const uint32_t lo = off[b * 64];
  const uint32_t hi = (b + 1 < nblocks) ? off[(b + 1) * 64] : (uint32_t)N;
  const uint32_t c0 = base[b];
  const int scene = (int)(b / blocks_per_scene);
  if (scene_item && b % blocks_per_scene == 0) scene_item[scene] = (int)c0;
  uint32_t c = c0;
  for (uint32_t s = lo; s < hi; s += item, ++c) {
    chunk_start[c] = (int)s;
    chunk_batch[c] = scene;
  }
  if (b == nblocks - 1) {
    chunk_start[c] = (int)N;
    *n_chunks = (int)c;
    if (scene_item) scene_item[nblocks / blocks_per_scene] = (int)c;
  }
}

// out[c][j] = in[c][perm[j]] for `planes` planes of stride N
__global__ void k_gather_planes(float* out, const float* in, const int* perm, int planes, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t s = perm[j];
  for (int c = 0; c < planes; ++c) out[c * N + j] = in[c * N + s];
}

// --------------------------------------------------------------------------
// Bucketed permutation of float planes: out[c][dest[s]] = in[c][s] for a
// permutation dest of [0, N).  Moving sorted particles to the caller's order
// (and back) is a random permutation; done as one gather it reads a 128-byte
// line per 4-byte element.  Here it takes two passes whose HBM traffic is in
// whole lines: sources are cut into tiles of ts, destinations into buckets
// of 2^shift.  Pass 1 writes each element to tmp at its bucket-major
// position (runs of about ts / buckets consecutive elements per tile and
// bucket); pass 2 gives each bucket (exactly 2^shift elements, the last one
// fewer) to one workgroup, which places its elements in LDS by destination
// and writes the bucket out contiguously.  Positions within a run follow LDS
// atomic order; the output does not depend on it.
// --------------------------------------------------------------------------
struct PlaneSet {
  static constexpr int kMax = 29;  // x, v, C, F and the five parameter arrays in one launch
  const float* in[kMax];
  float* out[kMax];
  int planes;
};

// counts[b * ntiles + tile] = elements of source tile `tile` bound for bucket b
__global__ __launch_bounds__(256) void k_perm_count(const int* dest, int64_t N, int shift, int64_t ts, int nb,
                                                    int64_t ntiles, uint32_t* counts) {
  extern __shared__ uint32_t hist[];  // nb
  for (int b = threadIdx.x; b < nb; b += 256) hist[b] = 0u;
  __syncthreads();
  const int64_t s0 = (int64_t)blockIdx.x * ts, s1 = min(N, s0 + ts);
  for (int64_t s = s0 + threadIdx.x; s < s1; s += 256) {
    const uint32_t b = (uint32_t)dest[s] >> shift;
    if (b < (uint32_t)nb) atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += 256) counts[(int64_t)b * ntiles + blockIdx.x] = hist[b];
}

// pos_src[s] = bucket-major position of source s (offsets = exclusive scan of
// counts); dst_of_pos[p] = destination of the element at position p
__global__ __launch_bounds__(256) void k_perm_rank(const int* dest, int64_t N, int shift, int64_t ts, int nb,
                                                   int64_t ntiles, const uint32_t* offsets, int* pos_src,
                                                   int* dst_of_pos) {
  extern __shared__ uint32_t cur[];  // nb
  for (int b = threadIdx.x; b < nb; b += 256) cur[b] = offsets[(int64_t)b * ntiles + blockIdx.x];
  __syncthreads();
  const int64_t s0 = (int64_t)blockIdx.x * ts, s1 = min(N, s0 + ts);
  for (int64_t s = s0 + threadIdx.x; s < s1; s += 256) {
    const int d = dest[s];
    const uint32_t b = (uint32_t)d >> shift;
    if (b >= (uint32_t)nb) continue;
    const uint32_t p = atomicAdd(&cur[b], 1u);
    if (p < (uint32_t)N) {
      pos_src[s] = (int)p;
      dst_of_pos[p] = d;
    }
  }
}

// pass 1: tmp[c][pos_src[s]] = in[c][s].  Workgroup w takes source chunk
// (w mod 8) q + w / 8 (q = gridDim / 8): workgroups are dealt to the 8 XCDs
// in turn, so XCD x handles one contiguous eighth of the sources, whose
// positions in every bucket are contiguous too, and its L2 assembles whole
// lines before they are written back.
constexpr int kPermChunk = 1024;  // sources per pass-1 workgroup (256 threads x 4)
constexpr int kPermPlanes = 3;    // planes per workgroup of the LDS-staged pass 1

__global__ __launch_bounds__(256) void k_perm_pass1(float* tmp, PlaneSet ps, const int* pos_src, int64_t N) {
  const int64_t q = gridDim.x >> 3;
  const int64_t chunk = (int64_t)(blockIdx.x & 7) * q + (blockIdx.x >> 3);
  const int64_t s0 = chunk * kPermChunk;
  int64_t p[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t s = s0 + k * 256 + threadIdx.x;
    p[k] = s < N ? (int64_t)pos_src[s] : -1;
  }
  for (int c = 0; c < ps.planes; ++c) {
    const float* in = ps.in[c];
    float* t = tmp + c * N;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (p[k] >= 0) t[p[k]] = in[s0 + k * 256 + threadIdx.x];
  }
}

// Pass 1 staged through LDS, one counting tile per workgroup (tiles dealt to
// XCDs as in k_perm_pass1).  The tile's elements are placed in LDS in
// position order (bucket by bucket: bucket b = position >> shift, its run
// starts at offsets[b][tile]), so consecutive lanes store consecutive
// positions and each run goes out in whole lines.  LDS: ts floats, ts
// 16-bit bucket ids, 2 nb run starts.
__global__ __launch_bounds__(512) void k_perm_pass1_staged(float* tmp, PlaneSet ps, const int* pos_src,
                                                           const uint32_t* offsets, int64_t N, int shift, int ts,
                                                           int nb, int ntiles) {
  extern __shared__ uint32_t smem[];
  float* buf = reinterpret_cast<float*>(smem);                   // ts
  uint16_t* bk = reinterpret_cast<uint16_t*>(smem + ts);        // ts
  uint32_t* base = smem + ts + ts / 2;                          // nb: run start (position)
  uint32_t* lst = base + nb;                                    // nb: run start (local index)
  __shared__ uint32_t sh[160];
  const int q = (int)(gridDim.x >> 3);
  const int t = (int)(blockIdx.x & 7) * q + (int)(blockIdx.x >> 3);
  if (t >= ntiles) return;  // uniform over the workgroup
  const int64_t s0 = (int64_t)t * ts;
  const int nt = (int)min((int64_t)ts, N - s0);
  // runs of this tile: start and length per bucket, exclusive scan of lengths
  constexpr int kPer = 8;  // buckets per thread (nb <= 512 x 8)
  uint32_t len[kPer], sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = threadIdx.x * kPer + k;
    len[k] = 0;
    if (b < nb) {
      const uint32_t o = offsets[(int64_t)b * ntiles + t];
      const uint32_t e = (t + 1 < ntiles) ? offsets[(int64_t)b * ntiles + t + 1]
                                          : (uint32_t)min((int64_t)(b + 1) << shift, N);
      base[b] = o;
      len[k] = e - o;
    }
    sum += len[k];
  }
  uint32_t total;
  uint32_t e = block_exclusive_scan(sum, sh, total);
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int b = threadIdx.x * kPer + k;
    if (b < nb) lst[b] = e;
    e += len[k];
  }
  __syncthreads();
  // local index of each source of the tile
  constexpr int kSrc = 16;  // sources per thread (ts <= 512 x 16)
  int loc[kSrc];
#pragma unroll
  for (int k = 0; k < kSrc; ++k) {
    const int i = k * 512 + (int)threadIdx.x;
    loc[k] = -1;
    if (i < nt) {
      const uint32_t pp = (uint32_t)pos_src[s0 + i];
      const uint32_t b = pp >> shift;
      if (b < (uint32_t)nb) {
        const uint32_t l = lst[b] + (pp - base[b]);
        if (l < (uint32_t)nt) {
          loc[k] = (int)l;
          bk[l] = (uint16_t)b;
        }
      }
    }
  }
  // planes kPermPlanes blockIdx.y ... (+ kPermPlanes - 1): fewer planes per
  // workgroup put more workgroups in flight, more share the prologue
  // the next plane's loads are issued before this plane's LDS round trip
  const int c0 = blockIdx.y * kPermPlanes;
  const int c1 = min(ps.planes, c0 + kPermPlanes);
  float nxt[kSrc];
#pragma unroll
  for (int k = 0; k < kSrc; ++k) nxt[k] = loc[k] >= 0 ? ps.in[c0][s0 + k * 512 + threadIdx.x] : 0.0f;
  for (int c = c0; c < c1; ++c) {
    float cur[kSrc];
#pragma unroll
    for (int k = 0; k < kSrc; ++k) cur[k] = nxt[k];
    if (c + 1 < c1) {
      const float* in = ps.in[c + 1] + s0;
#pragma unroll
      for (int k = 0; k < kSrc; ++k) nxt[k] = loc[k] >= 0 ? in[k * 512 + threadIdx.x] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kSrc; ++k)
      if (loc[k] >= 0) buf[loc[k]] = cur[k];
    __syncthreads();
    float* out = tmp + c * N;
    for (int l = threadIdx.x; l < nt; l += 512) {
      const uint32_t b = bk[l];
      out[base[b] + (uint32_t)l - lst[b]] = buf[l];
    }
    __syncthreads();
  }
}

// pass 2: workgroup b places bucket b's elements of each plane by
// destination in LDS and writes out[c][b 2^shift ...] contiguously
// (shift <= 14: each thread keeps its up to 16 LDS destinations over all planes)
__global__ __launch_bounds__(1024) void k_perm_pass2(PlaneSet ps, const float* tmp, const int* dst_of_pos,
                                                     int64_t N, int shift) {
  extern __shared__ float buf[];  // 2^shift
  constexpr int kPer = 16;
  const int64_t base = (int64_t)blockIdx.x << shift;
  const int cnt = (int)min((int64_t)1 << shift, N - base);
  int o[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int j = k * 1024 + (int)threadIdx.x;
    o[k] = -1;
    if (j < cnt) {
      const int64_t d = (int64_t)dst_of_pos[base + j] - base;
      if (d >= 0 && d < cnt) o[k] = (int)d;
    }
  }
  // the next plane's loads are issued before this plane's LDS round trip
  float nxt[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) nxt[k] = o[k] >= 0 ? tmp[base + k * 1024 + threadIdx.x] : 0.0f;
  for (int c = 0; c < ps.planes; ++c) {
    float cur[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) cur[k] = nxt[k];
    if (c + 1 < ps.planes) {
      const float* t = tmp + (c + 1) * N + base;
#pragma unroll
      for (int k = 0; k < kPer; ++k) nxt[k] = o[k] >= 0 ? t[k * 1024 + threadIdx.x] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (o[k] >= 0) buf[o[k]] = cur[k];
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += 1024) ps.out[c][base + k] = buf[k];
    __syncthreads();
  }
}

// one-pass form for very large N: out[c][dest[s]] = in[c][s]
__global__ void k_scatter_planes(PlaneSet ps, const int* dest, int64_t N) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= N) return;
  const int64_t d = dest[s];
  for (int c = 0; c < ps.planes; ++c) ps.out[c][d] = ps.in[c][s];
}

// internal particle parameters from the sorted parameter planes (mat id as
// int bits); pid = caller index per slot
// Parameters in sorted order: prm = (mass, V0, mu, lam) with the Lame
// parameters from (log E, nu) in float64, the material id and the caller
// index.  diag[6] (float bits) is raised to the largest squared P-wave speed
// c^2 = (lam + 2 mu) V0 / m of the particles (the stiffness bound of the
// elastic CFL condition c dt / dx < 1).
__global__ void k_params_planes(float4* prm, int* mat, int* pid, const float* mass, const float* vol0,
                                const float* log_E, const float* nu, const float* mat_bits, const int* perm,
                                int64_t N, unsigned long long* diag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float c2 = 0.0f;
  if (j < N) {
    const double E = exp((double)log_E[j]);
    const double nv = (double)nu[j];
    const double mu = E / (2.0 * (1.0 + nv));
    const double la = E * nv / ((1.0 + nv) * (1.0 - 2.0 * nv));
    prm[j] = make_float4(mass[j], vol0[j], (float)mu, (float)la);
    mat[j] = __float_as_int(mat_bits[j]);
    pid[j] = perm[j];
    const double w = (la + 2.0 * mu) * (double)vol0[j] / (double)mass[j];
    c2 = (w > 0.0 && w < 3.0e38) ? (float)w : 0.0f;
  }
  c2 = wave_maxf(c2);
  if (diag && (threadIdx.x & 63) == 0) raise_max(reinterpret_cast<unsigned*>(&diag[6]), c2);
}

__global__ void k_gather_misc(float4* prm_out, int* mat_out, int* pid_out, const float4* prm_in, const int* mat_in,
                              const int* pid_in, const int* perm, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int s = perm[j];
  prm_out[j] = prm_in[s];
  mat_out[j] = mat_in[s];
  pid_out[j] = pid_in[s];
}

// inv[pid[j]] = j
__global__ void k_invert(const int* pid, int* inv, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) inv[pid[j]] = (int)j;
}

// perm_out[j] = outer[perm_in[j]]
__global__ void k_compose(const int* outer, const int* perm_in, int* perm_out, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) perm_out[j] = outer[perm_in[j]];
}

__global__ void k_iota(int* p, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) p[j] = (int)j;
}

// grid state export: m [B n^3], mv / v [B n^3][3]
__global__ void k_grid_export(const float4* grid, int64_t nodes, SubstepArgs a, float* m, float* mv, float* v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nodes) return;
  const int n = a.n;
  const int64_t loc = t % ((int64_t)n * n * n);
  const int iz = (int)(loc % n), iy = (int)((loc / n) % n), ix = (int)(loc / ((int64_t)n * n));
  const float4 g = grid[t];
  if (m) m[t] = g.w;
  if (mv) {
    mv[3 * t] = g.x;
    mv[3 * t + 1] = g.y;
    mv[3 * t + 2] = g.z;
  }
  if (v) {
    float vv[3];
    grid_velocity(g, ix, iy, iz, a, vv);
    v[3 * t] = vv[0];
    v[3 * t + 1] = vv[1];
    v[3 * t + 2] = vv[2];
  }
}

// Sigma = F Sigma0 F^T, 6 unique entries
__global__ void k_covariance(const float* F, const float* cov0, float* cov, int64_t n) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float f[9], s[6];
#pragma unroll
  for (int k = 0; k < 9; ++k) f[k] = F[k * n + p];
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = cov0[k * n + p];
  const float S[3][3] = {{s[0], s[1], s[2]}, {s[1], s[3], s[4]}, {s[2], s[4], s[5]}};
  float FS[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) FS[i][j] = f[3 * i] * S[0][j] + f[3 * i + 1] * S[1][j] + f[3 * i + 2] * S[2][j];
  const int ii[6] = {0, 0, 0, 1, 1, 2}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = ii[k], j = jj[k];
    cov[k * n + p] = FS[i][0] * f[3 * j] + FS[i][1] * f[3 * j + 1] + FS[i][2] * f[3 * j + 2];
  }
}

// BGDO key-frame signals (Alg. 1, stage 2), one particle per thread in the
// caller's order: s = |tau(F)|_F of the particle's elastic model, whose
// log E derivative is s itself (tau is linear in (mu, lam), both
// proportional to E); delta = |F_next - I|_F; with eta = min(1, 0.1 log(1 + E))
// g_total += eta log(1 + s) - (1 - eta) (delta - delta_target).
__global__ void k_bgdo_accumulate(const float* F, const float* F_next, const float* log_E, const float* nu,
                                  const int* mat_id, const Material* mats, int n_materials, float delta_target,
                                  float* g_total, float* s_out, float* d_out, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double Fd[9], Fo[9], tau[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Fd[k] = (double)F[k * N + i];
  const double E = exp((double)log_E[i]);
  const double nv = (double)nu[i];
  const double mu = E / (2.0 * (1.0 + nv));
  const double lam = E * nv / ((1.0 + nv) * (1.0 - 2.0 * nv));
  int mid = mat_id[i];
  mid = (mid >= 0 && mid < n_materials) ? mid : 0;
  update_and_stress(mats[mid], mu, lam, Fd, false, true, Fo, tau);
  double s2 = 0.0, d2 = 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    s2 += tau[k] * tau[k];
    const double d = (double)F_next[k * N + i] - (k % 4 == 0 ? 1.0 : 0.0);
    d2 += d * d;
  }
  const double sn = sqrt(s2), delta = sqrt(d2);
  const double eta = fmin(1.0, 0.1 * log1p(E));
  g_total[i] += (float)(eta * log1p(sn) - (1.0 - eta) * (delta - (double)delta_target));
  if (s_out) s_out[i] = (float)sn;
  if (d_out) d_out[i] = (float)delta;
}

// log E -= g_total / n_keys (Alg. 1, the log-space update)
__global__ void k_bgdo_apply(float* log_E, const float* g_total, float inv_keys, int64_t N) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) log_E[i] -= g_total[i] * inv_keys;
}

}  // namespace fmpm
