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
// accumulates in an LDS tile covering the chunk's stencil box with
// staggered per-lane node order (lanes of one cell hit different nodes),
// then flushes the tile with one global FP32 atomic per node and channel.
// Chunks whose box exceeds the LDS tile fall back to global memory.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_math.hpp"

namespace fmpm {

constexpr int kBlock = 256;         // threads per workgroup = particles per chunk
constexpr int kTileCapMax = 1024;   // LDS tile nodes (4 double planes = 32 KiB)
constexpr int kMaxMaterials = 16;

enum { kP2G = 0, kFused = 1, kG2P = 2 };

struct SubstepArgs {
  float* x;
  float* v;
  float* C;
  float* F;
  const float4* prm;
  const int* mat;
  int64_t N;  // plane stride
  const int* chunk_start;  // [n_chunks + 1]
  const int* chunk_batch;  // [n_chunks]
  const int* n_chunks;     // device scalar
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
  Material mats[kMaxMaterials];
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
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
// The substep kernel
// --------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_substep(SubstepArgs a) {
  __shared__ double tile_d[4 * kTileCapMax];  // P2G: 4 double planes; G2P: 3 float planes
  float* tile = reinterpret_cast<float*>(tile_d);
  __shared__ int red[8 * (kBlock / 64)];
  __shared__ int box_s[6];

  const int n_chunks = *a.n_chunks;
  for (int chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
  const int start = a.chunk_start[chunk], end = a.chunk_start[chunk + 1];
  const int i = start + (int)threadIdx.x;
  const bool live = i < end;
  const int n = a.n;
  const int64_t gbase = (int64_t)a.chunk_batch[chunk] * n * n * n;
  const int64_t N = a.N;
  const float inv_dx = (float)n, dx = 1.0f / (float)n;
  const int cap = a.tile_cap;

  float xp[3] = {0.f, 0.f, 0.f}, vp[3] = {0.f, 0.f, 0.f}, Fd_f[9];
  float Cp[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  double Fd[9];
  float4 prm = make_float4(0.f, 0.f, 0.f, 0.f);
  int mid = 0;
  if (live) {
#pragma unroll
    for (int k = 0; k < 3; ++k) xp[k] = a.x[k * N + i];
#pragma unroll
    for (int k = 0; k < 9; ++k) Fd_f[k] = a.F[k * N + i];
    prm = a.prm[i];
    mid = a.mat[i];
    if (MODE == kP2G) {
#pragma unroll
      for (int k = 0; k < 3; ++k) vp[k] = a.v[k * N + i];
#pragma unroll
      for (int k = 0; k < 9; ++k) Cp[k] = a.C[k * N + i];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) Fd_f[k] = (k % 4 == 0) ? 1.f : 0.f;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) Fd[k] = (double)Fd_f[k];
  mid = (mid >= 0 && mid < a.n_materials) ? mid : 0;
  const Material mat = a.mats[mid];
  const double mu = (double)prm.z, lam = (double)prm.w;

  // SVD of the F whose stress enters P2G, kept for the stress
  double U[3][3], sig[3], V[3][3];
  bool ok = live;

  // ---------------------------------------------------------------- G2P
  if (MODE == kFused || MODE == kG2P) {
    int b0[3];
    float f0[3];
    bool in_grid = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) in_grid &= cell_of(xp[k], n, b0[k], f0[k]);
    const bool valid = live && in_grid;
    count_event(a.diag, 1, live && !in_grid);
    ok = valid;
    int box[6];
    block_box(valid, b0, red, box);
    const int ex = box[3] - box[0] + 3, ey = box[4] - box[1] + 3, ez = box[5] - box[2] + 3;
    const bool empty = box[0] > box[3];
    const int T = empty ? 0 : ex * ey * ez;
    const bool use_lds = !empty && T <= cap;
    if (!empty && !use_lds && threadIdx.x == 0) atomicAdd(&a.diag[2], 1ull);
    if (use_lds) {
      for (int t = threadIdx.x; t < T; t += kBlock) {
        const int tk = t % ez, tq = t / ez;
        const int tj = tq % ey, ti = tq / ey;
        const int ix = box[0] + ti, iy = box[1] + tj, iz = box[2] + tk;
        const float4 g = a.grid_in[gbase + ((int64_t)ix * n + iy) * n + iz];
        float vv[3];
        grid_velocity(g, ix, iy, iz, a, vv);
        tile[t] = vv[0];
        tile[cap + t] = vv[1];
        tile[2 * cap + t] = vv[2];
      }
    }
    __syncthreads();
    if (valid) {
      float wx[3], wy[3], wz[3];
      bspline_w(f0[0], wx);
      bspline_w(f0[1], wy);
      bspline_w(f0[2], wz);
      float vs[3] = {0.f, 0.f, 0.f};
      float M[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // sum w v_a o_b
      const int sz = ey * ez;
      const int a0 = ((b0[0] - box[0]) * ey + (b0[1] - box[1])) * ez + (b0[2] - box[2]);
#pragma unroll
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
          const float wxy = wx[ox] * wy[oy];
          const int row = a0 + ox * sz + oy * ez;
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            const float w = wxy * wz[oz];
            float vi[3];
            if (use_lds) {
              vi[0] = tile[row + oz];
              vi[1] = tile[cap + row + oz];
              vi[2] = tile[2 * cap + row + oz];
            } else {
              const int ix = b0[0] + ox, iy = b0[1] + oy, iz = b0[2] + oz;
              grid_velocity(a.grid_in[gbase + ((int64_t)ix * n + iy) * n + iz], ix, iy, iz, a, vi);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float wv = w * vi[c];
              vs[c] += wv;
              if (ox) M[c][0] += (float)ox * wv;
              if (oy) M[c][1] += (float)oy * wv;
              if (oz) M[c][2] += (float)oz * wv;
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
      // F_trial = (I + dt C') F, in double
      double Ftr[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double s = Fd[3 * r + c];
#pragma unroll
          for (int k = 0; k < 3; ++k) s += (double)a.dt * (double)Cp[3 * r + k] * Fd[3 * k + c];
          Ftr[3 * r + c] = s;
        }
      if (MODE == kFused || mat.plastic != 0) {
        svd3(Ftr, U, sig, V);
        double sig2[3];
        return_map(mat, mu, lam, Ftr, U, sig, V, Fd, sig2);
#pragma unroll
        for (int k = 0; k < 3; ++k) sig[k] = sig2[k];
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) Fd[k] = Ftr[k];
      }
#pragma unroll
      for (int k = 0; k < 9; ++k) Fd_f[k] = (float)Fd[k];
      bool fin = true;
#pragma unroll
      for (int k = 0; k < 3; ++k) fin &= isfinite(xp[k]);
#pragma unroll
      for (int k = 0; k < 9; ++k) fin &= isfinite(Fd_f[k]);
      count_event(a.diag, 0, !fin);
#pragma unroll
      for (int k = 0; k < 3; ++k) a.x[k * N + i] = xp[k];
#pragma unroll
      for (int k = 0; k < 9; ++k) a.F[k * N + i] = Fd_f[k];
      if (MODE == kG2P || a.write_vc) {
#pragma unroll
        for (int k = 0; k < 3; ++k) a.v[k * N + i] = vp[k];
#pragma unroll
        for (int k = 0; k < 9; ++k) a.C[k * N + i] = Cp[k];
      }
    }
    __syncthreads();  // everyone is done reading the G2P tile
    if (MODE == kG2P) continue;
  }

  // ---------------------------------------------------------------- P2G
  if (MODE == kP2G || MODE == kFused) {
    if (MODE == kP2G && ok) svd3(Fd, U, sig, V);
    // A = m C - 4/dx^2 dt V0 tau, folded with dx for the node offsets
    float q[3], Ad[9];
    const float mass = prm.x;
    {
      double tau[9];
      if (ok) {
        kirchhoff(mat, mu, lam, Fd, U, sig, V, tau);
      } else {
#pragma unroll
        for (int k = 0; k < 9; ++k) tau[k] = 0.0;
      }
      const float ks = 4.0f * inv_dx * inv_dx * a.dt * prm.y;
#pragma unroll
      for (int k = 0; k < 9; ++k) Ad[k] = (mass * Cp[k] - ks * (float)tau[k]) * dx;
    }
    int b1[3];
    float f1[3];
    bool in_grid = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) in_grid &= cell_of(xp[k], n, b1[k], f1[k]);
    if (MODE == kP2G) count_event(a.diag, 1, live && !in_grid);
    // contribution to node o: w (m v + A (o - f) dx) = w (q + Ad o)
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = mass * vp[r] - (Ad[3 * r] * f1[0] + Ad[3 * r + 1] * f1[1] + Ad[3 * r + 2] * f1[2]);
    const bool valid = ok && in_grid;
    int box[6];
    block_box(valid, b1, red, box);
    const int ex = box[3] - box[0] + 3, ey = box[4] - box[1] + 3, ez = box[5] - box[2] + 3;
    const bool empty = box[0] > box[3];
    const int T = empty ? 0 : ex * ey * ez;
    const bool use_lds = !empty && T <= cap;
    if (!empty && !use_lds && threadIdx.x == 0) atomicAdd(&a.diag[2], 1ull);
    // The LDS tile accumulates in double: native LDS f64 atomic adds run far
    // faster than f32 ones on this chip, and the sum is more accurate.
    if (use_lds) {
      for (int t = threadIdx.x; t < T; t += kBlock) {
        tile_d[t] = 0.0;
        tile_d[cap + t] = 0.0;
        tile_d[2 * cap + t] = 0.0;
        tile_d[3 * cap + t] = 0.0;
      }
    }
    __syncthreads();
    if (valid) {
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
      const int sz = ey * ez;
      const int a0 = ((b1[0] - box[0]) * ey + (b1[1] - box[1])) * ez + (b1[2] - box[2]);
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
          const int row = a0 + r[0][kx] * sz + r[1][ky] * ez;
#pragma unroll
          for (int kz = 0; kz < 3; ++kz) {
            const float oz = (float)r[2][kz];
            const float wgt = wxy * wr[2][kz];
            float val[4];
#pragma unroll
            for (int c = 0; c < 3; ++c) val[c] = wgt * (vy[c] + Ad[3 * c + 2] * oz);
            val[3] = wgt * mass;
            if (use_lds) {
              const int t = row + r[2][kz];
#pragma unroll
              for (int c = 0; c < 4; ++c) atomicAdd(&tile_d[c * cap + t], (double)val[c]);
            } else {
              const int ix = b1[0] + r[0][kx], iy = b1[1] + r[1][ky], iz = b1[2] + r[2][kz];
              float* gp = (float*)&a.grid_out[gbase + ((int64_t)ix * n + iy) * n + iz];
#pragma unroll
              for (int c = 0; c < 4; ++c) atomicAdd(gp + c, val[c]);
            }
          }
        }
      }
    }
    __syncthreads();
    if (use_lds) {
      for (int t = threadIdx.x; t < T; t += kBlock) {
        const double m = tile_d[3 * cap + t];
        if (m == 0.0) continue;
        const int tk = t % ez, tq = t / ez;
        const int tj = tq % ey, ti = tq / ey;
        float* gp = (float*)&a.grid_out[gbase + ((int64_t)(box[0] + ti) * n + (box[1] + tj)) * n + (box[2] + tk)];
        atomicAdd(gp + 0, (float)tile_d[t]);
        atomicAdd(gp + 1, (float)tile_d[cap + t]);
        atomicAdd(gp + 2, (float)tile_d[2 * cap + t]);
        atomicAdd(gp + 3, (float)m);
      }
    }
    __syncthreads();  // the tile is reused by the next chunk
  }
  }  // chunk loop
}


// --------------------------------------------------------------------------
// Fill, sort (counting sort by cell key), gather / scatter
// --------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n4 = n >> 2;
  if (i < n4) reinterpret_cast<uint4*>(p)[i] = make_uint4(v, v, v, v);
  const int64_t t = (n4 << 2) + i;
  if (i < (n & 3)) p[t] = v;
}

// key = scene * bins_per_scene + block(4^3 cells, linear) * 64 + morton(cell in block)
__device__ __forceinline__ uint32_t spread2(uint32_t v) {  // 2 bits -> positions 0, 3
  return (v & 1u) | ((v & 2u) << 2);
}

__global__ void k_cell_keys(const float* x, int64_t N, const int* chunk_start, const int* chunk_batch, int n, int nb,
                            uint32_t* key, uint32_t* slot, uint32_t* count) {
  const int chunk = blockIdx.x;
  const int i = chunk_start[chunk] + (int)threadIdx.x;
  if (i >= chunk_start[chunk + 1]) return;
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double t = (double)x[k * N + i] * (double)n - 0.5;
    int b = (t >= 0.0) ? (t < (double)(n - 1) ? (int)floor(t) : n - 1) : 0;  // NaN -> 0
    c[k] = b;
  }
  const uint32_t blk = ((uint32_t)(c[0] >> 2) * nb + (uint32_t)(c[1] >> 2)) * nb + (uint32_t)(c[2] >> 2);
  const uint32_t mort = spread2(c[0] & 3) << 2 | spread2(c[1] & 3) << 1 | spread2(c[2] & 3);
  const uint32_t k = (uint32_t)chunk_batch[chunk] * (uint32_t)(nb * nb * nb * 64) + blk * 64u + mort;
  key[i] = k;
  slot[i] = atomicAdd(&count[k], 1u);
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

// Chunk table after a sort: each 4^3-cell block's particles (a contiguous
// range of the sorted order) are cut into chunks of at most kBlock.
// off = exclusive bin offsets (64 bins per block), nchk[b] = chunks of block b.
__global__ void k_block_chunk_count(const uint32_t* off, int64_t nblocks, int64_t N, uint32_t* nchk) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const uint32_t lo = off[b * 64];
  const uint32_t hi = (b + 1 < nblocks) ? off[(b + 1) * 64] : (uint32_t)N;
  nchk[b] = (hi - lo + kBlock - 1) / kBlock;
}

// base = exclusive scan of nchk (same array, scanned in place beforehand)
__global__ void k_block_chunk_write(const uint32_t* off, const uint32_t* base, int64_t nblocks, int64_t N,
                                    int blocks_per_scene, int* chunk_start, int* chunk_batch, int* n_chunks) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblocks) return;
  const uint32_t lo = off[b * 64];
  const uint32_t hi = (b + 1 < nblocks) ? off[(b + 1) * 64] : (uint32_t)N;
  const uint32_t c0 = base[b];
  const int scene = (int)(b / blocks_per_scene);
  uint32_t c = c0;
  for (uint32_t s = lo; s < hi; s += kBlock, ++c) {
    chunk_start[c] = (int)s;
    chunk_batch[c] = scene;
  }
  if (b == nblocks - 1) {
    chunk_start[c] = (int)N;
    *n_chunks = (int)c;
  }
}

// out[c][j] = in[c][perm[j]] for `planes` planes of stride N
__global__ void k_gather_planes(float* out, const float* in, const int* perm, int planes, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t s = perm[j];
  for (int c = 0; c < planes; ++c) out[c * N + j] = in[c * N + s];
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

// internal arrays from the caller's (perm = caller index of each sorted slot)
__global__ void k_gather_params(float4* prm, int* mat, int* pid, const float* mass, const float* vol0,
                                const float* log_E, const float* nu, const int* mat_id, const int* perm, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int s = perm[j];
  const double E = exp((double)log_E[s]);
  const double nv = (double)nu[s];
  const double mu = E / (2.0 * (1.0 + nv));
  const double la = E * nv / ((1.0 + nv) * (1.0 - 2.0 * nv));
  prm[j] = make_float4(mass[s], vol0[s], (float)mu, (float)la);
  mat[j] = mat_id[s];
  pid[j] = s;
}

// out[c][pid[j]] = in[c][j]
__global__ void k_scatter_planes(float* out, const float* in, const int* pid, int planes, int64_t N) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t d = pid[j];
  for (int c = 0; c < planes; ++c) out[c * N + d] = in[c * N + j];
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

}  // namespace fmpm
