// Interior filling by instance-aware Monte Carlo importance sampling
// (Sec. 4.1, MCIS steps 1-5) on the GPU.  Included once, by fastmpm.hip,
// after mpm_kernels.hpp (whose scan kernels it reuses).
//
// Instance k owns the surface points [so_k, so_{k+1}) (the Gaussian
// centres) and the candidate points [co_k, co_{k+1}) that the caller's
// occupancy test kept.  For candidate j of instance k:
//   step 1  d_j = min over the instance's surface points of |q_j - c|_2
//   step 2  w_j = max(exp(-d_j^2 / (2 sigma^2)), eps)
//   step 3  p_j = w_j / sum w  (a positive factor common to the instance)
//   step 4  the n_k largest exponential keys log(u_j) / p_j are drawn
//           (sampling without replacement, Efraimidis & Spirakis 2006); the
//           common factor of step 3 does not change their order, so the
//           keys ranked here are log(u_j) / w_j;
//   step 5  the selections of all instances are written one after another.
//
// Nearest-surface search on a two-level uniform grid over [0, 1]^3:
//   * coarse cells of the search radius r_s = sigma sqrt(-2 ln eps) (the
//     distance where w reaches its floor, widened by 1e-9): a candidate
//     whose 27 coarse neighbours hold no surface point of its instance has
//     w = eps without a search;
//   * fine cells of r_s / rings (widened by 1e-9, so ring `rings` covers
//     the radius), searched ring by ring (Chebyshev shells of cells around
//     the candidate's cell).  After ring r every unvisited point is at least
//     r h away, so the search stops as soon as the best distance is within
//     r h, and at ring `rings` at the latest; a nearest point beyond r_s
//     counts as none (w = eps either way).  The candidates are first
//     counting-sorted by fine cell, so the lanes of a wave search nearly the
//     same cells.
// Distances are evaluated in float64 without contraction, in the order
// ((dx dx + dy dy) + dz dz), so the minimum is the same number a plain
// float64 evaluation gives.
//
// Selection: an MSB-first radix select over the 64-bit order-preserving
// image of the keys, eight 8-bit digits, all instances at once, finds each
// instance's n_k-th largest key T_k; keys above T_k are taken, and keys
// equal to T_k by ascending candidate index until n_k are taken.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace fmpm {

constexpr int kMcisRings = 12;       // fine cells per search radius (fewer when the grid would be too large)
constexpr int kMcisChunk = 4096;     // candidates per histogram chunk

struct McisGrid {
  int rings;           // fine cells per search radius
  int gf, gc;          // fine / coarse cells per axis over [0, 1]
  double hf, hc;       // fine / coarse cell size
  double r2;           // squared search radius
};

// instance of element j: the largest k with off[k] <= j (off ascending)
__device__ __forceinline__ int mcis_instance(const int64_t* off, int K, int64_t j) {
  int lo = 0, hi = K - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= j)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ bool mcis_in_domain(float x, float y, float z) {
  return x >= 0.0f && x <= 1.0f && y >= 0.0f && y <= 1.0f && z >= 0.0f && z <= 1.0f;
}

__device__ __forceinline__ int mcis_cell(float x, double h, int g) {
  return min((int)((double)x / h), g - 1);
}

// order-preserving map of a double onto uint64 (larger key -> larger image)
__device__ __forceinline__ uint64_t mcis_order(double k) {
  const uint64_t b = (uint64_t)__double_as_longlong(k);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Surface points: validate, flag their coarse cell, count their fine cell
// and remember their rank in it.
__global__ void k_mcis_bin_surface(const float* surf, int64_t S, const int64_t* so, int K, McisGrid g,
                                   uint32_t* fine_count, uint32_t* coarse_flag, uint32_t* key, uint32_t* slot,
                                   unsigned long long* bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S) return;
  const float x = surf[j], y = surf[S + j], z = surf[2 * S + j];
  if (!mcis_in_domain(x, y, z)) {  // NaN fails the test too
    atomicAdd(bad, 1ull);
    key[j] = 0xffffffffu;
    return;
  }
  const int k = mcis_instance(so, K, j);
  const int64_t g3 = (int64_t)g.gf * g.gf * g.gf, c3 = (int64_t)g.gc * g.gc * g.gc;
  const int64_t cf = ((int64_t)mcis_cell(x, g.hf, g.gf) * g.gf + mcis_cell(y, g.hf, g.gf)) * g.gf +
                     mcis_cell(z, g.hf, g.gf);
  const int64_t cc = ((int64_t)mcis_cell(x, g.hc, g.gc) * g.gc + mcis_cell(y, g.hc, g.gc)) * g.gc +
                     mcis_cell(z, g.hc, g.gc);
  coarse_flag[k * c3 + cc] = 1u;
  const uint32_t kk = (uint32_t)(k * g3 + cf);
  key[j] = kk;
  slot[j] = atomicAdd(&fine_count[kk], 1u);
}

// Candidates: count their fine cell and remember their rank in it, so the
// search can run in cell order (neighbouring lanes walk the same cells).
// Out-of-domain candidates go to an extra bin past the last cell.
__global__ void k_mcis_bin_candidates(const float* cand, int64_t M, const int64_t* co, int K, McisGrid g,
                                      uint32_t* count, uint32_t* key, uint32_t* slot) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  const float x = cand[j], y = cand[M + j], z = cand[2 * M + j];
  const int64_t g3 = (int64_t)g.gf * g.gf * g.gf;
  uint32_t kk = (uint32_t)((int64_t)K * g3);  // the extra bin
  if (mcis_in_domain(x, y, z)) {
    const int k = mcis_instance(co, K, j);
    kk = (uint32_t)(k * g3 + ((int64_t)mcis_cell(x, g.hf, g.gf) * g.gf + mcis_cell(y, g.hf, g.gf)) * g.gf +
                    mcis_cell(z, g.hf, g.gf));
  }
  key[j] = kk;
  slot[j] = atomicAdd(&count[kk], 1u);
}

// order[start[key[j]] + slot[j]] = j
__global__ void k_mcis_place_candidates(int64_t M, const uint32_t* key, const uint32_t* slot, const uint32_t* start,
                                        uint32_t* order) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < M) order[start[key[j]] + slot[j]] = (uint32_t)j;
}

// Scatter the surface points into fine-cell order (start = exclusive scan of
// the counts); float4 per point for one load in the search.
__global__ void k_mcis_place_surface(const float* surf, int64_t S, const uint32_t* key, const uint32_t* slot,
                                     const uint32_t* start, float4* sorted) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= S || key[j] == 0xffffffffu) return;
  sorted[start[key[j]] + slot[j]] = make_float4(surf[j], surf[S + j], surf[2 * S + j], 0.0f);
}

// Steps 1, 2 and the key of step 4 for every candidate.
// start: exclusive scan of the fine-cell counts over K g^3 + 1 entries, so
// cell c holds sorted[start[c] .. start[c + 1]).
// Thread t handles candidate j = order[t] (candidates in fine-cell order).
__global__ void k_mcis_keys(const float* cand, int64_t M, const int64_t* co, int K, const double* u, McisGrid g,
                            double sigma, double eps, const uint32_t* coarse_flag, const uint32_t* start,
                            const float4* sorted, const uint32_t* order, uint64_t* okey, double* d_out,
                            unsigned long long* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M) return;
  const int64_t j = order[t];
  const float x = cand[j], y = cand[M + j], z = cand[2 * M + j];
  const double uj = u[j];
  if (!mcis_in_domain(x, y, z) || !(uj > 0.0 && uj <= 1.0)) {
    atomicAdd(bad, 1ull);
    okey[j] = 0;
    if (d_out) d_out[j] = NAN;
    return;
  }
  const int k = mcis_instance(co, K, j);
  const int64_t g3 = (int64_t)g.gf * g.gf * g.gf, c3 = (int64_t)g.gc * g.gc * g.gc;
  // coarse test: any surface point of the instance within the search radius?
  bool near = false;
  {
    const int cx = mcis_cell(x, g.hc, g.gc), cy = mcis_cell(y, g.hc, g.gc), cz = mcis_cell(z, g.hc, g.gc);
    for (int a = max(cx - 1, 0); a <= min(cx + 1, g.gc - 1) && !near; ++a)
      for (int b = max(cy - 1, 0); b <= min(cy + 1, g.gc - 1) && !near; ++b)
        for (int c = max(cz - 1, 0); c <= min(cz + 1, g.gc - 1); ++c)
          if (coarse_flag[k * c3 + ((int64_t)a * g.gc + b) * g.gc + c]) {
            near = true;
            break;
          }
  }
  double best = INFINITY;  // squared distance
  if (near) {
    const double qx = (double)x, qy = (double)y, qz = (double)z;
    const int fx = mcis_cell(x, g.hf, g.gf), fy = mcis_cell(y, g.hf, g.gf), fz = mcis_cell(z, g.hf, g.gf);
    const uint32_t* st = start + k * g3;
    for (int r = 0; r <= g.rings; ++r) {
      for (int a = fx - r; a <= fx + r; ++a) {
        if (a < 0 || a >= g.gf) continue;
        for (int b = fy - r; b <= fy + r; ++b) {
          if (b < 0 || b >= g.gf) continue;
          const bool face_ab = (a == fx - r || a == fx + r || b == fy - r || b == fy + r);
          // on ring r only the shell: all c if (a, b) is on the shell, else c = fz +- r
          for (int c = fz - r; c <= fz + r; c += (face_ab || r == 0) ? 1 : 2 * r) {
            if (c < 0 || c >= g.gf) continue;
            const int64_t cell = ((int64_t)a * g.gf + b) * g.gf + c;
            const uint32_t s0 = st[cell], s1 = st[cell + 1];
            for (uint32_t q = s0; q < s1; ++q) {
              const float4 p = sorted[q];
              const double dx = __dsub_rn(qx, (double)p.x), dy = __dsub_rn(qy, (double)p.y),
                           dz = __dsub_rn(qz, (double)p.z);
              const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
              best = fmin(best, d2);
            }
          }
        }
      }
      const double reach = (double)r * g.hf * (1.0 - 1e-9);  // every unvisited point is this far or farther
      if (best <= reach * reach) break;
    }
    if (!(best <= g.r2)) best = INFINITY;  // beyond the search radius: the weight floor
  }
  const double d = sqrt(best);
  const double w = (d < INFINITY) ? fmax(exp(-(d * d) / (2.0 * sigma * sigma)), eps) : eps;
  okey[j] = mcis_order(log(uj) / w);
  if (d_out) d_out[j] = d;
}

// Radix select, one pass: histogram of the digit at `shift` over the keys
// that match each instance's decided prefix.  Chunks of kMcisChunk
// candidates use an LDS histogram for the chunk's first instance.
__global__ void k_mcis_hist(const uint64_t* okey, int64_t M, const int64_t* co, int K, const uint64_t* prefix,
                            const int64_t* rank, int shift, uint32_t* hist) {
  __shared__ uint32_t h[256];
  const uint64_t mask = (shift >= 56) ? 0ull : (~0ull << (shift + 8));
  for (int64_t c0 = (int64_t)blockIdx.x * kMcisChunk; c0 < M; c0 += (int64_t)gridDim.x * kMcisChunk) {
    const int64_t c1 = min(c0 + (int64_t)kMcisChunk, M);
    const int k0 = mcis_instance(co, K, c0);
    for (int t = threadIdx.x; t < 256; t += blockDim.x) h[t] = 0u;
    __syncthreads();
    for (int64_t j = c0 + threadIdx.x; j < c1; j += blockDim.x) {
      const int k = (j < co[k0 + 1]) ? k0 : mcis_instance(co, K, j);
      if (rank[k] <= 0) continue;  // instance already decided (nothing or everything)
      const uint64_t v = okey[j];
      if ((v & mask) != prefix[k]) continue;
      const uint32_t digit = (uint32_t)((v >> shift) & 255u);
      if (k == k0)
        atomicAdd(&h[digit], 1u);
      else
        atomicAdd(&hist[k * 256 + digit], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 256; t += blockDim.x)
      if (h[t]) atomicAdd(&hist[k0 * 256 + t], h[t]);
    __syncthreads();
  }
}

// Radix select, one pass: per instance pick the digit holding the rank-th
// largest key, narrow the prefix and the rank, and clear the histogram.
__global__ void k_mcis_pick(int K, int shift, uint32_t* hist, uint64_t* prefix, int64_t* rank) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  uint32_t* h = hist + k * 256;
  if (rank[k] > 0) {
    int64_t above = 0;
    int d = 255;
    for (; d > 0; --d) {
      if (above + (int64_t)h[d] >= rank[k]) break;
      above += h[d];
    }
    rank[k] -= above;
    prefix[k] |= (uint64_t)d << shift;
  }
  for (int t = 0; t < 256; ++t) h[t] = 0u;
}

// eq[j] = 1 if the key equals its instance's threshold (then scanned to rank ties by index)
__global__ void k_mcis_eq(const uint64_t* okey, int64_t M, const int64_t* co, int K, const uint64_t* thr,
                          uint32_t* eq) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  eq[j] = (okey[j] == thr[mcis_instance(co, K, j)]) ? 1u : 0u;
}

__device__ __forceinline__ bool mcis_taken(const uint64_t* okey, const int64_t* co, int K, const uint64_t* thr,
                                           const int64_t* tie, const uint32_t* eqscan, int64_t j, int& k) {
  k = mcis_instance(co, K, j);
  const uint64_t v = okey[j];
  if (v > thr[k]) return true;
  return v == thr[k] && (int64_t)(eqscan[j] - eqscan[co[k]]) < tie[k];
}

__global__ void k_mcis_sel(const uint64_t* okey, int64_t M, const int64_t* co, int K, const uint64_t* thr,
                           const int64_t* tie, const uint32_t* eqscan, uint32_t* sel) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int k;
  sel[j] = mcis_taken(okey, co, K, thr, tie, eqscan, j, k) ? 1u : 0u;
}

__global__ void k_mcis_write(const uint64_t* okey, int64_t M, const int64_t* co, int K, const uint64_t* thr,
                             const int64_t* tie, const uint32_t* eqscan, const uint32_t* selscan,
                             const int64_t* out_off, int64_t* out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= M) return;
  int k;
  if (mcis_taken(okey, co, K, thr, tie, eqscan, j, k))
    out[out_off[k] + (int64_t)(selscan[j] - selscan[co[k]])] = j;
}

}  // namespace fmpm
