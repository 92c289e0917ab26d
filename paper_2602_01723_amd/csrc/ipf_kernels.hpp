// Instance-aware candidate generation (Sec. 4.1) on the GPU: candidate
// points drawn uniformly in the axis-aligned box B_k of each instance's
// convex hull H_k, kept where the ray-cast occupancy of H_k exceeds a
// threshold (0.6 in the paper).  Included once, by fastmpm.hip, after
// mcis_kernels.hpp (whose instance lookup it reuses).
//
// The hull is the caller's: a triangle mesh per instance (Quickhull of the
// instance's points in the paper).  For raw candidate j of instance k, with
// the caller's uniforms u_j in [0, 1]^3:
//   B_k   = per-axis [min, max] over the vertices the triangles use
//   q_j   = b_min + u_j (b_max - b_min), in float64, rounded to float32
//   occ   = (rays among +x, -x, +y, -y, +z, -z from q_j that cross the
//           mesh an odd number of times) / 6
//   kept  when occ > threshold; kept candidates are written in raw order.
// Crossing test of the line through q along axis a (b, c the next two axes
// cyclically), all in float64 without contraction:
//   * q's projection must lie in the closed 2D box of the triangle's
//     projection;
//   * the 2D edge functions U = B x C, V = C x A, W = A x B of the vertices
//     relative to q (each one product minus another) must share one sign s,
//     a zero taking the sign the edge function gets when q moves by
//     (e, e^2) in (b, c), e -> 0 (simulation of simplicity): first the sign
//     of p_c - q_c, then of q_b - p_b, for the directed edge p -> q.  A
//     shared edge gives its two triangles exactly opposite values, so a ray
//     through it crosses exactly one of them;
//   * the crossing lies ahead of q (counts for the + ray) when
//     s ((U A_a + V B_a) + W C_a) >= 0 and behind (the - ray) when <= 0.
// Triangles are binned per instance and axis into a 2D grid of G x G cells
// over B_k's projection; a triangle is listed in every cell its 2D box
// touches, and the cell of a coordinate is monotone in it, so every
// triangle whose box holds q's projection is listed in q's cell.  The
// count of crossings does not depend on the order in which a cell lists
// its triangles, so the result is deterministic.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmpm {

// one triangle: v0.xyz v1.x | v1.yz v2.xy | v2.z (three float4 loads)
struct IpfTri {
  float4 p, q, r;
};

// per instance and axis: cells per side and the first cell of its grid
struct IpfGrid {
  int g;
  uint32_t base;
};

__device__ __forceinline__ void ipf_unpack(const IpfTri& t, float v[3][3]) {
  v[0][0] = t.p.x, v[0][1] = t.p.y, v[0][2] = t.p.z;
  v[1][0] = t.p.w, v[1][1] = t.q.x, v[1][2] = t.q.y;
  v[2][0] = t.q.z, v[2][1] = t.q.w, v[2][2] = t.r.x;
}

// B_k as float bits: box[6k + 0..2] min (starts at +inf), [6k + 3..5] max
// (starts at 0).  Non-negative floats order as their bit patterns.
__device__ __forceinline__ bool ipf_box_valid(const uint32_t* box, int k) { return box[6 * k] != 0x7f800000u; }

__device__ __forceinline__ int ipf_cell(float x, float lo, float hi, int g) {
  const double ext = __dsub_rn((double)hi, (double)lo);
  if (!(ext > 0.0)) return 0;
  const int c = (int)__dmul_rn(__dsub_rn((double)x, (double)lo), __ddiv_rn((double)g, ext));
  return min(max(c, 0), g - 1);
}

// q = b_min + u (b_max - b_min) per axis, rounded to float32
__device__ __forceinline__ void ipf_point(const double* u, int64_t R, int64_t j, const uint32_t* box, int k,
                                          float q[3], bool& u_ok) {
  u_ok = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double ua = u[a * R + j];
    u_ok = u_ok && (ua >= 0.0 && ua <= 1.0);
    const double lo = (double)__uint_as_float(box[6 * k + a]), hi = (double)__uint_as_float(box[6 * k + 3 + a]);
    q[a] = (float)__dadd_rn(lo, __dmul_rn(ua, __dsub_rn(hi, lo)));
  }
}

__global__ void k_ipf_box_init(uint32_t* box, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 6 * K) box[i] = (i % 6 < 3) ? 0x7f800000u : 0u;
}

// Triangles: check the indices and the vertices, pack the record, and
// widen the instance's box.  A wave whose lanes all belong to one instance
// reduces the box in registers and widens it with six atomics.
__global__ __launch_bounds__(256) void k_ipf_tris(const float* hv, int64_t V, const int32_t* ht, int64_t T,
                                                  const int64_t* hv_off, const int64_t* ht_off, int K, IpfTri* tri,
                                                  uint32_t* box, unsigned long long* bad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < T;
  int k = live ? mcis_instance(ht_off, K, t) : -1;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {0.0f, 0.0f, 0.0f};
  if (live) {
    const int64_t v0 = hv_off[k], nv = hv_off[k + 1] - v0;
    float v[3][3];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int32_t idx = ht[i * T + t];
      const bool in = idx >= 0 && idx < nv;
      ok = ok && in;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float x = in ? hv[a * V + v0 + idx] : 0.0f;
        ok = ok && (x >= 0.0f && x <= 1.0f);  // NaN fails
        v[i][a] = x;
        lo[a] = fminf(lo[a], x);
        hi[a] = fmaxf(hi[a], x);
      }
    }
    if (!ok) atomicAdd(bad, 1ull);
    tri[t].p = make_float4(v[0][0], v[0][1], v[0][2], v[1][0]);
    tri[t].q = make_float4(v[1][1], v[1][2], v[2][0], v[2][1]);
    tri[t].r = make_float4(v[2][2], 0.0f, 0.0f, 0.0f);
  }
  const int k0 = __shfl(k, 0);
  if (__all(!live || k == k0)) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        lo[a] = fminf(lo[a], __shfl_xor(lo[a], o));
        hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], o));
      }
    if ((threadIdx.x & 63) == 0 && k0 >= 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        atomicMin(&box[6 * k0 + a], __float_as_uint(lo[a]));
        atomicMax(&box[6 * k0 + 3 + a], __float_as_uint(hi[a]));
      }
    }
  } else if (live) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      atomicMin(&box[6 * k + a], __float_as_uint(lo[a]));
      atomicMax(&box[6 * k + 3 + a], __float_as_uint(hi[a]));
    }
  }
}

// 2D cell range of triangle t's projection along axis a
__device__ __forceinline__ void ipf_tri_cells(const IpfTri& rec, const uint32_t* box, int k, int a, int g, int& b0,
                                              int& b1, int& c0, int& c1) {
  float v[3][3];
  ipf_unpack(rec, v);
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const float lob = __uint_as_float(box[6 * k + b]), hib = __uint_as_float(box[6 * k + 3 + b]);
  const float loc = __uint_as_float(box[6 * k + c]), hic = __uint_as_float(box[6 * k + 3 + c]);
  b0 = ipf_cell(fminf(fminf(v[0][b], v[1][b]), v[2][b]), lob, hib, g);
  b1 = ipf_cell(fmaxf(fmaxf(v[0][b], v[1][b]), v[2][b]), lob, hib, g);
  c0 = ipf_cell(fminf(fminf(v[0][c], v[1][c]), v[2][c]), loc, hic, g);
  c1 = ipf_cell(fmaxf(fmaxf(v[0][c], v[1][c]), v[2][c]), loc, hic, g);
}

// Binning, pass 1 (place = false): count the triangles of every cell and
// each grid's references; pass 2 (place = true): write the references.
// Thread = (triangle, axis).
template <bool kPlace>
__global__ __launch_bounds__(256) void k_ipf_bin(const IpfTri* tri, int64_t T, const int64_t* ht_off, int K,
                                                 const uint32_t* box, const IpfGrid* grid, uint32_t* count,
                                                 unsigned long long* refs_per_grid, const uint32_t* start,
                                                 uint32_t* cursor,
                                                 uint32_t* refs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * T) return;
  const int64_t t = i / 3;
  const int a = (int)(i - 3 * t);
  const int k = mcis_instance(ht_off, K, t);
  const IpfGrid gr = grid[3 * k + a];
  int b0, b1, c0, c1;
  ipf_tri_cells(tri[t], box, k, a, gr.g, b0, b1, c0, c1);
  for (int bb = b0; bb <= b1; ++bb)
    for (int cc = c0; cc <= c1; ++cc) {
      const uint32_t cell = gr.base + (uint32_t)(bb * gr.g + cc);
      if (kPlace)
        refs[start[cell] + atomicAdd(&cursor[cell], 1u)] = (uint32_t)t;
      else
        atomicAdd(&count[cell], 1u);
    }
  if (!kPlace && b1 >= b0 && c1 >= c0)
    atomicAdd(&refs_per_grid[3 * k + a], (unsigned long long)(b1 - b0 + 1) * (unsigned long long)(c1 - c0 + 1));
}

__device__ __forceinline__ int ipf_tie(float pb, float pc, float qb, float qc) {
  const int t1 = (pc > qc) - (pc < qc);
  return t1 ? t1 : (qb > pb) - (qb < pb);
}

__device__ __forceinline__ int ipf_sign(double e, int tie) { return e > 0.0 ? 1 : (e < 0.0 ? -1 : tie); }

// Occupancy: flag[j] = 1 when more than `threshold` of the six rays from
// q_j cross the instance's mesh an odd number of times.
__global__ __launch_bounds__(256) void k_ipf_occupancy(const double* u, int64_t R, const int64_t* ro, int K,
                                                       const uint32_t* box, const IpfGrid* grid,
                                                       const uint32_t* start, const uint32_t* refs,
                                                       const IpfTri* tri, double threshold, uint32_t* flag,
                                                       unsigned long long* bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const int k = mcis_instance(ro, K, j);
  if (!ipf_box_valid(box, k)) {  // no triangles: nothing is inside
    flag[j] = 0u;
    return;
  }
  float q[3];
  bool u_ok;
  ipf_point(u, R, j, box, k, q, u_ok);
  if (!u_ok) {
    atomicAdd(bad, 1ull);
    flag[j] = 0u;
    return;
  }
  int votes = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const IpfGrid gr = grid[3 * k + a];
    const int cb = ipf_cell(q[b], __uint_as_float(box[6 * k + b]), __uint_as_float(box[6 * k + 3 + b]), gr.g);
    const int cc = ipf_cell(q[c], __uint_as_float(box[6 * k + c]), __uint_as_float(box[6 * k + 3 + c]), gr.g);
    const uint32_t cell = gr.base + (uint32_t)(cb * gr.g + cc);
    const double qa = (double)q[a], qb = (double)q[b], qc = (double)q[c];
    int fwd = 0, bwd = 0;
    for (uint32_t r = start[cell], r1 = start[cell + 1]; r < r1; ++r) {
      float v[3][3];
      ipf_unpack(tri[refs[r]], v);
      const bool in_box = q[b] >= fminf(fminf(v[0][b], v[1][b]), v[2][b]) &&
                          q[b] <= fmaxf(fmaxf(v[0][b], v[1][b]), v[2][b]) &&
                          q[c] >= fminf(fminf(v[0][c], v[1][c]), v[2][c]) &&
                          q[c] <= fmaxf(fmaxf(v[0][c], v[1][c]), v[2][c]);
      if (!in_box) continue;
      double P[3][3];  // vertices relative to q: P[vertex][axis slot a, b, c]
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        P[i][0] = __dsub_rn((double)v[i][a], qa);
        P[i][1] = __dsub_rn((double)v[i][b], qb);
        P[i][2] = __dsub_rn((double)v[i][c], qc);
      }
      const double U = __dsub_rn(__dmul_rn(P[1][1], P[2][2]), __dmul_rn(P[1][2], P[2][1]));
      const double Vv = __dsub_rn(__dmul_rn(P[2][1], P[0][2]), __dmul_rn(P[2][2], P[0][1]));
      const double W = __dsub_rn(__dmul_rn(P[0][1], P[1][2]), __dmul_rn(P[0][2], P[1][1]));
      const int su = ipf_sign(U, ipf_tie(v[1][b], v[1][c], v[2][b], v[2][c]));
      const int sv = ipf_sign(Vv, ipf_tie(v[2][b], v[2][c], v[0][b], v[0][c]));
      const int sw = ipf_sign(W, ipf_tie(v[0][b], v[0][c], v[1][b], v[1][c]));
      if (su == 0 || su != sv || sv != sw) continue;
      const double Tn = __dadd_rn(__dadd_rn(__dmul_rn(U, P[0][0]), __dmul_rn(Vv, P[1][0])), __dmul_rn(W, P[2][0]));
      const int st = su * ((Tn > 0.0) - (Tn < 0.0));
      fwd += st >= 0;
      bwd += st <= 0;
    }
    votes += (fwd & 1) + (bwd & 1);
  }
  flag[j] = ((double)votes / 6.0 > threshold) ? 1u : 0u;
}

// offsets[k] = scanned flag at the first raw candidate of instance k
__global__ void k_ipf_offsets(const uint32_t* scan, const int64_t* ro, int K, uint32_t* offsets) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= K) offsets[k] = scan[ro[k]];
}

// Kept candidates, in raw order: out[3][M_in] (stride M_in), source[i] = j.
__global__ __launch_bounds__(256) void k_ipf_write(const double* u, int64_t R, const int64_t* ro, int K,
                                                   const uint32_t* box, const uint32_t* scan, int64_t M_in,
                                                   float* out, int64_t* source) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const uint32_t pos = scan[j];
  if (scan[j + 1] == pos) return;
  const int k = mcis_instance(ro, K, j);
  float q[3];
  bool u_ok;
  ipf_point(u, R, j, box, k, q, u_ok);
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a * M_in + pos] = q[a];
  if (source) source[pos] = j;
}

}  // namespace fmpm
