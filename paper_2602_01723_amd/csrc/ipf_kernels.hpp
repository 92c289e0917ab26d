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
// triangle whose box holds q's projection is listed in q's cell.  The raw
// candidates are then put in column order (by that cell, per axis) so that
// the lanes of a wave test the same triangles.  The count of crossings does
// not depend on the order of a cell's triangles or of a column's
// candidates, so the result is deterministic.
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

// Widen box k to [lo, hi]; an atomic only where the stored bound is not
// already at least as wide (every wave of an instance targets the same six
// words, and most find them settled).
__device__ __forceinline__ void ipf_widen_box(uint32_t* box, int k, const float lo[3], const float hi[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t l = __float_as_uint(lo[a]), h = __float_as_uint(hi[a]);
    if (l < __atomic_load_n(&box[6 * k + a], __ATOMIC_RELAXED)) atomicMin(&box[6 * k + a], l);
    if (h > __atomic_load_n(&box[6 * k + 3 + a], __ATOMIC_RELAXED)) atomicMax(&box[6 * k + 3 + a], h);
  }
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
    if ((threadIdx.x & 63) == 0 && k0 >= 0) ipf_widen_box(box, k0, lo, hi);
  } else if (live) {
    ipf_widen_box(box, k, lo, hi);
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
// Thread = triangle, for the three axes; a wave whose lanes all belong to
// one instance adds its reference counts with one atomic per axis.
template <bool kPlace>
__global__ __launch_bounds__(256) void k_ipf_bin(const IpfTri* tri, int64_t T, const int64_t* ht_off, int K,
                                                 const uint32_t* box, const IpfGrid* grid, uint32_t* count,
                                                 unsigned long long* refs_per_grid, const uint32_t* start,
                                                 uint32_t* cursor, uint32_t* refs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = t < T;
  const int k = live ? mcis_instance(ht_off, K, t) : -1;
  unsigned long long nref[3] = {0ull, 0ull, 0ull};
  if (live) {
    const IpfTri rec = tri[t];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const IpfGrid gr = grid[3 * k + a];
      int b0, b1, c0, c1;
      ipf_tri_cells(rec, box, k, a, gr.g, b0, b1, c0, c1);
      for (int bb = b0; bb <= b1; ++bb)
        for (int cc = c0; cc <= c1; ++cc) {
          const uint32_t cell = gr.base + (uint32_t)(bb * gr.g + cc);
          if (kPlace)
            refs[start[cell] + atomicAdd(&cursor[cell], 1u)] = (uint32_t)t;
          else
            atomicAdd(&count[cell], 1u);
        }
      if (b1 >= b0 && c1 >= c0) nref[a] = (unsigned long long)(b1 - b0 + 1) * (unsigned long long)(c1 - c0 + 1);
    }
  }
  if (kPlace) return;
  const int k0 = __shfl(k, 0);
  if (__all(!live || k == k0)) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) nref[a] += __shfl_xor(nref[a], o);
    if ((threadIdx.x & 63) == 0 && k0 >= 0)
#pragma unroll
      for (int a = 0; a < 3; ++a) atomicAdd(&refs_per_grid[3 * k0 + a], nref[a]);
  } else if (live) {
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(&refs_per_grid[3 * k + a], nref[a]);
  }
}

__device__ __forceinline__ int ipf_tie(float pb, float pc, float qb, float qc) {
  const int t1 = (pc > qc) - (pc < qc);
  return t1 ? t1 : (qb > pb) - (qb < pb);
}

__device__ __forceinline__ int ipf_sign(double e, int tie) { return e > 0.0 ? 1 : (e < 0.0 ? -1 : tie); }

// Column (2D cell of the axis-a grid) of a point of instance k
__device__ __forceinline__ uint32_t ipf_column(const float q[3], const uint32_t* box, int k, int a,
                                               const IpfGrid& gr) {
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  const int cb = ipf_cell(q[b], __uint_as_float(box[6 * k + b]), __uint_as_float(box[6 * k + 3 + b]), gr.g);
  const int cc = ipf_cell(q[c], __uint_as_float(box[6 * k + c]), __uint_as_float(box[6 * k + 3 + c]), gr.g);
  return gr.base + (uint32_t)(cb * gr.g + cc);
}

// Raw candidates: q_j into qbuf (w = the instance, as int bits, or -1 when
// the instance has no triangles or u_j is invalid), and each valid one
// counted in its column of every axis.
__global__ __launch_bounds__(256) void k_ipf_points(const double* u, int64_t R, const int64_t* ro, int K,
                                                    const uint32_t* box, const IpfGrid* grid, float4* qbuf,
                                                    uint32_t* ccount, unsigned long long* bad) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const int k = mcis_instance(ro, K, j);
  if (!ipf_box_valid(box, k)) {  // no triangles: nothing is inside
    qbuf[j] = make_float4(0.0f, 0.0f, 0.0f, __int_as_float(-1));
    return;
  }
  float q[3];
  bool u_ok;
  ipf_point(u, R, j, box, k, q, u_ok);
  if (!u_ok) atomicAdd(bad, 1ull);
  qbuf[j] = make_float4(q[0], q[1], q[2], __int_as_float(u_ok ? k : -1));
  if (!u_ok) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) atomicAdd(&ccount[ipf_column(q, box, k, a, grid[3 * k + a])], 1u);
}

// Column order: order[cstart[col] + rank] = j | a << 30 for each valid
// candidate j and axis a (rank within the column in atomic order: the
// crossing counts do not depend on it).
__global__ __launch_bounds__(256) void k_ipf_columns(const float4* qbuf, int64_t R, const uint32_t* box,
                                                     const IpfGrid* grid, const uint32_t* cstart, uint32_t* ccursor,
                                                     uint32_t* order) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const float4 p = qbuf[j];
  const int k = __float_as_int(p.w);
  if (k < 0) return;
  const float q[3] = {p.x, p.y, p.z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const uint32_t col = ipf_column(q, box, k, a, grid[3 * k + a]);
    order[cstart[col] + atomicAdd(&ccursor[col], 1u)] = (uint32_t)j | ((uint32_t)a << 30);
  }
}

// Crossings of the line through q along axis A with the triangles listed
// in column `col`: bit 0 = odd count ahead (+ ray), bit 1 = odd behind.
template <int A>
__device__ __forceinline__ uint32_t ipf_parity(const float q[3], uint32_t col, const uint32_t* start,
                                               const uint32_t* refs, const IpfTri* tri) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  const double qa = (double)q[A], qb = (double)q[B], qc = (double)q[C];
  int fwd = 0, bwd = 0;
  for (uint32_t r = start[col], r1 = start[col + 1]; r < r1; ++r) {
    float v[3][3];
    ipf_unpack(tri[refs[r]], v);
    const bool in_box = q[B] >= fminf(fminf(v[0][B], v[1][B]), v[2][B]) &&
                        q[B] <= fmaxf(fmaxf(v[0][B], v[1][B]), v[2][B]) &&
                        q[C] >= fminf(fminf(v[0][C], v[1][C]), v[2][C]) &&
                        q[C] <= fmaxf(fmaxf(v[0][C], v[1][C]), v[2][C]);
    if (!in_box) continue;
    double P[3][3];  // vertices relative to q: P[vertex][axis slot A, B, C]
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      P[i][0] = __dsub_rn((double)v[i][A], qa);
      P[i][1] = __dsub_rn((double)v[i][B], qb);
      P[i][2] = __dsub_rn((double)v[i][C], qc);
    }
    const double U = __dsub_rn(__dmul_rn(P[1][1], P[2][2]), __dmul_rn(P[1][2], P[2][1]));
    const double Vv = __dsub_rn(__dmul_rn(P[2][1], P[0][2]), __dmul_rn(P[2][2], P[0][1]));
    const double W = __dsub_rn(__dmul_rn(P[0][1], P[1][2]), __dmul_rn(P[0][2], P[1][1]));
    const int su = ipf_sign(U, ipf_tie(v[1][B], v[1][C], v[2][B], v[2][C]));
    const int sv = ipf_sign(Vv, ipf_tie(v[2][B], v[2][C], v[0][B], v[0][C]));
    const int sw = ipf_sign(W, ipf_tie(v[0][B], v[0][C], v[1][B], v[1][C]));
    if (su == 0 || su != sv || sv != sw) continue;
    const double Tn = __dadd_rn(__dadd_rn(__dmul_rn(U, P[0][0]), __dmul_rn(Vv, P[1][0])), __dmul_rn(W, P[2][0]));
    const int st = su * ((Tn > 0.0) - (Tn < 0.0));
    fwd += st >= 0;
    bwd += st <= 0;
  }
  return (uint32_t)(fwd & 1) | ((uint32_t)(bwd & 1) << 1);
}

// Ray parities in column order: the lanes of a wave mostly share one
// column and so read the same triangles.  par[a R + j] = the two bits.
__global__ __launch_bounds__(256) void k_ipf_rays(const float4* qbuf, int64_t R, const uint32_t* box,
                                                  const IpfGrid* grid, const uint32_t* start, const uint32_t* refs,
                                                  const IpfTri* tri, const uint32_t* order, const uint32_t* n_entries,
                                                  uint8_t* par) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)*n_entries) return;
  const uint32_t e = order[t];
  const int64_t j = e & 0x3fffffffu;
  const int a = (int)(e >> 30);
  const float4 p = qbuf[j];
  const int k = __float_as_int(p.w);
  const float q[3] = {p.x, p.y, p.z};
  const uint32_t col = ipf_column(q, box, k, a, grid[3 * k + a]);
  uint32_t bits;
  if (a == 0)
    bits = ipf_parity<0>(q, col, start, refs, tri);
  else if (a == 1)
    bits = ipf_parity<1>(q, col, start, refs, tri);
  else
    bits = ipf_parity<2>(q, col, start, refs, tri);
  par[a * R + j] = (uint8_t)bits;
}

// flag[j] = 1 when more than `threshold` of the six rays cross an odd number of times
__global__ __launch_bounds__(256) void k_ipf_flags(const float4* qbuf, int64_t R, const uint8_t* par,
                                                   double threshold, uint32_t* flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  if (__float_as_int(qbuf[j].w) < 0) {
    flag[j] = 0u;
    return;
  }
  const int votes = __popc((uint32_t)par[j]) + __popc((uint32_t)par[R + j]) + __popc((uint32_t)par[2 * R + j]);
  flag[j] = ((double)votes / 6.0 > threshold) ? 1u : 0u;
}

// offsets[k] = scanned flag at the first raw candidate of instance k
__global__ void k_ipf_offsets(const uint32_t* scan, const int64_t* ro, int K, uint32_t* offsets) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= K) offsets[k] = scan[ro[k]];
}

// Kept candidates, in raw order: out[3][M_in] (stride M_in), source[i] = j.
__global__ __launch_bounds__(256) void k_ipf_write(const float4* qbuf, int64_t R, const uint32_t* scan,
                                                   int64_t M_in, float* out, int64_t* source) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R) return;
  const uint32_t pos = scan[j];
  if (scan[j + 1] == pos) return;
  const float4 p = qbuf[j];
  out[pos] = p.x;
  out[M_in + pos] = p.y;
  out[2 * M_in + pos] = p.z;
  if (source) source[pos] = j;
}

}  // namespace fmpm
