// libmpm_probes.so: measurement probes for bench.py.  They time, on the
// device the process uses, the atomic operations the substep kernel is built
// on, so that its achieved atomic rates can be set against what the chip
// delivers in the same run:
//   * LDS 64-bit integer adds (ds_add_u64), the P2G tile's accumulation, in
//     two address patterns: lane-consecutive words (no bank conflicts) and
//     the tile pattern of the P2G scatter (lanes of one cell visit the 27
//     nodes of the cell's stencil in a per-lane rotated order; 4 channel
//     planes; the tile geometry of a 4^3-cell item grown by one cell);
//   * global FP32 adds, the tile flush into the grid, to lane-distinct
//     addresses and in the flush pattern (the 4 channels of a node).
// Each probe runs two workgroups of 256 threads per CU (the substep kernel's
// occupancy) and returns the elapsed time and the lane operations done.
// The LDS probe also runs with 32-bit integer and FP32 words (ds_add_u32,
// ds_add_f32), the alternatives to the 64-bit tile words.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 1331;  // nodes per channel plane, as the P2G tile

__device__ __forceinline__ int rot3(int s, int k) {
  const int r = k + s;
  return r >= 3 ? r - 3 : r;
}

// pattern 0: lane-consecutive words; pattern 1: the P2G scatter's node
// order.  Every address stays inside the 4 x 1331-word tile.  T is the
// word: unsigned long long (ds_add_u64), unsigned (ds_add_u32) or float
// (ds_add_f32).
template <typename T>
__global__ __launch_bounds__(kThreads, 2) void k_lds_add(int pattern, int reps, T* sink) {
  __shared__ T tile[4 * kTile];
  for (int t = threadIdx.x; t < 4 * kTile; t += kThreads) tile[t] = (T)0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // P2G geometry: box of 6^3 base cells -> 8^3 nodes, x stride 8*8+3
  constexpr int pz = 8, SX = 8 * 8 + 3;
  const int cell = lane / 24 + 3 * wave;  // about 24 particles per cell, cells along z then y
  const int cz = cell % 4, cy = (cell / 4) % 4, cx = 1 + (cell / 16);
  const int a1 = cx * SX + cy * pz + cz;  // base node of the cell's stencil (< 3*67+3*8+3+... < 1331)
  const int g = lane % 27;
  const int gs[3] = {g / 9, (g / 3) % 3, g % 3};
  const T v = (T)(1 + (threadIdx.x & 7));
  for (int it = 0; it < reps; ++it) {
#pragma unroll
    for (int kx = 0; kx < 3; ++kx)
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kz = 0; kz < 3; ++kz) {
          int t;
          if (pattern == 0) {
            t = (threadIdx.x + 256 * (kx * 9 + ky * 3 + kz)) % kTile;
          } else {
            t = a1 + rot3(gs[0], kx) * SX + rot3(gs[1], ky) * pz + rot3(gs[2], kz);
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) atomicAdd(&tile[c * kTile + t], v);
        }
  }
  __syncthreads();
  if (threadIdx.x == 0) sink[blockIdx.x] = tile[(blockIdx.x * 7) % (4 * kTile)];
}

// pattern 0: every lane its own float (stride 1); pattern 1: thread t adds
// to the 4 channels (x, y, z, m) of node t of a float4 grid, like the flush.
__global__ __launch_bounds__(kThreads) void k_global_add_f32(int pattern, int reps, float* grid, int64_t floats) {
  const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * kThreads;
  for (int it = 0; it < reps; ++it) {
    if (pattern == 0) {
      const int64_t a = (tid + it * nthreads) % floats;
      atomicAdd(grid + a, 1.0f);
    } else {
      const int64_t node = (tid + it * nthreads) % (floats / 4);
#pragma unroll
      for (int c = 0; c < 4; ++c) atomicAdd(grid + 4 * node + c, 1.0f);
    }
  }
}

int device_cus(int* cus) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -3;
  *cus = prop.multiProcessorCount;
  return 0;
}

template <typename T>
int lds_probe(int pattern, int reps, void* sink, float* ms, double* lane_ops) {
  if ((pattern != 0 && pattern != 1) || reps < 1 || !sink || !ms || !lane_ops) return -1;
  int cus = 0;
  if (device_cus(&cus)) return -3;
  const int blocks = 2 * cus;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
  k_lds_add<T><<<blocks, kThreads>>>(pattern, 1, (T*)sink);  // warm-up
  hipEventRecord(e0, nullptr);
  k_lds_add<T><<<blocks, kThreads>>>(pattern, reps, (T*)sink);
  hipEventRecord(e1, nullptr);
  const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *lane_ops = (double)blocks * kThreads * reps * 108.0;
  return ok && hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace

extern "C" {

// LDS adds: pattern 0 (lane-consecutive) or 1 (P2G tile pattern); reps
// rounds of 108 adds per thread.  *ms = kernel time, *lane_ops = adds.
// sink: device memory of at least 2 x (number of CUs) 64-bit words.
int probe_lds_add_u64(int pattern, int reps, void* sink, float* ms, double* lane_ops) {
  return lds_probe<unsigned long long>(pattern, reps, sink, ms, lane_ops);
}
int probe_lds_add_u32(int pattern, int reps, void* sink, float* ms, double* lane_ops) {
  return lds_probe<unsigned>(pattern, reps, sink, ms, lane_ops);
}
int probe_lds_add_f32(int pattern, int reps, void* sink, float* ms, double* lane_ops) {
  return lds_probe<float>(pattern, reps, sink, ms, lane_ops);
}

// Global FP32 adds into grid (device, `floats` floats, multiple of 4):
// pattern 0 (lane-distinct) or 1 (4 channels of a node per thread); reps
// rounds over blocks x 256 threads.
int probe_global_add_f32(int pattern, int reps, int blocks, float* grid, int64_t floats, float* ms, double* lane_ops) {
  if ((pattern != 0 && pattern != 1) || reps < 1 || blocks < 1 || !grid || floats < 4 || (floats & 3) || !ms ||
      !lane_ops)
    return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
  k_global_add_f32<<<blocks, kThreads>>>(pattern, 1, grid, floats);  // warm-up
  hipEventRecord(e0, nullptr);
  k_global_add_f32<<<blocks, kThreads>>>(pattern, reps, grid, floats);
  hipEventRecord(e1, nullptr);
  const bool ok = hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *lane_ops = (double)blocks * kThreads * reps * (pattern == 0 ? 1.0 : 4.0);
  return ok && hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
