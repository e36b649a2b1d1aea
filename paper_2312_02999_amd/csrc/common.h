// Shared device/host helpers for the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#define PDIPC_WAVE 64

namespace pdipc {

// ---- small fixed-size linear algebra (row-major 3x3) -----------------------
template <typename T>
struct M3 {
  T a[9];
  __host__ __device__ T& operator()(int r, int c) { return a[3 * r + c]; }
  __host__ __device__ T operator()(int r, int c) const { return a[3 * r + c]; }
};

template <typename T>
__device__ __forceinline__ T det3(const M3<T>& A) {
  return A(0, 0) * (A(1, 1) * A(2, 2) - A(1, 2) * A(2, 1)) - A(0, 1) * (A(1, 0) * A(2, 2) - A(1, 2) * A(2, 0)) +
         A(0, 2) * (A(1, 0) * A(2, 1) - A(1, 1) * A(2, 0));
}

template <typename T>
__device__ __forceinline__ M3<T> mul(const M3<T>& A, const M3<T>& B) {
  M3<T> C;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) C(r, c) = A(r, 0) * B(0, c) + A(r, 1) * B(1, c) + A(r, 2) * B(2, c);
  return C;
}

template <typename T>
__device__ __forceinline__ T dot3(const T* a, const T* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <typename T>
__device__ __forceinline__ void cross3(const T* a, const T* b, T* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// ---- wave-level reductions (64 lanes) ---------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, PDIPC_WAVE);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, PDIPC_WAVE);
  return v;
}
__device__ __forceinline__ int32_t wave_sum_i32(int32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, PDIPC_WAVE);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, PDIPC_WAVE));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, PDIPC_WAVE));
  return v;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) round-robin;
// this bijection of the block index gives each XCD one contiguous range of
// logical blocks, so neighbouring elements (which share vertices) meet in the
// same L2.
constexpr int PDIPC_XCDS = 8;
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t q = nb / PDIPC_XCDS, r = nb % PDIPC_XCDS, x = b % PDIPC_XCDS, j = b / PDIPC_XCDS;
  return x * q + (x < r ? x : r) + j;
}

// Number of set bits of a wave mask below the calling lane.
__device__ __forceinline__ int32_t lanes_below(uint64_t m) {
  return static_cast<int32_t>(
      __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u)));
}

// Minimum over a 256-thread block (wave butterflies, then the four waves).
// Every thread calls it; all hold the result.
__device__ __forceinline__ double block256_min(double v, double* sh4) {
  v = wave_min(v);
  if (threadIdx.x % PDIPC_WAVE == 0) sh4[threadIdx.x / PDIPC_WAVE] = v;
  __syncthreads();
  return fmin(fmin(sh4[0], sh4[1]), fmin(sh4[2], sh4[3]));
}

inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return static_cast<unsigned>(g < 1 ? 1 : g);
}

}  // namespace pdipc
