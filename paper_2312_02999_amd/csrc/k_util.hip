// Scans, deterministic reductions and small vector kernels.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;
constexpr int RED_T = 256;
constexpr int RED_BLOCKS = 512;

int64_t nblocks(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

// Block-local exclusive scan; writes the block total to bsum[blockIdx].
__global__ void __launch_bounds__(SCAN_T) scan_block_kernel(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                            int64_t n, int32_t* __restrict__ bsum) {
  __shared__ int32_t sh[SCAN_T];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t idx = base + k;
    v[k] = idx < n ? in[idx] : 0;
    acc += v[k];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int32_t t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - acc;          // exclusive prefix of this thread
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t idx = base + k;
    if (idx < n) out[idx] = run;
    run += v[k];
  }
  if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = sh[SCAN_T - 1];
}

__global__ void scan_add_kernel(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ boff) {
  int64_t idx = static_cast<int64_t>(blockIdx.x) * SCAN_T * SCAN_ITEMS + threadIdx.x;
  int32_t add = boff[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    int64_t j = idx + k * SCAN_T;
    if (j < n) out[j] += add;
  }
}

__global__ void scan_total_kernel(const int32_t* __restrict__ in_last, const int32_t* __restrict__ out_last,
                                  int32_t* d_total) {
  *d_total = *in_last + *out_last;
}

size_t scan_temp_bytes(int64_t n) {
  size_t b = 0;
  int64_t m = n;
  while (true) {
    int64_t nb = nblocks(m);
    b += align256(sizeof(int32_t) * (nb + 1)) * 2;
    if (nb <= 1) break;
    m = nb;
  }
  return b + 256;
}

static void scan_rec(const int32_t* in, int32_t* out, int64_t n, char* temp, hipStream_t st) {
  int64_t nb = nblocks(n);
  int32_t* bsum = reinterpret_cast<int32_t*>(temp);
  int32_t* boff = reinterpret_cast<int32_t*>(temp + align256(sizeof(int32_t) * (nb + 1)));
  char* next = temp + 2 * align256(sizeof(int32_t) * (nb + 1));
  scan_block_kernel<<<static_cast<unsigned>(nb), SCAN_T, 0, st>>>(in, out, n, bsum);
  if (nb > 1) {
    scan_rec(bsum, boff, nb, next, st);
    scan_add_kernel<<<static_cast<unsigned>(nb), SCAN_T, 0, st>>>(out, n, boff);
  }
}

// The input may alias the output; the last input element is saved first so
// the total stays correct.
__global__ void copy_last_kernel(const int32_t* in, int64_t n, int32_t* dst) { *dst = in[n - 1]; }

void launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total, void* temp,
                           hipStream_t st) {
  if (n <= 0) {
    launch_fill_i32(d_total, 1, 0, st);
    return;
  }
  char* t = static_cast<char*>(temp);
  int32_t* last = reinterpret_cast<int32_t*>(t);
  copy_last_kernel<<<1, 1, 0, st>>>(in, n, last);
  scan_rec(in, out, n, t + 256, st);
  scan_total_kernel<<<1, 1, 0, st>>>(last, out + n - 1, d_total);
}

// ---- deterministic FP64 sums -------------------------------------------------
__device__ double block_sum(double v) {
  __shared__ double sh[RED_T / PDIPC_WAVE];
  v = wave_sum(v);
  int lane = threadIdx.x % PDIPC_WAVE, wid = threadIdx.x / PDIPC_WAVE;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < RED_T / PDIPC_WAVE; ++k) r += sh[k];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(RED_T) sum_partial_kernel(const double* __restrict__ a, int64_t na,
                                                            const double* __restrict__ b, int64_t nb,
                                                            double* __restrict__ part) {
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * RED_T;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * RED_T + threadIdx.x; i < na; i += stride) acc += a[i];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * RED_T + threadIdx.x; i < nb; i += stride) acc += b[i];
  double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(RED_T) sum_final_kernel(const double* __restrict__ part, int nparts,
                                                          double* __restrict__ out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += RED_T) acc += part[i];
  double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

size_t sum_temp_bytes(int64_t) { return sizeof(double) * RED_BLOCKS + 256; }

void launch_sum2(const double* a, int64_t na, const double* b, int64_t nb, double* d_out, void* temp,
                 hipStream_t st) {
  double* part = static_cast<double*>(temp);
  sum_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(a, na, b, nb, part);
  sum_final_kernel<<<1, RED_T, 0, st>>>(part, RED_BLOCKS, d_out);
}

void launch_sum(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  launch_sum2(in, n, nullptr, 0, d_out, temp, st);
}

// ---- order-free min / max -----------------------------------------------------
__global__ void __launch_bounds__(RED_T) minmax_partial_kernel(const double* __restrict__ in, int64_t n, int mode,
                                                               double* __restrict__ part) {
  __shared__ double sh[RED_T / PDIPC_WAVE];
  double acc = mode == 0 ? 1.0 : 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * RED_T;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * RED_T + threadIdx.x; i < n; i += stride)
    acc = mode == 0 ? fmin(acc, in[i]) : fmax(acc, fabs(in[i]));
  acc = mode == 0 ? wave_min(acc) : wave_max(acc);
  int lane = threadIdx.x % PDIPC_WAVE, wid = threadIdx.x / PDIPC_WAVE;
  if (lane == 0) sh[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int k = 1; k < RED_T / PDIPC_WAVE; ++k) r = mode == 0 ? fmin(r, sh[k]) : fmax(r, sh[k]);
    part[blockIdx.x] = r;
  }
}

__global__ void minmax_final_kernel(const double* __restrict__ part, int nparts, int mode, double* out) {
  if (threadIdx.x != 0) return;
  double r = mode == 0 ? 1.0 : 0.0;
  for (int i = 0; i < nparts; ++i) r = mode == 0 ? fmin(r, part[i]) : fmax(r, part[i]);
  *out = r;
}

void launch_min_clamp1(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  double* part = static_cast<double*>(temp);
  minmax_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(in, n, 0, part);
  minmax_final_kernel<<<1, 64, 0, st>>>(part, RED_BLOCKS, 0, d_out);
}

void launch_max_abs(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  double* part = static_cast<double*>(temp);
  minmax_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(in, n, 1, part);
  minmax_final_kernel<<<1, 64, 0, st>>>(part, RED_BLOCKS, 1, d_out);
}

// ---- fills and updates ------------------------------------------------------
__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void axpy_kernel(int64_t n, double alpha, const double* __restrict__ dx, double* __restrict__ x) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] + alpha * dx[i];
}

__global__ void count_nonfinite_kernel(const double* __restrict__ x, int64_t n, int32_t* __restrict__ out) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n && !isfinite(x[i])) atomicAdd(out, 1);
}
void launch_count_nonfinite(const double* x, int64_t n, int32_t* d_out, hipStream_t st) {
  launch_fill_i32(d_out, 1, 0, st);
  if (n > 0) count_nonfinite_kernel<<<grid_for(n, 256), 256, 0, st>>>(x, n, d_out);
}

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t st) {
  if (n > 0) fill_i32_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
}
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n > 0) fill_f64_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
}
void launch_axpy_positions(int64_t n3, double alpha, const double* dx, double* x, hipStream_t st) {
  if (n3 > 0) axpy_kernel<<<grid_for(n3, 256), 256, 0, st>>>(n3, alpha, dx, x);
}

}  // namespace pdipc
