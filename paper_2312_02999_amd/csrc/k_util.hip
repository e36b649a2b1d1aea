// Scans, deterministic reductions and small vector kernels.
#include "common.h"
#include "kernels.h"

namespace pdipc {

namespace {
constexpr int SCAN_T = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_T * SCAN_ITEMS;
constexpr int RED_T = 256;
constexpr int RED_BLOCKS = 512;

int64_t nblocks(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE; }
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

// Exclusive scans in two launches: per-tile sums, then every tile adds the
// sums of the tiles before it (read from the small bsum array) to its local
// scan.  Up to two independent arrays share the launches (their tiles follow
// each other in the grid).  The last tile of an array writes its total; a
// tile may also copy its output to a second array and hand over the scanned
// value at one index.  The input may alias the output: each tile reads its
// inputs into registers before writing.
__device__ __forceinline__ int scan_job_index(const ScanJobs& js, int64_t b) { return b < js.nb0 ? 0 : 1; }

__global__ void __launch_bounds__(SCAN_T) scan_reduce_kernel(ScanJobs js, int32_t* __restrict__ bsum) {
  __shared__ int32_t sh[SCAN_T / PDIPC_WAVE];
  const int w = scan_job_index(js, blockIdx.x);
  const ScanJob& J = js.j[w];
  const int64_t tile = w ? blockIdx.x - js.nb0 : blockIdx.x;
  const int64_t base = tile * SCAN_TILE;
  int32_t acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t idx = base + k * SCAN_T + threadIdx.x;
    acc += idx < J.n ? J.in[idx] : 0;
  }
  acc = wave_sum_i32(acc);
  if (threadIdx.x % PDIPC_WAVE == 0) sh[threadIdx.x / PDIPC_WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int v = 0; v < SCAN_T / PDIPC_WAVE; ++v) t += sh[v];
    bsum[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(SCAN_T) scan_apply_kernel(ScanJobs js, const int32_t* __restrict__ bsum) {
  __shared__ int32_t sh[SCAN_T];
  __shared__ int32_t wsum[SCAN_T / PDIPC_WAVE];
  const int w = scan_job_index(js, blockIdx.x);
  const ScanJob& J = js.j[w];
  const int64_t first = w ? js.nb0 : 0;
  const int64_t tile = blockIdx.x - first;
  const int64_t ntiles = (J.n + SCAN_TILE - 1) / SCAN_TILE;
  // offset of this tile: sum of the tile sums before it (same array)
  int32_t off = 0;
  for (int64_t b = first + threadIdx.x; b < static_cast<int64_t>(blockIdx.x); b += SCAN_T) off += bsum[b];
  off = wave_sum_i32(off);
  if (threadIdx.x % PDIPC_WAVE == 0) wsum[threadIdx.x / PDIPC_WAVE] = off;
  const int64_t base = tile * SCAN_TILE + static_cast<int64_t>(threadIdx.x) * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t idx = base + k;
    v[k] = idx < J.n ? J.in[idx] : 0;
    acc += v[k];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  int32_t tile_off = 0;
  for (int q = 0; q < SCAN_T / PDIPC_WAVE; ++q) tile_off += wsum[q];
  for (int o = 1; o < SCAN_T; o <<= 1) {
    const int32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = tile_off + sh[threadIdx.x] - acc;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t idx = base + k;
    if (idx < J.n) {
      J.out[idx] = run;
      if (J.copy) J.copy[idx] = run;
      if (idx == J.pick && J.pick_out) *J.pick_out = run;
    }
    run += v[k];
  }
  if (tile == ntiles - 1 && threadIdx.x == SCAN_T - 1) *J.d_total = tile_off + sh[SCAN_T - 1];
}

size_t scan_temp_bytes(int64_t n) { return align256(sizeof(int32_t) * (2 * nblocks(n) + 2)) + 256; }

void launch_exclusive_scans(const ScanJob* jobs, int njobs, void* temp, hipStream_t st) {
  ScanJobs js{};
  int64_t nbt = 0;
  int k = 0;
  for (int q = 0; q < njobs; ++q) {
    if (jobs[q].n <= 0) {
      launch_fill_i32(jobs[q].d_total, 1, 0, st);
      continue;
    }
    js.j[k] = jobs[q];
    if (k == 0) js.nb0 = nblocks(jobs[q].n);
    nbt += nblocks(jobs[q].n);
    ++k;
  }
  if (k == 0) return;
  if (k == 1) js.j[1] = js.j[0];
  int32_t* bsum = static_cast<int32_t*>(temp);
  scan_reduce_kernel<<<static_cast<unsigned>(nbt), SCAN_T, 0, st>>>(js, bsum);
  scan_apply_kernel<<<static_cast<unsigned>(nbt), SCAN_T, 0, st>>>(js, bsum);
}

void launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* d_total, void* temp,
                           hipStream_t st) {
  ScanJob j{in, out, n, d_total, nullptr, -1, nullptr};
  launch_exclusive_scans(&j, 1, temp, st);
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
                                                            const double* __restrict__ ls,
                                                            double* __restrict__ part) {
  if (ls && ls[LS_STATE] != 0.0) return;
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * RED_T;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * RED_T + threadIdx.x; i < na; i += stride) acc += a[i];
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * RED_T + threadIdx.x; i < nb; i += stride) acc += b[i];
  double s = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(RED_T) sum_final_kernel(const double* __restrict__ part, int nparts,
                                                          const double* __restrict__ ls, double* __restrict__ out) {
  if (ls && ls[LS_STATE] != 0.0) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += RED_T) acc += part[i];
  double s = block_sum(acc);
  if (threadIdx.x == 0) *out = s;
}

size_t sum_temp_bytes(int64_t) { return sizeof(double) * RED_BLOCKS + 256; }

void launch_sum2(const double* a, int64_t na, const double* b, int64_t nb, double* d_out, void* temp,
                 hipStream_t st, const double* ls) {
  double* part = static_cast<double*>(temp);
  sum_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(a, na, b, nb, ls, part);
  sum_final_kernel<<<1, RED_T, 0, st>>>(part, RED_BLOCKS, ls, d_out);
}

void launch_sum(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  launch_sum2(in, n, nullptr, 0, d_out, temp, st, nullptr);
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

// one wave: strided loads, then a wave reduction (min and max are order-free)
__global__ void __launch_bounds__(PDIPC_WAVE) minmax_final_kernel(const double* __restrict__ part, int nparts,
                                                                  int mode, double* out) {
  double r = mode == 0 ? 1.0 : 0.0;
  for (int i = threadIdx.x; i < nparts; i += PDIPC_WAVE) r = mode == 0 ? fmin(r, part[i]) : fmax(r, part[i]);
  r = mode == 0 ? wave_min(r) : wave_max(r);
  if (threadIdx.x == 0) *out = r;
}

void launch_min_clamp1(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  double* part = static_cast<double*>(temp);
  minmax_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(in, n, 0, part);
  minmax_final_kernel<<<1, PDIPC_WAVE, 0, st>>>(part, RED_BLOCKS, 0, d_out);
}

void launch_max_abs(const double* in, int64_t n, double* d_out, void* temp, hipStream_t st) {
  double* part = static_cast<double*>(temp);
  minmax_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(in, n, 1, part);
  minmax_final_kernel<<<1, PDIPC_WAVE, 0, st>>>(part, RED_BLOCKS, 1, d_out);
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

// ---- device line-search state (Section 2.2 back-tracking; see kernels.h) ---------
// alpha_m = min(1, minimum over the CCD blocks' minima); one wave
__global__ void __launch_bounds__(PDIPC_WAVE) ls_init_kernel(double* ls, const double* __restrict__ part, int nparts) {
  double a = 1.0;
  for (int i = threadIdx.x; i < nparts; i += PDIPC_WAVE) a = fmin(a, part[i]);
  a = wave_min(a);
  if (threadIdx.x != 0) return;
  ls[LS_ALPHA] = a;
  ls[LS_STATE] = 0.0;
  ls[LS_HALVINGS] = 0.0;
  ls[LS_ALPHA_M] = a;
}
__global__ void axpy_ls_kernel(int64_t n, const double* __restrict__ ls, const double* __restrict__ dx,
                               double* __restrict__ x) {
  if (ls[LS_STATE] != 1.0) return;
  const double alpha = ls[LS_ALPHA];
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = x[i] + alpha * dx[i];
}
void launch_ls_init(double* ls, const double* part, int nparts, hipStream_t st) {
  ls_init_kernel<<<1, PDIPC_WAVE, 0, st>>>(ls, part, nparts);
}
// dE of a trial: the second stage of launch_sum2 (the same partials and the
// same block reduction as sum_final_kernel), then the decision: accept when
// dE <= 0; otherwise halve alpha, and give up (state -1) after max_halvings
// halvings.
__global__ void __launch_bounds__(RED_T) ls_final_decide_kernel(double* ls, const double* __restrict__ part,
                                                                int nparts, int32_t max_halvings) {
  if (ls[LS_STATE] != 0.0) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += RED_T) acc += part[i];
  const double dE = block_sum(acc);
  if (threadIdx.x != 0) return;
  ls[LS_DE] = dE;
  if (dE <= 0.0) {
    ls[LS_STATE] = 1.0;
  } else if (ls[LS_HALVINGS] >= max_halvings) {
    ls[LS_STATE] = -1.0;
  } else {
    ls[LS_HALVINGS] += 1.0;
    ls[LS_ALPHA] *= 0.5;
  }
}
void launch_sum2_decide(const double* a, int64_t na, const double* b, int64_t nb, double* ls, void* temp,
                        int32_t max_halvings, hipStream_t st) {
  double* part = static_cast<double*>(temp);
  sum_partial_kernel<<<RED_BLOCKS, RED_T, 0, st>>>(a, na, b, nb, ls, part);
  ls_final_decide_kernel<<<1, RED_T, 0, st>>>(ls, part, RED_BLOCKS, max_halvings);
}
void launch_axpy_ls(int64_t n3, const double* ls, const double* dx, double* x, hipStream_t st) {
  if (n3 > 0) axpy_ls_kernel<<<grid_for(n3, 256), 256, 0, st>>>(n3, ls, dx, x);
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
__global__ void fill2_i32_kernel(int32_t* a, int64_t na, int32_t* b, int64_t nb, int32_t v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < na) a[i] = v;
  else if (i < na + nb) b[i - na] = v;
}
void launch_fill2_i32(int32_t* a, int64_t na, int32_t* b, int64_t nb, int32_t v, hipStream_t st) {
  if (na + nb > 0) fill2_i32_kernel<<<grid_for(na + nb, 256), 256, 0, st>>>(a, na, b, nb, v);
}
void launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n > 0) fill_f64_kernel<<<grid_for(n, 256), 256, 0, st>>>(p, n, v);
}
void launch_axpy_positions(int64_t n3, double alpha, const double* dx, double* x, hipStream_t st) {
  if (n3 > 0) axpy_kernel<<<grid_for(n3, 256), 256, 0, st>>>(n3, alpha, dx, x);
}

}  // namespace pdipc
