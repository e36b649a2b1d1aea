// Dense SPD factor / solve / inverse on caller data without any allocation.
//
// The same kernels as the reduced contact system of Eq. (11) (blocked
// Cholesky with L^-1 along the factorisation, two triangular products per
// solve, Y^T Y for the inverse), with every work buffer carved out of one
// file-scope device array instead of device memory allocated per call.  This
// is for callers that cannot allocate device memory (code under HIP graph
// capture, serving loops that must not call the allocator).
//
// The array exists once per device for the lifetime of the process; the host
// never uses its name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.  All
// calls on one device share the array, so calls that overlap on one device
// (different streams, or different host threads) race.
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "pdipc.h"

namespace pdipc {

namespace {

// Largest system: 1024 unknowns (the reduced system of 341 contact vertices).
// The 32-wide blocked path (n <= 2048) keeps L^-1 and its transpose, so the
// inverse needs no work matrix beyond the auxiliary buffer.
constexpr int64_t kMaxN = 1024;
constexpr int32_t kMaxRhs = 4;
static_assert(kMaxN <= 2048, "the layout below assumes the 32-wide blocked factorisation");

constexpr size_t align256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

// Byte offsets of the work buffers for element type T (size e) and order n:
// W (factorisation workspace, n^2), F (L^-1, n^2), aux (dense_aux_size(n));
// the FP32 path also stages the right-hand sides (n x kMaxRhs) and the
// inverse (n^2) before widening them into the caller's FP64 arrays.
struct Layout {
  size_t W, F, aux, rhs, inv, end;
};
constexpr Layout layout(size_t e, int64_t n, bool staged) {
  Layout L{};
  size_t o = 0;
  L.W = o; o += align256(e * n * n);
  L.F = o; o += align256(e * n * n);
  L.aux = o; o += align256(e * dense_aux_size(n));
  L.rhs = o; o += staged ? align256(e * n * kMaxRhs) : 0;
  L.inv = o; o += staged ? align256(e * n * n) : 0;
  L.end = o;
  return L;
}
constexpr size_t kScratchBytes = layout(sizeof(double), kMaxN, false).end;
static_assert(layout(sizeof(float), kMaxN, true).end <= kScratchBytes, "the FP32 layout must fit the array");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

// The scratch array: never addressed by its name on the host.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of this device's copy of the array (looked up once per
// device, with the device current).
static hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace pdipc

using namespace pdipc;

extern "C" int32_t pdipc_dense_spd_noalloc(const double* A, int64_t n, double* b, int32_t nrhs, double* Ainv,
                                           int32_t precision, int32_t* info, void* stream) {
  if (!A || !info || n <= 0 || nrhs < 0 || nrhs > kMaxRhs || (nrhs > 0 && !b) ||
      (precision != PDIPC_FP64 && precision != PDIPC_MIXED_FP32)) {
    set_last_error("pdipc_dense_spd_noalloc: invalid argument");
    return PDIPC_E_INVALID;
  }
  if (n > kMaxN) {
    set_last_error("pdipc_dense_spd_noalloc: n exceeds the maximum order of 1024");
    return PDIPC_E_INVALID;
  }
  void* base = nullptr;
  if (scratch_address(&base) != hipSuccess) {
    set_last_error("pdipc_dense_spd_noalloc: device address of the scratch array not available");
    return PDIPC_E_HIP;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned char* s = static_cast<unsigned char*>(base);
  const int64_t nn = n * n;
  const bool solve = b && nrhs > 0;
  if (precision == PDIPC_FP64) {
    const Layout L = layout(sizeof(double), n, false);
    double* W = reinterpret_cast<double*>(s + L.W);
    double* F = reinterpret_cast<double*>(s + L.F);
    double* aux = reinterpret_cast<double*>(s + L.aux);
    if (hipMemcpyAsync(W, A, sizeof(double) * nn, hipMemcpyDeviceToDevice, st) != hipSuccess) {
      set_last_error("pdipc_dense_spd_noalloc: copy of A failed");
      return PDIPC_E_HIP;
    }
    dense_cholesky<double>(W, n, F, aux, info, st);
    if (solve) dense_chol_solve<double>(F, aux, n, b, nrhs, st);
    if (Ainv) dense_chol_inverse<double>(F, aux, n, Ainv, nullptr, st);
  } else {
    const Layout L = layout(sizeof(float), n, true);
    float* W = reinterpret_cast<float*>(s + L.W);
    float* F = reinterpret_cast<float*>(s + L.F);
    float* aux = reinterpret_cast<float*>(s + L.aux);
    float* rhs = reinterpret_cast<float*>(s + L.rhs);
    float* inv = reinterpret_cast<float*>(s + L.inv);
    launch_convert_f64_f32(A, W, nn, st);
    dense_cholesky<float>(W, n, F, aux, info, st);
    if (solve) {
      launch_convert_f64_f32(b, rhs, n * nrhs, st);
      dense_chol_solve<float>(F, aux, n, rhs, nrhs, st);
      launch_convert_f32_f64(rhs, b, n * nrhs, st);
    }
    if (Ainv) {
      dense_chol_inverse<float>(F, aux, n, inv, nullptr, st);
      launch_convert_f32_f64(inv, Ainv, nn, st);
    }
  }
  if (hipGetLastError() != hipSuccess) {
    set_last_error("pdipc_dense_spd_noalloc: kernel launch failed");
    return PDIPC_E_HIP;
  }
  return PDIPC_OK;
}
