// qrk_solve_banded_noalloc: the banded step (Givens QR of [J; sqrt(lambda) D], back-substitution
// and float64-residual sweeps) for callers that cannot allocate device memory.  Every buffer the
// banded path needs beyond the caller's inputs and outputs is carved from one fixed device array,
// `scratch`, of kScratchBytes per GPU; nothing is allocated per call.
//
// The array is a file-scope __device__ variable: each GPU that the library runs on holds its own
// copy at its own address until the process ends.  Its device address is taken once per device
// with hipGetSymbolAddress (the array's name in host code is only a host-side stand-in) and kept
// in g_scratch[dev]; kernels are given carved pointers into that address only.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "qrk_banded.hpp"
#include "qrk_device.hpp"
#include "qrk_host.hpp"
#include "qrkit.h"

using namespace qrk;

namespace {

constexpr size_t kScratchBytes = (size_t)QRK_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {nullptr};
bool g_gfx950[kMaxDevices] = {false};

// Device address of this device's scratch array (looked up once per device), or an error.
qrk_status scratch_for_current_device(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return QRK_EHIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return QRK_EHIP;
    g_gfx950[dev] = std::string(prop.gcnArchName).rfind("gfx950", 0) == 0;
    if (!g_gfx950[dev]) return QRK_ENODEVICE;
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return QRK_EHIP;
    g_scratch[dev] = ptr;
  }
  *out = static_cast<unsigned char*>(g_scratch[dev]);
  return QRK_OK;
}

__global__ void k_zero_words(uint32_t* __restrict__ a, int64_t na, uint32_t* __restrict__ b, int64_t nb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < na) a[i] = 0u;
  if (i < nb) b[i] = 0u;
}

__global__ void k_copy_status(const int* __restrict__ src, int32_t* __restrict__ dst) {
  if (threadIdx.x == 0) *dst = *src;
}

// Bump allocator over the scratch array: 256-byte aligned pieces.
struct Carve {
  size_t used = 0;
  size_t take(size_t bytes) {
    const size_t off = used;
    used += (bytes + 255) & ~(size_t)255;
    return off;
  }
};

struct Layout {
  size_t R, c, inv, fr, r, g, lam, status, r16;
  size_t total;
  bool keep16;
};

Layout layout(int64_t P, int64_t M, int64_t N, int w, size_t es) {
  Layout L{};
  Carve cv;
  const size_t PN = (size_t)(P * N), PM = (size_t)(P * (M > 0 ? M : 1));
  L.R = cv.take(es * PN * (size_t)w);
  L.c = cv.take(es * PN);
  L.inv = cv.take(sizeof(double) * PN);
  L.fr = cv.take(sizeof(int32_t) * (size_t)(P * (N + 1)));
  L.r = cv.take(sizeof(double) * PM);
  L.g = cv.take(sizeof(double) * PN);
  L.lam = cv.take(sizeof(double) * (size_t)P);
  L.status = cv.take(sizeof(int) * 4);
  L.keep16 = bsweep_w_fits(P, N, w, es);
  L.r16 = L.keep16 ? cv.take(es * 16 * (PN + 2 * (size_t)kBandPad)) : 0;
  L.total = cv.used;
  return L;
}

}  // namespace

extern "C" {

qrk_status qrk_solve_banded_noalloc(int32_t P, int64_t M, int64_t N, int32_t w, qrk_dtype dtype,
                                    const int32_t* row_start, const void* vals, const void* b, const double* d,
                                    double lambda, double* p, int32_t sweeps, int32_t* status_dev, void* stream) {
  // the argument checks of qrk_create_banded_batched, qrk_factor_banded and qrk_solve
  if (P < 1 || M < 0 || N < 1 || w < 1 || w > QRK_MAX_BAND || w > N) return QRK_EINVAL;
  if (dtype != QRK_F32 && dtype != QRK_F64) return QRK_EINVAL;
  if ((M > 0 && (!row_start || !vals || !b)) || !d || !p) return QRK_EINVAL;
  if (!(lambda >= 0.0) || !std::isfinite(lambda)) return QRK_EINVAL;
  if (sweeps < 0 || sweeps > 8) return QRK_EINVAL;
  if (P > (int64_t)1 << 24 || N > (int64_t)1 << 30 || M > (int64_t)1 << 30) return QRK_ETOOLARGE;
  const size_t es = dtype == QRK_F32 ? 4 : 8;
  const Layout L = layout(P, M, N, w, es);
  if (L.total > kScratchBytes) return QRK_ETOOLARGE;
  unsigned char* base = nullptr;
  qrk_status s = scratch_for_current_device(&base);
  if (s != QRK_OK) return s;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);

  // a handle on the host stack whose workspace pointers are pieces of the scratch array; the
  // banded factor and solve below are the handle path's own functions
  qrk_handle_s h;
  h.kind = KIND_BANDED;
  h.dtype = dtype;
  h.P = P;
  h.M = M;
  h.N = N;
  h.w = w;
  h.bandR = base + L.R;
  h.bandc = base + L.c;
  h.bandinv = reinterpret_cast<double*>(base + L.inv);
  h.bandfr = reinterpret_cast<int32_t*>(base + L.fr);
  h.rbuf = reinterpret_cast<double*>(base + L.r);
  h.gbuf = reinterpret_cast<double*>(base + L.g);
  h.lam_d = reinterpret_cast<double*>(base + L.lam);
  h.status = reinterpret_cast<int*>(base + L.status);
  h.bandR16 = L.keep16 ? base + L.r16 + es * 16 * kBandPad : nullptr;
  h.row_start = row_start;
  h.A = vals;
  h.b = b;
  h.d = d;
  h.lam = lambda;
  h.lam_ptr = h.lam_d;
  h.factored = true;

  // the sweep copy's padding rows must read as zero; an earlier, larger call on this device may
  // have left band values there (the status word is cleared by the factor itself)
  if (L.keep16) {
    const int64_t pad_words = (int64_t)(es * 16 * kBandPad / 4);
    uint32_t* pad0 = reinterpret_cast<uint32_t*>(base + L.r16);
    uint32_t* pad1 = reinterpret_cast<uint32_t*>(base + L.r16 + es * 16 * ((size_t)(P * N) + kBandPad));
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((pad_words + 255) / 256)), dim3(256), 0, st, pad0, pad_words,
                       pad1, pad_words);
    if (hipGetLastError() != hipSuccess) return QRK_EHIP;
  }
  if (launch_fill_double(h.lam_d, P, lambda, st) != hipSuccess) return QRK_EHIP;
  if ((s = banded_factor(&h, st)) != QRK_OK) return s;
  if ((s = banded_solve(&h, p, sweeps, st)) != QRK_OK) return s;
  if (status_dev) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, h.status, status_dev);
    if (hipGetLastError() != hipSuccess) return QRK_EHIP;
  }
  return QRK_OK;
}

}  // extern "C"
