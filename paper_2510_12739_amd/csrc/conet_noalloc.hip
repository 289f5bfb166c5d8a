// Allocation-free forward: the activation arena of a forward pass (residual-stream
// ping-pong buffers and the middle-activation buffers of every branch) lives in a
// file-scope device array instead of the model's workspace, so a caller that cannot
// allocate device memory (code under HIP graph capture, a serving loop that forbids
// hipMalloc) still gets a forward with only its inputs and outputs passed in.
//
// The array's host-side name is not a device address: its address on each device is
// taken once, with that device current, by hipGetSymbolAddress in noalloc_setup (called
// from conet_create), and only that address is handed to kernels. Every call on one
// device shares that device's array, so calls that overlap on one device race; nothing
// in the array needs to start at zero (every buffer is written before it is read).
#include <hip/hip_runtime.h>

#include <mutex>

#include "conet_model.h"

namespace conet {

constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) uint8_t scratch[CONET_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static uint8_t* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// Record the scratch array's address on `device` (the current device). Idempotent.
conet_status noalloc_setup(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(CONET_EDEVICE, "device %d out of range", device);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return CONET_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!p || ((uintptr_t)p & 255) != 0) return fail(CONET_EDEVICE, "scratch array address %p is not 256-byte aligned", p);
  g_noalloc_ptr[device] = static_cast<uint8_t*>(p);
  return CONET_OK;
}

// Largest B*T*F whose activation arena fits the scratch array for configuration c.
static int64_t noalloc_capacity(const conet_config& c) {
  int64_t lo = 0, hi = (int64_t)1 << 31;
  while (lo < hi) {  // arena_bytes grows monotonically with the RE count
    const int64_t mid = lo + (hi - lo + 1) / 2;
    if (arena_bytes(c, mid) <= (size_t)CONET_NOALLOC_SCRATCH_BYTES) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace conet

using namespace conet;

extern "C" int64_t conet_forward_noalloc_capacity(const conet_model* M) {
  return M ? noalloc_capacity(M->cfg) : 0;
}

extern "C" conet_status conet_forward_noalloc(conet_model* M, const float* x, int32_t B, int32_t T, int32_t F,
                                              float* llr, void* stream) {
  if (!M) return fail(CONET_EINVAL, "null model");
  if (B == 0) return CONET_OK;
  if (!x || !llr) return fail(CONET_EINVAL, "null tensor pointer");
  if (B < 0 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad shape B=%d T=%d F=%d (need T in 1..14)", B, T, F);
  const int64_t cap = noalloc_capacity(M->cfg);
  const int64_t n_re = (int64_t)B * T * F;
  if (n_re > cap)
    return fail(CONET_ESHAPE, "B*T*F = %lld exceeds the %lld REs the %llu-byte static scratch holds for this model",
                (long long)n_re, (long long)cap, (unsigned long long)CONET_NOALLOC_SCRATCH_BYTES);
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales (set or calibrate)");
  if (M->cfg.train && M->cfg.norm == CONET_NORM_BN)
    return fail(CONET_EINVAL, "a BatchNorm model in training keeps its batch statistics in the model's workspace");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != M->device) return fail(CONET_EDEVICE, "current device %d is not the model's device %d", dev, M->device);
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    base = (dev >= 0 && dev < NOALLOC_MAX_DEVICES) ? g_noalloc_ptr[dev] : nullptr;
  }
  if (!base) return fail(CONET_ESTATE, "static scratch of device %d was not set up (conet_create does it)", dev);
  Arena ar;
  arena_carve(M->cfg, n_re, base, ar);
  Geometry geo;
  geo.uniform = true; geo.B = B; geo.T = T; geo.F = F;
  return run_forward(M, ar, x, geo, llr, (hipStream_t)stream, nullptr);
}
