// Energy-adaptive gradient G = Psi - X (Psi^* X)^-1 (the same operation as
// eahp_ea_gradient) without any device allocation, for callers that cannot
// allocate: every intermediate (the p x p products Psi^* X and their
// inverses, the split-K partial tiles of the Gram product, the Gauss-Jordan
// work array and the pivot flags) lives in one file-scope device array of
// fixed size.  Each device holds its own copy of the array; its device
// address is looked up once per device when a context is created on it.
#include <mutex>

#include "ops.h"

using namespace eahp;

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

namespace eahp {

// Device address of this device's copy of the scratch array (the host-side
// name of the array is not a device address), looked up with the device
// current; called by eahp_ctx_create.
void noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) fail(EAHP_EINVAL, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) fail(EAHP_EDEVICE, std::string("hipGetSymbolAddress of the scratch array failed: ") +
                                                    hipGetErrorString(e));
  g_ptr[device] = p;
}

}  // namespace eahp

extern "C" size_t eahp_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int eahp_ea_gradient_noalloc(eahp_problem* pb, const void* Psi, const void* X, void* G) {
  try {
    if (!pb || !Psi || !X || !G) fail(EAHP_EINVAL, "null argument");
    const int dev = pb->ctx->device;
    HIPCK(hipSetDevice(dev));
    void* base = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      base = (dev >= 0 && dev < kMaxDevices) ? g_ptr[dev] : nullptr;
    }
    if (!base) fail(EAHP_EDEVICE, "no-allocation scratch not set up on this device (create a context on it first)");
    const int p = pb->p, nk = pb->nk;
    const int64_t pp = (int64_t)p * p;
    AutotuneHold hold;  // the products take kept launch shapes, never tuned here
    if (p > 1024) fail(EAHP_EINVAL, "p > 1024");
    if (nk > 1024) fail(EAHP_EINVAL, "more than 1024 k-points");
    // layout: M (nk p^2), the Gauss-Jordan work (2 p^2 per k-point, p > 128),
    // the pivot flags (nk ints), then the partial tiles of the Gram product
    const size_t bM = up256(sizeof(z64) * nk * pp);
    const size_t bW = p > 128 ? up256(sizeof(z64) * 2 * nk * pp) : 0;
    const size_t bI = up256(sizeof(int) * nk);
    const size_t fixed = bM + bW + bI;
    const size_t need_part = sizeof(z64) * gemm_hn_min_part(p, p, 1);
    if (fixed + need_part > kScratchBytes)
      fail(EAHP_EINVAL, "ea_gradient_noalloc: needs " + std::to_string(fixed + need_part) +
                            " bytes of scratch (nk p^2 products), more than the " + std::to_string(kScratchBytes) +
                            " bytes available");
    char* s = static_cast<char*>(base);
    z64* M = reinterpret_cast<z64*>(s);
    z64* Wk = reinterpret_cast<z64*>(s + bM);
    int* info = reinterpret_cast<int*>(s + bM + bW);
    z64* part = reinterpret_cast<z64*>(s + fixed);
    const size_t part_elems = (kScratchBytes - fixed) / sizeof(z64);
    hipStream_t st = pb->ctx->stream;
    const z64* Phi = static_cast<const z64*>(Psi);
    const z64* Xf = static_cast<const z64*>(X);
    z64* Gf = static_cast<z64*>(G);
    for (int ik = 0; ik < nk; ++ik) {
      const auto& K = pb->kp[ik];
      const int64_t o = (int64_t)p * K.off;
      gemm_hn_mfma_ws<double>(st, K.npw, p, p, Phi + o, K.npw, Xf + o, K.npw, M + ik * pp, p, 1.0, 0.0, part,
                              part_elems, 1, 0, 0, 0);
    }
    inverse(st, p, M, p, pp, Wk, nk, info);
    for (int ik = 0; ik < nk; ++ik) {
      const auto& K = pb->kp[ik];
      const int64_t o = (int64_t)p * K.off;
      axpby<double>(st, K.npw * p, 1.0, Phi + o, 0.0, Gf + o);
      gemm_nn<double>(st, K.npw, p, p, Xf + o, K.npw, M + ik * pp, p, 0, Gf + o, K.npw, -1.0, 0.0, 1.0);
    }
    HIPCK(hipMemcpyAsync(pb->h_info, info, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
    HIPCK(hipStreamSynchronize(st));
    for (int ik = 0; ik < nk; ++ik)
      if (pb->h_info[ik]) fail(EAHP_EFOM, "Phi^H X is singular in the energy-adaptive gradient");
    return EAHP_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (...) {
    g_last_error = "unknown error";
    return EAHP_EDEVICE;
  }
}
