// The library's own device workspace, for callers that cannot allocate device memory
// (adafac_bind_static in include/adafac.h), and the fill kernel that clears a workspace.
//
// `scratch` is one file-scope device array per GPU, held from the code object's load until the
// process ends.  Host code never passes the array's name to a kernel or a copy: the name is a
// host-side stand-in, not a device address.  The device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and kept in g_base[device].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "adafac.h"
#include "adafac_internal.hpp"

namespace adafac {

int bind_workspace(adafac_ctx* c, void* ws, size_t bytes, void* stream, bool clear_by_kernel);
const char* ctx_workspace(const adafac_ctx* c);
void ctx_unbind(adafac_ctx* c, const char* why);
int ctx_fail(adafac_ctx* c, int code, const char* msg);

namespace {

constexpr size_t kStaticBytes = size_t(ADAFAC_STATIC_WORKSPACE_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticBytes];

std::mutex g_mu;
void* g_base[kMaxDevices] = {};          // device address of scratch, per device (nullptr: not taken yet)
adafac_ctx* g_owner[kMaxDevices] = {};   // context bound to the device's array, or nullptr

__global__ void __launch_bounds__(256) k_zero_fill(uint4* p, size_t n16, unsigned char* tail, size_t ntail) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

}  // namespace

hipError_t launch_zero_fill(void* p, size_t bytes, hipStream_t s) {
  if (!bytes) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 16) return hipErrorInvalidValue;
  const size_t n16 = bytes / 16;
  const size_t blocks = std::min<size_t>(4096, std::max<size_t>(1, (n16 + 255) / 256));
  hipLaunchKernelGGL(k_zero_fill, dim3(unsigned(blocks)), dim3(256), 0, s, static_cast<uint4*>(p), n16,
                     static_cast<unsigned char*>(p) + n16 * 16, bytes % 16);
  return hipGetLastError();
}

// A context that stops using the static array (destroyed, re-bound, regridded) gives it up.
void static_ws_forget(const adafac_ctx* c) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (int i = 0; i < kMaxDevices; ++i)
    if (g_owner[i] == c) g_owner[i] = nullptr;
}

}  // namespace adafac

using namespace adafac;

int adafac_bind_static(adafac_ctx* c, void* stream) {
  if (!c) return ADAFAC_EINVAL;
  size_t need = 0;
  int rc = adafac_workspace_bytes(c, &need);
  if (rc) return ctx_fail(c, rc, "build_operators first");
  if (need > kStaticBytes)
    return ctx_fail(c, ADAFAC_ENOMEM,
                    ("the hierarchy needs " + std::to_string(need) + " bytes of workspace, more than the " +
                     std::to_string(kStaticBytes) + " of the static workspace; use adafac_bind").c_str());
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = -1;
  if (hipStreamGetDevice(st, &dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return ctx_fail(c, ADAFAC_EDEVICE, "adafac_bind_static: cannot tell the stream's device");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_base[dev]) {
      int cur = -1;
      if (hipGetDevice(&cur) != hipSuccess) return ctx_fail(c, ADAFAC_EDEVICE, "adafac_bind_static: hipGetDevice");
      if (cur != dev && hipSetDevice(dev) != hipSuccess)
        return ctx_fail(c, ADAFAC_EDEVICE, "adafac_bind_static: hipSetDevice");
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (cur != dev) (void)hipSetDevice(cur);
      if (e != hipSuccess || !p)
        return ctx_fail(c, ADAFAC_EDEVICE,
                        (std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(e)).c_str());
      g_base[dev] = p;
    }
    base = g_base[dev];
    // the array holds one hierarchy: a context bound to it before loses its binding
    adafac_ctx* prev = g_owner[dev];
    if (prev && prev != c && ctx_workspace(prev) == static_cast<const char*>(base))
      ctx_unbind(prev, "the static workspace was taken by another context; bind again");
    g_owner[dev] = nullptr;
  }
  rc = bind_workspace(c, base, kStaticBytes, stream, true);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  g_owner[dev] = c;
  return ADAFAC_OK;
}
