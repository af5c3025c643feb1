// hist_u8_noalloc: the single-buffer histogram for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops that forbid hipMalloc).  It runs the same
// counting kernel as hist_u8; only the launch's scratch differs.  hist_u8 keeps a scratch
// block per HIP stream, allocated on first use; here it is one fixed array per device,
// compiled into the library, whose device address is looked up once per device.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "histmi.h"
#include "histmi_dev.h"
#include "runtime.h"

namespace histmi {
namespace {

// Layout of the array, in 32-bit words:
//   [0, 64)      tile counter block (Params::ctr)
//   [64, 128)    per-segment tickets (Params::seg_done; a single launch uses word 64)
//   [128, 192)   diagnostics counters of these launches (Params::diag; cumulative)
//   [256, ...)   partial copies of the histogram, kNoallocCopies x 256 words
constexpr uint32_t kCtrWord = 0;
constexpr uint32_t kSegDoneWord = 64;
constexpr uint32_t kDiagWord = 128;
constexpr uint32_t kPartialWord = 256;
constexpr uint32_t kNoallocWords = HIST_NOALLOC_SCRATCH_BYTES / 4;
constexpr uint32_t kNoallocCopies = (kNoallocWords - kPartialWord) / 256;
static_assert(kNoallocCopies >= 16, "room for the partial copies of a single launch");

// Every device the library runs on holds its own instance of this array until the process
// ends.  In host code `scratch` names a host-side stand-in: device work is only ever handed
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint32_t scratch[kNoallocWords];

constexpr int kMaxDevices = 64;
struct NoallocDev {
  uint32_t *ptr = nullptr;   // this device's `scratch`
  int cus = 0;
};
std::mutex g_noalloc_mu;
NoallocDev g_noalloc[kMaxDevices];

// Zero the words a launch needs zero at its start: counters, tickets and `copies` partial
// copies.  A kernel rather than hipMemsetAsync, so that a captured graph holds kernel nodes only.
__global__ void __launch_bounds__(kBlock) clear_scratch_kernel(uint32_t *s, uint32_t copies) {
  const uint32_t t = threadIdx.x;
  if (t < kDiagWord) s[kCtrWord + t] = 0u;
  for (uint32_t i = t; i < copies * 256u; i += kBlock) s[kPartialWord + i] = 0u;
}

// Set-up on the current device, once: the array's device address and the CU count.
hist_status_t noalloc_dev(NoallocDev **out) {
  int dev = 0;
  TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HIST_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  NoallocDev &nd = g_noalloc[dev];
  if (!nd.ptr) {
    hipDeviceProp_t pr;
    TRY_HIP(hipGetDeviceProperties(&pr, dev));
    if (std::strncmp(pr.gcnArchName, "gfx950", 6) != 0) return HIST_ENOTSUP;
    const size_t lds_cu = pr.maxSharedMemoryPerMultiProcessor ? pr.maxSharedMemoryPerMultiProcessor
                                                              : pr.sharedMemPerBlock;
    if (set_kernel_attrs((uint32_t)(lds_cu - rt::kStaticLdsReserve)) != hipSuccess) (void)hipGetLastError();
    void *p = nullptr;
    TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return HIST_EDEVICE;
    nd.cus = pr.multiProcessorCount;
    nd.ptr = static_cast<uint32_t *>(p);
  }
  *out = &nd;
  return HIST_OK;
}

}  // namespace

// Diagnostics counters of the no-allocation launches on the current device (zeros before
// the first such launch), for hist_diag_read.
hist_status_t noalloc_diag(uint32_t out[3]) {
  out[0] = out[1] = out[2] = 0;
  int dev = 0;
  TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return HIST_OK;
  uint32_t *p;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    p = g_noalloc[dev].ptr;
  }
  if (!p) return HIST_OK;
  TRY_HIP(hipMemcpy(out, p + kDiagWord, 3 * sizeof(uint32_t), hipMemcpyDeviceToHost));
  return HIST_OK;
}

}  // namespace histmi

using namespace histmi;
using namespace histmi::rt;

extern "C" hist_status_t hist_u8_noalloc(const void *d_in, size_t n, uint32_t *d_out, hist_mode_t mode,
                                         const hist_pattern_t *h_pat, void *stream) {
  if (!d_out || (n && !d_in) || !mode_ok(mode)) return HIST_EINVAL;
  if ((uint64_t)n > kMaxSegBytes) return HIST_EOVERFLOW;
  Params P;
  init_params(&P);
  TRY(select_kind(mode, h_pat, &P));
  NoallocDev *nd;
  TRY(noalloc_dev(&nd));
  // the launch shape of hist_u8 (run_single): one workgroup per 16 KiB step at most, else
  // the whole grid
  const uint32_t lds = lds_bytes(P);
  const uint32_t G = (uint32_t)nd->cus * blocks_per_cu(P.kind, lds);
  const uint32_t ntiles = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(G, ceil_div(n, 16384)));
  const uint32_t copies = std::min<uint32_t>(g_single_copies, pow2ceil32(ntiles));
  if (copies > kNoallocCopies) return HIST_ENOMEM;   // more scratch than the array holds
  hipStream_t s = static_cast<hipStream_t>(stream);
  P.seg0.ptr = static_cast<const uint8_t *>(d_in);
  P.seg0.size = n;
  P.seg0.out = d_out;
  P.seg0.tile0 = 0;
  P.seg0.ntiles = ntiles;
  P.nseg = 1;
  P.single = 1;
  P.ntiles = ntiles;
  P.dynamic = 0;
  P.clog2 = log2u(copies);
  P.ctr = nd->ptr + kCtrWord;
  P.seg_done = nd->ptr + kSegDoneWord;
  P.partial = nd->ptr + kPartialWord;
  P.diag = nd->ptr + kDiagWord;
  hipLaunchKernelGGL(clear_scratch_kernel, dim3(1), dim3(kBlock), 0, s, nd->ptr, copies);
  TRY_HIP(hipGetLastError());
  return dev_err(launch_hist(P, LaunchShape{ntiles, lds, 4}, s));
}
