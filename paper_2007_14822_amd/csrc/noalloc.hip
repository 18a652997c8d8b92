// Allocation-free dense H_eff*psi.  Its scratch (psi transposed, the
// W-stage output, converted environments, the W-stage tables) is carved from
// one fixed device array of the library instead of the handle's workspace,
// so the call makes no device allocation.
#include <mutex>

#include "handle.h"

namespace {

// Largest scratch one call may use (bf16, d = 2, w = 5, nv = 1: chi up to
// about 1180; checked per call, with a message naming the need).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;

// Every device the library runs on holds its own copy of this array until
// the process ends.  Host code never passes its name to a kernel: the
// device address is looked up per device below.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
bool g_done[kMaxDevices];
hipError_t g_err[kMaxDevices];
void* g_ptr[kMaxDevices];

}  // namespace

namespace itn {

// Look up this device's address of the scratch array, once per device, with
// the device current (called by itn_create).  The status is kept and
// reported by the entry point.
void noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_done[device] = true;
}

}  // namespace itn

using namespace itn;

extern "C" {

itn_status itn_heff_apply_noalloc(itn_handle* h, const itn_tensor* L, const itn_tensor* W1,
                                  const itn_tensor* W2, const itn_tensor* R, const itn_tensor* psi,
                                  int32_t nv, itn_tensor* out, itn_prec prec, void* hip_stream) {
  if (!h) return ITN_E_ARG;
  if (h->device < 0) return fail(h, ITN_E_NODEVICE, "host-only handle cannot launch work");
  if (h->device >= kMaxDevices) return fail(h, ITN_E_UNSUPPORTED, "device index %d too large", h->device);
  void* p = nullptr;
  hipError_t e = hipSuccess;
  bool done = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    done = g_done[h->device];
    e = g_err[h->device];
    p = g_ptr[h->device];
  }
  if (!done) return fail(h, ITN_E_HIP, "scratch of device %d was not set up", h->device);
  if (e != hipSuccess || !p) return hip_fail(h, e, "hipGetSymbolAddress(scratch)");
  FixedScratch fs;
  fs.base = p;
  fs.bytes = kScratchBytes;
  return heff_apply_terms(h, 1, &L, &W1, &W2, &R, psi, nv, out, prec, hip_stream, &fs);
}

itn_status itn_heff_noalloc_max_bytes(size_t* bytes) {
  if (!bytes) return ITN_E_ARG;
  *bytes = kScratchBytes;
  return ITN_OK;
}

}  // extern "C"
