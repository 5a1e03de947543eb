// Allocation-free binding: alch_nb_bind_static() binds a context to a
// device array that the library owns, for callers that cannot allocate
// device memory (code under graph capture, serving loops, harnesses that
// forbid hipMalloc).
//
// The array is a file-scope __device__ object: every GPU the library runs
// on holds its own copy, of kScratchBytes, until the process ends.  In host
// code its name is only a stand-in for the symbol, so the device address is
// fetched once per device with hipGetSymbolAddress (that device current) and
// kept; kernels receive that address through the context's workspace
// layout, never the symbol itself.
//
// One device array serves one context at a time: binding a context takes
// the array over (the previous owner's calls then fail with
// ALCH_NB_E_NOT_BOUND), and the binding clears the whole workspace, so no
// state of an earlier owner survives.  Work of two contexts on one device
// that overlaps in time races on the array: the caller must let the
// previous owner's enqueued work finish (same stream, or a sync) before
// binding another context.
#include <hip/hip_runtime.h>

#include <mutex>

#include "alch_nb.h"
#include "anb_kernels.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // ALCH_NB_STATIC_SCRATCH_BYTES
static_assert(kScratchBytes == ALCH_NB_STATIC_SCRATCH_BYTES, "header and library agree on the scratch size");
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};               // device address of the array, per device
const alch_nb_ctx* g_owner[kMaxDevices] = {};  // context bound to it

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

bool anb_static_owns(const alch_nb_ctx* ctx, int device) {
  if (device < 0 || device >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_owner[device] == ctx;
}

void anb_static_release(const alch_nb_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (int k = 0; k < kMaxDevices; ++k)
    if (g_owner[k] == ctx) g_owner[k] = nullptr;
}

extern "C" alch_nb_status alch_nb_bind_static(alch_nb_ctx* ctx, void* stream) {
  if (!ctx) return ALCH_NB_E_INVALID_ARG;
  size_t need = 0;
  alch_nb_status st = alch_nb_workspace_size(ctx, &need);
  if (st != ALCH_NB_OK) return st;
  if (need > kScratchBytes) return ALCH_NB_E_SCRATCH_SIZE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return ALCH_NB_E_NO_DEVICE;
  if (dev >= kMaxDevices) return ALCH_NB_E_UNSUPPORTED;
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ALCH_NB_E_HIP;
      g_addr[dev] = p;
    }
    base = g_addr[dev];
    // take the array over from the previous owner, if any
    for (int k = 0; k < kMaxDevices; ++k)
      if (g_owner[k] == ctx) g_owner[k] = nullptr;
    g_owner[dev] = ctx;
  }
  st = anb_bind(ctx, base, kScratchBytes, stream, dev);
  if (st != ALCH_NB_OK) anb_static_release(ctx);
  return st;
}
