// tt_round_rand_noalloc: the rounding of tt_round_rand for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation).  Its workspace is a fixed
// file-scope device array of TT_NOALLOC_SCRATCH_BYTES; each GPU the library
// runs on holds its own copy from module load to process end.
//
// In host code the array's name is only a stand-in for its device address:
// the address is fetched once per device with hipGetSymbolAddress (on the
// first call on that device, with the device current) and only that pointer
// is handed to kernels.  Every call on a GPU shares that GPU's array, so
// calls that overlap on one GPU (two host threads, or two streams without
// ordering) race; the rounding needs no part of the array to start at zero
// (every value it reads is written earlier in the same call).
#include <mutex>

#include "tt_internal.h"

namespace ttr {
namespace {

__device__ __align__(256) char scratch[TT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array
int scratch_address(void **out) {
  int dev = -1;
  TTR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(TT_EUNSUPPORTED, "tt_round_rand_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    TTR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(TT_EHIP, "tt_round_rand_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TT_OK;
}

}  // namespace
}  // namespace ttr

using namespace ttr;

extern "C" {

int tt_round_rand_noalloc(int32_t N, const int64_t *dims, const int64_t *ranks,
                          const void *const *cores, int32_t dtype, int64_t target_rank,
                          int64_t oversample, uint64_t sketch_seed, int32_t prec,
                          void *const *out_cores, void *stream) {
  size_t need = 0;
  TTR_TRY(tt_round_rand_workspace(N, dims, ranks, target_rank, oversample, prec, &need));
  if (need > (size_t)TT_NOALLOC_SCRATCH_BYTES)
    return fail(TT_EUNSUPPORTED, "tt_round_rand_noalloc: this rounding needs " +
                                     std::to_string(need) + " bytes of workspace, the fixed "
                                     "scratch array holds " +
                                     std::to_string((size_t)TT_NOALLOC_SCRATCH_BYTES));
  void *ws = nullptr;
  TTR_TRY(scratch_address(&ws));
  // the guarded form: no read-back, no synchronisation, no host buffer
  struct SpecOff {
    bool prev = g_spec_off;
    SpecOff() { g_spec_off = true; }
    ~SpecOff() { g_spec_off = prev; }
  } guard;
  return tt_round_rand(N, dims, ranks, cores, dtype, target_rank, oversample, sketch_seed, prec,
                       out_cores, ws, (size_t)TT_NOALLOC_SCRATCH_BYTES, stream);
}

}  // extern "C"
