// noalloc.hip -- the relinearisation key switch without device allocation,
// for callers that cannot allocate (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Its working rows live in
// one file-scope device array, `scratch`, of a fixed size; every GPU the
// library runs on holds its own copy until the process ends.
#include <mutex>

#include "internal.hpp"

namespace sfhe {

// 64 MiB: at N = 2^14 with five data and three special primes a key switch
// at the top level needs 39 rows of 128 KiB, so up to 13 ciphertexts fit
constexpr int64_t kScratchBytes = (int64_t)64 << 20;
static __device__ __align__(256) u64 scratch[kScratchBytes / sizeof(u64)];

// the array's device address per device: the host-side name `scratch` is a
// stand-in, not a device address, so kernels get this pointer instead
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static u64* g_scratch_ptr[kMaxDevices] = {};

int noalloc_setup(sfhe_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return SFHE_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[c->device]) return SFHE_OK;
  int cur = -1;
  SFHE_HIP(hipGetDevice(&cur));
  if (cur != c->device) SFHE_HIP(hipSetDevice(c->device));
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != c->device) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return SFHE_E_DEVICE;
  }
  g_scratch_ptr[c->device] = (u64*)p;
  return SFHE_OK;
}

static u64* scratch_of(const sfhe_ctx* c) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return c->device >= 0 && c->device < kMaxDevices ? g_scratch_ptr[c->device] : nullptr;
}

}  // namespace sfhe

using namespace sfhe;

extern "C" {

int sfhe_keyswitch_noalloc(sfhe_ctx* c, int32_t level, const uint64_t* d2, uint64_t* out, int32_t batch,
                           void* stream) {
  try {
    if (!c || !d2 || !out) { set_error("NULL argument"); return SFHE_E_INVALID_ARG; }
    if (!c->has_keys) { set_error("keygen first"); return SFHE_E_STATE; }
    if (level < 0 || level >= c->L || batch < 0) { set_error("bad level or batch"); return SFHE_E_LEVEL; }
    const int64_t words = keyswitch_scratch_words(c, level, batch);
    if (words * (int64_t)sizeof(u64) > kScratchBytes) {
      set_error("sfhe_keyswitch_noalloc: the batch needs " + std::to_string(words * sizeof(u64)) +
                " bytes of scratch, above the fixed " + std::to_string(kScratchBytes) +
                "; split it into smaller batches");
      return SFHE_E_INVALID_ARG;
    }
    if (batch == 0) return SFHE_OK;
    u64* p = scratch_of(c);
    if (!p) { set_error("scratch not set up for this device"); return SFHE_E_DEVICE; }
    const int64_t nl = level + 1, N = c->N;
    return keyswitch_batch(c, level, d2, nl * N, out, 2 * nl * N, false, batch, (hipStream_t)stream, nullptr, p);
  } catch (...) {
    set_error("unexpected internal error");
    return SFHE_E_INVALID_ARG;
  }
}

}  // extern "C"
