// ka_wah_index_noalloc: the composed index build (radix sort of (value, row)
// pairs, then the WAH encoder) for callers that cannot allocate device memory.
//
// Every scratch buffer the kernels need -- the sorted pairs, the sort's
// ping-pong pair, its digit tables and plan, the look-back status words of its
// table scans and the encoder's tile counts -- is carved out of one
// file-scope device array, `scratch`, whose device address is looked up once
// per device.  Nothing here calls hipMalloc, hipFree, hipMemset or any other
// allocating routine; the kernels are the same ones ka_wah_index launches.
// The array keeps the contents of the last call: the status words are cleared
// by a fill kernel at the start of every call, and every other region is fully
// written before it is read.  Calls that overlap on one device (different
// streams, or threads without ordering) share the array and race.
#include <mutex>

#include "runtime_internal.hpp"

namespace ka {
namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kMaxN = KA_NOALLOC_MAX_N;
constexpr uint64_t kStatusWords = 8192;  // look-back status words of the table scans (kLbSpread per tile)
constexpr uint64_t kStatusBytes = kStatusWords * 8;
constexpr uint64_t kPairBytes = kMaxN * 4;               // one uint32 array of kMaxN elements
constexpr uint64_t kTableBytes = (kMaxN / 4096 + 1) * 256 * 4;  // digit table at the smallest sort tile
constexpr uint64_t kTileBytes = (kMaxN / 4096 + 1) * 8 + 4096;  // orand, encoder tile counts, group totals
constexpr uint64_t kEncStatusBytes = (kMaxN / 4096 + 1) * 8 * kLbSpread;  // encoder status slots
constexpr uint64_t kScratchBytes =
    kStatusBytes + kSortPlanBytes + 4 * kPairBytes + 2 * kTableBytes + 6 * kTileBytes + kEncStatusBytes + 16 * kAlign;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up on the first call with
// that device current.
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(KA_E_DEVICE, "device ordinal beyond the supported count");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(KA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return KA_OK;
}

// Launch environment over the static array: scratch by bump allocation, one
// cleared status region with a fresh epoch per look-back launch.
class NoAllocEnv final : public Env {
 public:
  NoAllocEnv(char* base, hipStream_t s) : base_(base), s_(s) {
    arena_.status = reinterpret_cast<uint64_t*>(base_);
    arena_.status_words = kStatusWords;
    arena_.plan = base_ + kStatusBytes;
    used_ = kStatusBytes + kSortPlanBytes;
  }
  hipStream_t stream() override { return s_; }
  void* scratch(uint64_t bytes) override {
    const uint64_t at = (used_ + kAlign - 1) / kAlign * kAlign;
    if (at + bytes > kScratchBytes) return nullptr;
    used_ = at + bytes;
    return base_ + at;
  }
  bool lookback(uint64_t words, LbArgs* out) override {
    if (words > kStatusWords || arena_.epoch + 1 >= (1u << 30)) return false;
    out->status = arena_.status;
    out->epoch = ++arena_.epoch;
    out->spin_limit = kLbSpinLimit;
    return true;
  }
  LookbackArena* arena() override { return &arena_; }
  void prof_begin(const char*) override {}
  void prof_end(const char*) override {}
  int fail(int code, const char* msg) override { return set_error(code, msg); }

 private:
  char* base_;
  hipStream_t s_;
  uint64_t used_ = 0;
  LookbackArena arena_;
};

}  // namespace
}  // namespace ka

using namespace ka;

extern "C" KA_API int ka_wah_index_noalloc(const uint32_t* values, uint64_t n, uint32_t* keys, uint32_t* offsets,
                                           uint32_t* words, uint64_t* lengths, void* stream) {
  try {
    if (!offsets || !lengths || (n && (!values || !keys || !words))) return set_error(KA_E_ARG, "null argument");
    if (n > kMaxN)
      return set_error(KA_E_ARG, "ka_wah_index_noalloc: n exceeds KA_NOALLOC_MAX_N (the static scratch size)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(KA_E_DEVICE, "no current HIP device");
    void* base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc) return rc;
    NoAllocEnv env(static_cast<char*>(base), static_cast<hipStream_t>(stream));
    // Status words start at zero in every call (a fill kernel: no memset node
    // if the caller captures the call into a graph).
    if ((rc = launch_fill_u64(env, reinterpret_cast<uint64_t*>(base), kStatusWords, 0))) return rc;
    uint32_t* skeys = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
    uint32_t* srows = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
    if (!skeys || !srows) return set_error(KA_E_ARG, "ka_wah_index_noalloc: scratch exhausted");
    if ((rc = launch_radix_sort_pairs(env, values, nullptr, skeys, srows, n))) return rc;
    return launch_wah_encode(env, skeys, srows, n, keys, offsets, words, lengths, lengths + 1, lengths + 2);
  } catch (...) {
    return set_error(KA_E_DEVICE, "unexpected internal error");
  }
}
