// Shared internals of the kernel library: launch environment handed from the
// runtime to the kernel launchers, and device helpers (wave64 scans and
// decoupled look-back).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ka {

// ------------------------------------------------------------------------------
// Host side: what a launcher needs from the runtime.
// ------------------------------------------------------------------------------

// Look-back state of one stream.  A look-back kernel numbers its tiles by
// work-group id, and every wait in its look-back is bounded (see
// lb_lookback), so it needs no co-residency guarantee, no cooperative launch
// and no ticket counter.  Status words are tagged with a per-launch epoch, so
// stale words from earlier launches read as "not yet published" and nothing
// has to be cleared between launches.
struct LookbackArena {
  uint64_t* status = nullptr;  // device status words
  uint64_t status_words = 0;
  uint64_t status_bytes = 0;   // size of the pool block holding `status`
  uint32_t epoch = 0;          // last epoch handed out (1 .. 2^30-1)
  void* plan = nullptr;        // radix sort plan: kSortPlanBytes of device memory
};

constexpr uint32_t kSortPlanBytes = 8192;

// Per-launch arguments of a look-back kernel.
struct LbArgs {
  uint64_t* status;
  uint32_t epoch;
  uint32_t spin_limit;  // polls of a silent predecessor before the fallback (>= 1)
};

constexpr uint32_t kLbSpinLimit = 16;  // the default spin_limit

class Env {
 public:
  virtual ~Env() = default;
  virtual hipStream_t stream() = 0;
  // Temporary device memory, freed in stream order after the launch is queued.
  virtual void* scratch(uint64_t bytes) = 0;
  // Reserves `words` status words and one epoch.
  virtual bool lookback(uint64_t words, LbArgs* out) = 0;
  virtual LookbackArena* arena() = 0;
  // Optional timing of one launch (no-ops unless profiling is on).
  virtual void prof_begin(const char* kernel) = 0;
  virtual void prof_end(const char* kernel) = 0;
  // Records a failure message; returns the code.
  virtual int fail(int code, const char* msg) = 0;
};

// Launchers (one file each).  They queue work on env.stream() and return a
// KA_* code.  `d_n`, when not null, points to the true element count on the
// device (at most n_cap), written by an earlier stage.
int launch_affine(Env& env, uint32_t* x, uint64_t n_cap, const uint64_t* d_n, uint64_t offset, uint32_t a,
                  uint32_t b);
int launch_exclusive_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n);
int launch_compact_nonzero(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n,
                           uint64_t* d_out_len);
int launch_radix_sort_pairs(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys,
                            uint32_t* srows, uint64_t n, int shape = 0);
// Number of tile shapes launch_radix_sort_pairs offers (shape 0 is the default).
int sort_shape_count();
int launch_wah_encode(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                      uint64_t* d_len_words, const uint32_t* req_base = nullptr, uint32_t req_shift = 32);
// Batched index build: nreq requests, values concatenated, req_off[j] the
// first position of request j (req_off[nreq] = n).  max_req: the largest
// request, when the caller knows it (kMaxReqUnknown otherwise); batches of
// small requests take a one-work-group-per-request path.
constexpr uint32_t kMaxReqUnknown = 0xFFFFFFFFu;
int launch_wah_batch(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                     uint32_t value_bits, uint32_t* keys, uint32_t* offsets, uint32_t* words, uint32_t* key_start,
                     uint32_t* word_start, uint64_t* len_keys, uint64_t* len_offsets, uint64_t* len_words,
                     uint64_t* len_key_start, uint64_t* len_word_start, int sort_shape = 0,
                     uint32_t max_req = kMaxReqUnknown);
// Exclusive scan of each of nreq requests concatenated in in[0..n) (req_off as
// for the batched index).
int launch_segmented_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* req_off,
                          uint32_t nreq);
int launch_fill_u64(Env& env, uint64_t* p, uint64_t count, uint64_t value);
int launch_fill_u32(Env& env, uint32_t* p, uint64_t count, uint32_t value);
int launch_set_len(Env& env, uint64_t* d_len, uint64_t value);
int launch_copy_len(Env& env, uint64_t* dst, const uint64_t* src);

// Status codes shared with ka.h.
constexpr int kOk = 0, kErrArg = -1, kErrDevice = -5, kErrOom = -6, kErrLaunch = -10;

inline int check_launch(Env& env, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return env.fail(kErrLaunch, what);
  return kOk;
}

// ------------------------------------------------------------------------------
// Device side.
// ------------------------------------------------------------------------------
#if defined(__HIP_DEVICE_COMPILE__) || defined(__HIPCC__)

constexpr uint32_t kLbAggregate = 1u;  // status flag: tile total only
constexpr uint32_t kLbInclusive = 2u;  // status flag: prefix including the tile

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Native 4 x uint32 vector: one 16-byte global access.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Inclusive wave64 prefix sum: row_shr 1,2,4,8 inside each row of 16 lanes,
// then row_bcast:15 and row_bcast:31 carry row totals across rows.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
  return x;
}

__device__ __forceinline__ uint32_t wave_read_last(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x) { return wave_read_last(wave_incl_scan(x)); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

// Exclusive block-wide prefix sum of one value per thread.  s_wave needs
// BLOCK/64 words; the caller separates reuses of s_wave with a barrier.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wave, uint32_t* total) {
  constexpr int kWaves = BLOCK / 64;
  const uint32_t inc = wave_incl_scan(x);
  const uint32_t w = threadIdx.x / 64;
  if (lane_id() == 63) s_wave[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t t = s_wave[i];
    before += (i < (int)w) ? t : 0u;
    tot += t;
  }
  *total = tot;
  return before + inc - x;
}

// ---- decoupled look-back -------------------------------------------------------

__device__ __forceinline__ uint64_t lb_pack(uint32_t value, uint32_t epoch, uint32_t flag) {
  return ((uint64_t)value << 32) | ((uint64_t)epoch << 2) | flag;
}

__device__ __forceinline__ void lb_publish(uint64_t* p, uint32_t value, uint32_t epoch, uint32_t flag) {
  __hip_atomic_store(p, lb_pack(value, epoch, flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Flag of a status word in this launch (0: not yet published).
__device__ __forceinline__ uint32_t lb_flag(uint64_t w, uint32_t epoch) {
  return (((uint32_t)w >> 2) == epoch) ? ((uint32_t)w & 3u) : 0u;
}

// Decoupled look-back with fallback by one whole wave; status[t] is tile t's
// status word.  In a round, lane l inspects the kDepth predecessors
// j - kDepth*l .. j - kDepth*l - kDepth + 1, so one round trip to memory covers
// 64*kDepth tiles; the window slides back until an inclusive prefix is found.
// A predecessor that has published nothing after spin_limit polls is no
// longer waited for: the wave computes its total itself with reduce(t) --
// every lane calls it, and it returns the tile's total in every lane -- adds
// it and goes on from the tile before it.  Every wait is therefore bounded
// whatever order the work-groups run in, so tiles can be numbered by
// work-group id.  reduce(t) may only read data that no work-group of the
// launch writes.  Returns the exclusive prefix of `tile` in every lane.
template <int kDepth, class Reduce>
__device__ __forceinline__ uint32_t lb_lookback(const uint64_t* status, uint32_t tile, uint32_t epoch,
                                                uint32_t spin_limit, Reduce&& reduce) {
  const uint32_t lane = lane_id();
  uint32_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    uint64_t w[kDepth];
#pragma unroll
    for (int k = 0; k < kDepth; ++k) {
      const int64_t idx = j - (int64_t)(kDepth * lane + k);
      w[k] = idx >= 0 ? lb_load(status + idx) : 0ull;
    }
    // This lane's run of predecessors, nearest first: state 2 = reaches an
    // inclusive prefix (or the start), 1 = all aggregates, 0 = meets an
    // unpublished tile, at position `gap`; sum = the values before it.
    uint32_t state = 1, sum = 0, gap = 0;
#pragma unroll
    for (int k = 0; k < kDepth; ++k) {
      if (state != 1) break;
      const int64_t idx = j - (int64_t)(kDepth * lane + k);
      if (idx < 0) {
        state = 2;
        break;
      }
      const uint32_t f = lb_flag(w[k], epoch);
      if (f == 0) {
        state = 0;
        gap = (uint32_t)k;
        break;
      }
      sum += (uint32_t)(w[k] >> 32);
      if (f == kLbInclusive) state = 2;
    }
    const uint64_t inc = __ballot(state == 2);
    const uint64_t stall = __ballot(state == 0);
    const uint32_t stop = inc ? (uint32_t)__builtin_ctzll(inc) : 63u;
    const uint64_t need = (stop == 63u) ? ~0ull : ((2ull << stop) - 1ull);
    const uint64_t blocked = stall & need;
    if (blocked) {
      if (++spins < spin_limit) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      // The nearest unpublished tile u: lanes below s saw aggregates only,
      // lane s those before u.  Take u's total from its input.
      const uint32_t s = (uint32_t)__builtin_ctzll(blocked);
      const uint32_t gs = (uint32_t)__builtin_amdgcn_readlane((int)gap, (int)s);
      excl += wave_sum(lane <= s ? sum : 0u);
      const int64_t u = j - (int64_t)(kDepth * s + gs);
      excl += reduce((uint32_t)u);
      j = u - 1;
      spins = 0;
      continue;
    }
    excl += wave_sum(lane <= stop ? sum : 0u);
    if (inc) break;
    j -= 64 * kDepth;
    spins = 0;
  }
  return excl;
}

// Reads the element count: the device-resident one when given.
__device__ __forceinline__ uint64_t device_count(uint64_t n_cap, const uint64_t* d_n) {
  if (!d_n) return n_cap;
  const uint64_t n = *d_n;
  return n < n_cap ? n : n_cap;
}

#endif  // device

}  // namespace ka
