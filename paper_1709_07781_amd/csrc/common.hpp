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
// lb_lookback_st), so it needs no co-residency guarantee, no cooperative launch
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
  // Polls of a silent predecessor before a look-back takes the fallback.
  virtual uint32_t spin_limit() { return kLbSpinLimit; }
  // Optional timing of one launch (no-ops unless profiling is on).
  virtual void prof_begin(const char* kernel) = 0;
  virtual void prof_end(const char* kernel) = 0;
  // Records a failure message; returns the code.
  virtual int fail(int code, const char* msg) = 0;
};

// Launchers (one file each).  They queue work on env.stream() and return a
// KA_* code.  `d_n`, when not null, points to the true element count on the
// device (at most n_cap), written by an earlier stage.
// The stages x <- a[i] x + b[i], i = 0 .. len-1, applied in one pass over x
// (one launch per 16 stages): the served form's chain requests.
int launch_affine_chain(Env& env, uint32_t* x, uint64_t n, const uint32_t* a, const uint32_t* b, uint32_t len);
int launch_affine(Env& env, uint32_t* x, uint64_t n_cap, const uint64_t* d_n, uint64_t offset, uint32_t a,
                  uint32_t b);
int launch_exclusive_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n);
int launch_compact_nonzero(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n,
                           uint64_t* d_out_len);
int launch_radix_sort_pairs(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys,
                            uint32_t* srows, uint64_t n, int shape = 0, const uint64_t* d_n = nullptr);
// Number of tile shapes launch_radix_sort_pairs offers (shape 0 is the default).
int sort_shape_count();
// Number of variants of the batched index build (its sort_shape argument):
// 0 the segmented sort with the even digit split for values of at most 16
// bits, else the tagged sort with tile shape 0; 1 and 2 the tagged sort with
// tile shapes 1 and 2; 3 the segmented sort with the byte digit split.  A
// batch of small requests takes its own path: variant 1 the persistent fused
// launch, the others the three-launch form.
int batch_variant_count();
// Sort of a batch of requests (request j: values[req_off[j] .. req_off[j+1]),
// all below 2^value_bits, value_bits 1..16) by value inside each request,
// stable: skeys[i] = j << value_bits | value, srows[i] = the position inside
// the request, request j's pairs at [req_off[j], req_off[j+1]).  A value at or
// above 2^value_bits sets req_bad[j] (or *bad without req_bad); the caller
// clears them.
int launch_radix_sort_segments(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                               uint32_t value_bits, uint32_t* skeys, uint32_t* srows, uint32_t* bad,
                               uint32_t* req_bad, bool even_split = true);
// Device address of the OR of all keys of the last launch_radix_sort_pairs on
// this stream (valid once that sort has run, for n > 0).
const uint32_t* sort_plan_keys_or(Env& env);
// Stable sort of (key, row = position) for keys below 2^value_bits, value_bits
// 1..16, with uint16 sorted keys; a key at or above 2^value_bits sets
// *reject to 1 (0 otherwise; *reject is device memory).
int launch_radix_sort_rows16(Env& env, const uint32_t* keys, uint16_t* skeys, uint32_t* srows, uint64_t n,
                             uint32_t value_bits, uint32_t* reject, int shape = 0, const uint64_t* d_n = nullptr);
// WAH encoder over sorted pairs.  reject_flag, when given, voids the result
// (every output length 0) if (*reject_flag >> reject_shift) != 0 once the
// earlier kernels of the stream have run.
int launch_wah_encode(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                      uint64_t* d_len_words, const uint32_t* req_base = nullptr, uint32_t req_shift = 32,
                      const uint32_t* reject_flag = nullptr, uint32_t reject_shift = 32,
                      const uint64_t* d_n = nullptr);
// The same over uint16 sorted keys (values below 2^16).
int launch_wah_encode16(Env& env, const uint16_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                        uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                        uint64_t* d_len_words, const uint32_t* reject_flag = nullptr, uint32_t reject_shift = 32,
                        const uint64_t* d_n = nullptr);
// Index words in an encoder format (0 the paper's form, 1 canonical WAH with
// 1-fills, 2 PLWAH) from sorted pairs, through the group list.  A fill longer
// than the format's length field sets *reject (every output length 0).
int launch_wah_encode_format(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t fmt,
                             uint32_t* keys, uint32_t* offsets, uint32_t* words, uint64_t* len_keys,
                             uint64_t* len_offsets, uint64_t* len_words, uint32_t* reject,
                             const uint64_t* d_n = nullptr);
// One bitmap (m words, the count on the device when m_len is given) decoded
// into ngroups 31-bit group words; more groups than ngroups sets *reject.
int launch_wah_decode(Env& env, const uint32_t* words, uint64_t m_cap, const uint64_t* m_len, uint32_t fmt,
                      uint32_t ngroups, uint32_t* groups, uint32_t* reject);
// AND (op 0) / OR (op 1) of two bitmaps over ngroups groups, encoded in
// out_fmt into words (capacity 2 ngroups), its length in *len_words.
int launch_wah_combine(Env& env, const uint32_t* a, uint64_t a_cap, const uint64_t* a_len, const uint32_t* b,
                       uint64_t b_cap, const uint64_t* b_len, uint32_t in_fmt, uint32_t ngroups, uint32_t op,
                       uint32_t out_fmt, uint32_t* words, uint64_t* len_words, uint32_t* reject);
// slots[i] = d with keys[d] == queries[i], or 0xFFFFFFFF (keys ascending).
// q_len, when given, is the query count on the device (at most q).
int launch_wah_lookup(Env& env, const uint32_t* keys, uint64_t d_cap, const uint64_t* d_len, const uint32_t* queries,
                      uint64_t q, uint32_t* slots, const uint64_t* q_len = nullptr);
int launch_wah_encode_format16(Env& env, const uint16_t* skeys, const uint32_t* srows, uint64_t n, uint32_t fmt,
                               uint32_t* keys, uint32_t* offsets, uint32_t* words, uint64_t* len_keys,
                               uint64_t* len_offsets, uint64_t* len_words, uint32_t* reject,
                               const uint64_t* d_n = nullptr);
int launch_zero_u32(Env& env, uint32_t* p);
// *reject = 1 if (*keys_or >> bits) != 0 (bits < 32).
int launch_reject_above(Env& env, const uint32_t* keys_or, uint32_t bits, uint32_t* reject);
// *len = *reject ? 0 : value.
int launch_len_unless(Env& env, uint64_t* len, uint64_t value, const uint32_t* reject);
// Batched index build: nreq requests, values concatenated, req_off[j] the
// first position of request j (req_off[nreq] = n).  max_req: the largest
// request, when the caller knows it (kMaxReqUnknown otherwise); batches of
// small requests take a one-work-group-per-request path.  A value at or above
// 2^value_bits rejects the whole batch (every output length 0), or, with
// req_bad (nreq device words), only its own request: req_bad[j] = 1 and that
// request's slices are unspecified while every other request's are exact.
constexpr uint32_t kMaxReqUnknown = 0xFFFFFFFFu;
int launch_wah_batch(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                     uint32_t value_bits, uint32_t* keys, uint32_t* offsets, uint32_t* words, uint32_t* key_start,
                     uint32_t* word_start, uint64_t* len_keys, uint64_t* len_offsets, uint64_t* len_words,
                     uint64_t* len_key_start, uint64_t* len_word_start, int sort_shape = 0,
                     uint32_t max_req = kMaxReqUnknown, uint32_t* req_bad = nullptr,
                     const uint64_t* d_n = nullptr);
// Exclusive scan of each of nreq requests concatenated in in[0..n) (req_off as
// for the batched index).
int launch_segmented_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* req_off,
                          uint32_t nreq);
int launch_fill_u64(Env& env, uint64_t* p, uint64_t count, uint64_t value);
int launch_fill_u32(Env& env, uint32_t* p, uint64_t count, uint32_t value);
int launch_set_len(Env& env, uint64_t* d_len, uint64_t value);
int launch_copy_len(Env& env, uint64_t* dst, const uint64_t* src);
// *dst = *src (a uint32 count, e.g. a request table's last entry, as a length).
int launch_len_from_u32(Env& env, uint64_t* dst, const uint32_t* src);

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
// Status slots of every look-back chain: one status word per 64-byte line,
// at status[kLbSpread * tile].  Each slot is stored twice (aggregate, then
// inclusive) while later tiles poll it, and with eight words to a line those
// stores and polls queue on the same lines: the WAH encoder over 2^26 Zipf
// pairs took 228 us packed and 215 us spread (4 to 32 words apart: 214-216 us).
constexpr uint32_t kLbSpread = 8;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Native 4 x uint32 vector: one 16-byte global access.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Four words at word alignment: global loads and stores of 16 bytes need only
// 4-byte alignment on this target.
typedef uint32_t u32x4w __attribute__((ext_vector_type(4), aligned(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// Four consecutive keys p[4q .. 4q+3] from one 16-byte (uint32 keys) or 8-byte
// (uint16 keys) non-temporal load; p must be aligned to that size.
__device__ __forceinline__ void load_key4(const uint32_t* __restrict__ p, uint64_t q, uint32_t (&k)[4]) {
  const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p) + q);
  k[0] = a.x, k[1] = a.y, k[2] = a.z, k[3] = a.w;
}
__device__ __forceinline__ void load_key4(const uint16_t* __restrict__ p, uint64_t q, uint32_t (&k)[4]) {
  const u32x2 a = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(p) + q);
  k[0] = a.x & 0xFFFFu, k[1] = a.x >> 16, k[2] = a.y & 0xFFFFu, k[3] = a.y >> 16;
}

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

__device__ __forceinline__ void lb_publish_raw(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Status words of a look-back chain.  LbEpoch: [value:32 | epoch:30 | flag:2],
// stale words of earlier launches read as unpublished, nothing is cleared.
// LbPair: two counts [a:32 | b:30 | flag:2] with no epoch, in a region cleared
// before the launch (b sums below 2^30, so adding whole words never carries
// into a).
struct LbEpoch {
  typedef uint32_t sum_t;
  uint32_t epoch;
  __device__ __forceinline__ uint32_t flag(uint64_t w) const { return lb_flag(w, epoch); }
  __device__ __forceinline__ sum_t payload(uint64_t w) const { return (uint32_t)(w >> 32); }
  __device__ __forceinline__ static sum_t zero() { return 0u; }
  __device__ __forceinline__ static sum_t add(sum_t x, sum_t y) { return x + y; }
  __device__ __forceinline__ static sum_t wave_total(sum_t x) { return wave_sum(x); }
};

struct LbPairSum {
  uint32_t a, b;
};

__device__ __forceinline__ uint64_t lb_pack_pair(uint32_t a, uint32_t b, uint32_t flag) {
  return ((uint64_t)a << 32) | ((uint64_t)b << 2) | flag;
}

struct LbPair {
  typedef LbPairSum sum_t;
  __device__ __forceinline__ uint32_t flag(uint64_t w) const { return (uint32_t)w & 3u; }
  __device__ __forceinline__ sum_t payload(uint64_t w) const { return {(uint32_t)(w >> 32), (uint32_t)w >> 2}; }
  __device__ __forceinline__ static sum_t zero() { return {0u, 0u}; }
  __device__ __forceinline__ static sum_t add(sum_t x, sum_t y) { return {x.a + y.a, x.b + y.b}; }
  __device__ __forceinline__ static sum_t wave_total(sum_t x) { return {wave_sum(x.a), wave_sum(x.b)}; }
};

// One step over a window of status words: lane l holds w, the word of tile
// j - l.  Adds the aggregates up to the nearest inclusive prefix (returns true,
// done) or up to the nearest unpublished tile, which becomes the new j; with
// all 64 aggregates, j moves 64 tiles back.
template <class St>
__device__ __forceinline__ bool lb_window_step(uint64_t w, const St& st, int64_t& j, typename St::sum_t& excl) {
  typedef typename St::sum_t S;
  const uint32_t lane = lane_id();
  const int64_t idx = j - (int64_t)lane;
  const uint32_t f = idx >= 0 ? st.flag(w) : kLbInclusive;  // before tile 0: a zero prefix
  const S v = idx >= 0 && f ? st.payload(w) : St::zero();
  const uint64_t stop = __ballot(f == kLbInclusive);
  const uint64_t gap = __ballot(f == 0);
  const uint32_t first_stop = stop ? (uint32_t)__builtin_ctzll(stop) : 64u;
  const uint32_t first_gap = gap ? (uint32_t)__builtin_ctzll(gap) : 64u;
  if (first_gap < first_stop) {  // lanes below the gap hold aggregates
    excl = St::add(excl, St::wave_total(lane < first_gap ? v : St::zero()));
    j -= first_gap;
    return false;
  }
  if (first_stop < 64u) {
    excl = St::add(excl, St::wave_total(lane <= first_stop ? v : St::zero()));
    return true;
  }
  excl = St::add(excl, St::wave_total(v));
  j -= 64;
  return false;
}

// Decoupled look-back with fallback by one whole wave; status[kStride * t] is
// tile t's status word, read through the policy St (LbEpoch or LbPair).  The wave waits
// on the nearest tile it has not yet accounted for, j, with one status read per
// poll (every lane reads the same word, one request): polling a wide window
// instead makes every waiting wave re-read kilobytes per poll, which competes
// with the streaming traffic of the whole chip.  Once tile j has published, a
// window of the 64 tiles j, j-1, ..., j-63 (lane l reads tile j - l) is summed
// up to the nearest inclusive prefix; an unpublished tile inside the window
// becomes the next tile waited on.  A tile that has published nothing after
// spin_limit polls is no longer waited for: the wave computes its total itself
// with reduce(t) -- every lane calls it, and it returns the tile's total in
// every lane -- and goes on from the tile before it.  Every wait is therefore
// bounded whatever order the work-groups run in, so tiles can be numbered by
// work-group id.  reduce(t) may only read data that no work-group of the
// launch writes.  Returns the exclusive prefix of `tile` in every lane.
template <uint32_t kStride = 1, class St, class Reduce>
__device__ __forceinline__ typename St::sum_t lb_lookback_st(const uint64_t* status, uint32_t tile, const St& st,
                                                             uint32_t spin_limit, Reduce&& reduce) {
  typedef typename St::sum_t S;
  const uint32_t lane = lane_id();
  S excl = St::zero();
  int64_t j = (int64_t)tile - 1;
  uint32_t spins = 0;
  while (j >= 0) {
    const uint64_t w0 = lb_load(status + kStride * j);
    const uint32_t f0 = st.flag(w0);
    if (f0 == 0) {
      if (++spins < spin_limit) {
        __builtin_amdgcn_s_sleep(2);
        continue;
      }
      excl = St::add(excl, reduce((uint32_t)j));
      j -= 1;
      spins = 0;
      continue;
    }
    spins = 0;
    if (f0 == kLbInclusive) {
      excl = St::add(excl, st.payload(w0));
      break;
    }
    // Tile j holds an aggregate: sum the window below it.
    const int64_t idx = j - (int64_t)lane;
    const uint64_t w = (lane && idx >= 0) ? lb_load(status + kStride * idx) : w0;
    if (lb_window_step(w, st, j, excl)) break;
  }
  return excl;
}

// Look-back without fallback, for chains whose every tile is being worked on
// by a running work-group (tiles handed out in order by a ticket counter, so a
// tile waited for is held by a work-group that waits only for earlier ones):
// polls the nearest tile not yet accounted for, then sums windows of 64 as
// lb_lookback_st does (tile t's word at status[kStride * t]).
template <uint32_t kStride = 1, class St>
__device__ __forceinline__ typename St::sum_t lb_lookback_ticket(const uint64_t* status, uint32_t tile,
                                                                 const St& st) {
  typedef typename St::sum_t S;
  const uint32_t lane = lane_id();
  S excl = St::zero();
  int64_t j = (int64_t)tile - 1;
  while (j >= 0) {
    const uint64_t w0 = lb_load(status + kStride * j);
    const uint32_t f0 = st.flag(w0);
    if (f0 == 0) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    if (f0 == kLbInclusive) {
      excl = St::add(excl, st.payload(w0));
      break;
    }
    const int64_t idx = j - (int64_t)lane;
    const uint64_t w = (lane && idx >= 0) ? lb_load(status + kStride * idx) : w0;
    if (lb_window_step(w, st, j, excl)) break;
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
