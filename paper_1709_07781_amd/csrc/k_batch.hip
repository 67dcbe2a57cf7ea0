// Batched WAH index build: many independent requests in one pass of the
// pipeline (Sec. 3.6 names nesting data parallelism inside a kernel as an
// alternative level of composition to one actor per stage; Sec. 4 is the
// per-request index).
//
// The requests' values are concatenated; request j owns positions
// [req_off[j], req_off[j+1]).  Each value is tagged with its request in the
// key's high bits, key = j << value_bits | value, so that one stable radix
// sort of the tagged keys (rows = batch positions) orders every request by
// value at once, requests in order.  The WAH encoder then sees a new value
// wherever the request changes and takes rows relative to the request's first
// position, which gives each request exactly its own index.  Finally the one
// lookup table is split per request:
//   key_start[j]   first lookup entry of request j (key_start[nreq] = D),
//   word_start[j]  first word of request j (word_start[nreq] = W),
//   keys[d]        the value (request tag removed),
//   offsets        request j's D_j + 1 offsets, relative to its own words, at
//                  offsets[key_start[j] + j ...]: D + nreq entries in all.
// A batch with a value at or above 2^value_bits is rejected on the device:
// all five outputs get length 0.
#include <algorithm>

#include "common.hpp"

namespace ka {
namespace {

constexpr int kKeyBlock = 256;
constexpr int kKeyItems = 16;  // consecutive values per work-item
constexpr int kSplitBlock = 256;
constexpr uint32_t kSplitGrid = 1024;

__device__ __forceinline__ uint32_t tag_shift_ok(uint32_t value_bits) { return value_bits < 32; }

// key[i] = request(i) << value_bits | values[i]; any value with bits at or
// above value_bits sets *bad.
__global__ __launch_bounds__(kKeyBlock) void k_batch_keys(const uint32_t* __restrict__ values, uint32_t n,
                                                          const uint32_t* __restrict__ req_off, uint32_t nreq,
                                                          uint32_t value_bits, uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ bad) {
  const uint64_t i0 = ((uint64_t)blockIdx.x * kKeyBlock + threadIdx.x) * kKeyItems;
  if (i0 >= n) return;
  // request of i0: the last j with req_off[j] <= i0 (binary search over [0, nreq))
  uint32_t lo = 0, hi = nreq;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (req_off[mid] <= i0)
      lo = mid;
    else
      hi = mid;
  }
  uint32_t j = lo;
  uint32_t next = j + 1 < nreq ? req_off[j + 1] : n;
  uint32_t over = 0;
  const bool tagged = tag_shift_ok(value_bits);
#pragma unroll
  for (int c = 0; c < kKeyItems; ++c) {
    const uint64_t i = i0 + c;
    if (i < n) {
      while (i >= next && j + 1 < nreq) {  // crossing into the next (possibly empty) requests
        ++j;
        next = j + 1 < nreq ? req_off[j + 1] : n;
      }
      const uint32_t v = values[i];
      over |= tagged ? v >> value_bits : 0u;
      keys[i] = (tagged ? j << value_bits : 0u) | v;
    }
  }
  if (over) *bad = 1u;
}

// key_start[j] = first lookup entry whose request is >= j (lower bound of the
// tag j << value_bits in the sorted tagged keys); word_start[j] = its offset.
__global__ __launch_bounds__(kSplitBlock) void k_batch_starts(const uint32_t* __restrict__ tkeys,
                                                              const uint64_t* __restrict__ d_len_keys,
                                                              const uint32_t* __restrict__ g_off, uint32_t nreq,
                                                              uint32_t value_bits, uint32_t* __restrict__ key_start,
                                                              uint32_t* __restrict__ word_start) {
  const uint32_t D = (uint32_t)*d_len_keys;
  for (uint32_t j = blockIdx.x * kSplitBlock + threadIdx.x; j <= nreq; j += gridDim.x * kSplitBlock) {
    uint32_t lo = 0, hi = D;  // first d in [0, D] with request(d) >= j
    while (lo < hi) {
      const uint32_t mid = (lo + hi) / 2;
      const uint32_t r = tag_shift_ok(value_bits) ? tkeys[mid] >> value_bits : 0u;
      if (r < j)
        lo = mid + 1;
      else
        hi = mid;
    }
    key_start[j] = lo;
    word_start[j] = g_off[lo];  // g_off[D] = W
  }
}

// Per-request tables: strip the tags, rebase the offsets on each request's
// words, add each request's closing offset; set the output lengths (all 0 if
// the batch was rejected).
__global__ __launch_bounds__(kSplitBlock) void k_batch_tables(
    uint32_t* __restrict__ keys, const uint32_t* __restrict__ g_off, uint32_t nreq, uint32_t value_bits,
    const uint32_t* __restrict__ key_start, const uint32_t* __restrict__ word_start, const uint32_t* __restrict__ bad,
    uint32_t* __restrict__ offsets, uint64_t* __restrict__ len_keys, uint64_t* __restrict__ len_offsets,
    uint64_t* __restrict__ len_words, uint64_t* __restrict__ len_key_start, uint64_t* __restrict__ len_word_start) {
  const uint32_t D = key_start[nreq];
  const uint32_t stride = gridDim.x * kSplitBlock;
  const uint32_t first = blockIdx.x * kSplitBlock + threadIdx.x;
  const bool tagged = tag_shift_ok(value_bits);
  const uint32_t mask = tagged ? (1u << value_bits) - 1u : ~0u;
  for (uint32_t d = first; d < D; d += stride) {
    const uint32_t k = keys[d];
    const uint32_t j = tagged ? k >> value_bits : 0u;
    offsets[d + j] = g_off[d] - word_start[j];
    keys[d] = k & mask;
  }
  for (uint32_t j = first; j < nreq; j += stride) offsets[key_start[j + 1] + j] = word_start[j + 1] - word_start[j];
  if (first == 0) {
    const bool ok = *bad == 0u;
    *len_keys = ok ? D : 0u;
    *len_offsets = ok ? (uint64_t)D + nreq : 0u;
    *len_words = ok ? word_start[nreq] : 0u;
    *len_key_start = ok ? (uint64_t)nreq + 1 : 0u;
    *len_word_start = ok ? (uint64_t)nreq + 1 : 0u;
  }
}

}  // namespace

int launch_wah_batch(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                     uint32_t value_bits, uint32_t* keys, uint32_t* offsets, uint32_t* words, uint32_t* key_start,
                     uint32_t* word_start, uint64_t* len_keys, uint64_t* len_offsets, uint64_t* len_words,
                     uint64_t* len_key_start, uint64_t* len_word_start) {
  if (!req_off || !offsets || !key_start || !word_start || !len_keys || !len_offsets || !len_words || !len_key_start ||
      !len_word_start)
    return env.fail(kErrArg, "wah_index_batch: null buffer");
  if (nreq == 0) return env.fail(kErrArg, "wah_index_batch: no requests");
  if (value_bits == 0 || value_bits > 32) return env.fail(kErrArg, "wah_index_batch: value_bits must be 1..32");
  const uint32_t req_bits = nreq > 1 ? 32u - (uint32_t)__builtin_clz(nreq - 1) : 0u;
  if (value_bits + req_bits > 32)
    return env.fail(kErrArg, "wah_index_batch: value_bits + bits of the request count exceed 32");
  if (n >= (1ull << 30)) return env.fail(kErrArg, "wah_index_batch: n must be below 2^30");
  if (n && (!values || !keys || !words)) return env.fail(kErrArg, "wah_index_batch: null buffer");
  const uint32_t nn = (uint32_t)n;

  uint32_t* bad = static_cast<uint32_t*>(env.scratch(4));
  uint32_t* tkeys = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* skeys = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* srows = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* g_off = static_cast<uint32_t*>(env.scratch(4 * (n + 1)));
  uint64_t* g_len = static_cast<uint64_t*>(env.scratch(8));
  if (!bad || !tkeys || !skeys || !srows || !g_off || !g_len) return env.fail(kErrOom, "wah_index_batch: scratch");
  int rc = launch_fill_u32(env, bad, 1, 0);
  if (rc) return rc;
  if (n) {
    const uint64_t blocks = (n + (uint64_t)kKeyBlock * kKeyItems - 1) / ((uint64_t)kKeyBlock * kKeyItems);
    env.prof_begin("batch_keys");
    k_batch_keys<<<dim3((uint32_t)blocks), dim3(kKeyBlock), 0, env.stream()>>>(values, nn, req_off, nreq, value_bits,
                                                                              tkeys, bad);
    env.prof_end("batch_keys");
    if ((rc = check_launch(env, "batch_keys launch"))) return rc;
    if ((rc = launch_radix_sort_pairs(env, tkeys, nullptr, skeys, srows, n))) return rc;
  }
  // The tagged keys are the encoder's keys; rows become request-relative.
  if ((rc = launch_wah_encode(env, skeys, srows, n, keys, g_off, words, len_keys, g_len, len_words, req_off,
                              value_bits)))
    return rc;
  const uint32_t sgrid = std::min<uint32_t>(kSplitGrid, (nreq + kSplitBlock) / kSplitBlock);
  env.prof_begin("batch_split");
  k_batch_starts<<<dim3(sgrid), dim3(kSplitBlock), 0, env.stream()>>>(keys, len_keys, g_off, nreq, value_bits,
                                                                       key_start, word_start);
  if ((rc = check_launch(env, "batch_starts launch"))) return rc;
  k_batch_tables<<<dim3(kSplitGrid), dim3(kSplitBlock), 0, env.stream()>>>(
      keys, g_off, nreq, value_bits, key_start, word_start, bad, offsets, len_keys, len_offsets, len_words,
      len_key_start, len_word_start);
  env.prof_end("batch_split");
  return check_launch(env, "batch_tables launch");
}

}  // namespace ka
