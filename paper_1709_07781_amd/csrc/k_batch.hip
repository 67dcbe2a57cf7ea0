// Batched WAH index build: many independent requests in one pass of the
// pipeline (Sec. 3.6 names nesting data parallelism inside a kernel as an
// alternative level of composition to one actor per stage; Sec. 4 is the
// per-request index).
//
// The requests' values are concatenated; request j owns positions
// [req_off[j], req_off[j+1]).  With values of at most 16 bits the segmented
// sort (k_sort.hip) orders every request by value inside its own positions,
// with rows relative to the request, and writes each key tagged with its
// request, key = j << value_bits | value.  Wider values are tagged first and
// one stable radix sort of the tagged keys (rows = batch positions) orders
// every request by value at once, requests in order.  The WAH encoder then
// sees a new value wherever the request changes (and, after the tagged sort,
// takes rows relative to the request's first position), which gives each
// request exactly its own index.  Finally the one lookup table is split per
// request:
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
constexpr int kKeyVecs = 4;                        // 16-byte vectors per work-item
constexpr int kKeyTile = kKeyBlock * kKeyVecs * 4;  // 4096 values
constexpr int kKeyReqs = 1024;                     // requests per tile searched in LDS
constexpr int kSplitBlock = 256;
constexpr uint32_t kSplitGrid = 1024;

__device__ __forceinline__ uint32_t tag_shift_ok(uint32_t value_bits) { return value_bits < 32; }

// Last j in [lo, hi) with off[j] <= i, given off[lo] <= i (binary search).
template <typename T>
__device__ __forceinline__ uint32_t request_of(const T* off, uint32_t lo, uint32_t hi, uint64_t i) {
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Per-value maps that need the request of each value.
// key = request << value_bits | value; a value with bits at or above
// value_bits is flagged, and only its low value_bits bits enter the key, so the
// request field of every key stays below nreq even in a rejected batch.
// With req_bad, a value at or above 2^value_bits flags its own request
// (req_bad[j] = 1) instead of the whole batch; either way the tag keeps only
// the value bits, so the other requests' keys and results are untouched.
struct TagOp {
  uint32_t value_bits;
  uint32_t* req_bad;
  __device__ __forceinline__ uint32_t operator()(uint32_t v, uint32_t j, uint32_t& over) const {
    if (!tag_shift_ok(value_bits)) return v;
    const uint32_t hi = v >> value_bits;
    if (req_bad) {
      if (hi) req_bad[j] = 1u;
    } else {
      over |= hi;
    }
    return j << value_bits | (v & ((1u << value_bits) - 1u));
  }
};
struct RebaseOp {  // a batch-wide exclusive scan minus its value at the request's first position
  const uint32_t* base;
  __device__ __forceinline__ uint32_t operator()(uint32_t v, uint32_t j, uint32_t&) const { return v - base[j]; }
};

// out[i] = op(in[i], request(i)) over tiles of kKeyTile values (16-byte loads
// and stores; in == out is allowed).  The tile's requests j0..j1 are found
// once; when there are at most kKeyReqs of them their boundaries are searched
// in LDS.  Any `over` bit an op reports sets *bad.
template <class Op>
__global__ __launch_bounds__(kKeyBlock) void k_batch_map(const uint32_t* in, uint32_t* out, uint32_t n_cap,
                                                         const uint32_t* __restrict__ req_off, uint32_t nreq, Op op,
                                                         uint32_t* __restrict__ bad,
                                                         const uint64_t* __restrict__ d_n = nullptr) {
  __shared__ uint32_t s_off[kKeyReqs + 1];
  __shared__ uint32_t s_j[2];
  const uint32_t tid = threadIdx.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * kKeyTile;
  const uint32_t n = (uint32_t)device_count(n_cap, d_n);  // the count on the device: tiles past it leave
  if (b0 >= n) return;
  const uint32_t len = (uint32_t)min((uint64_t)kKeyTile, n - b0);
  if (tid < 2) s_j[tid] = request_of(req_off, 0, nreq, tid == 0 ? b0 : b0 + len - 1);
  __syncthreads();
  const uint32_t j0 = s_j[0], cnt = s_j[1] - j0 + 1;  // requests met by this tile
  const bool local = cnt <= (uint32_t)kKeyReqs;
  if (local)
    for (uint32_t k = tid; k <= cnt; k += kKeyBlock) s_off[k] = j0 + k < nreq ? req_off[j0 + k] : n;
  __syncthreads();
  const bool vec = len == (uint32_t)kKeyTile &&
                   ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
  uint32_t over = 0;
#pragma unroll
  for (int r = 0; r < kKeyVecs; ++r) {
    const uint32_t e = 4 * (r * kKeyBlock + tid);  // tile-local index of this vector's first value
    uint32_t v[4], k[4];
    if (vec) {
      const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(in + b0 + e));
      v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] = e + c < len ? in[b0 + e + c] : 0u;
    }
    // request of the vector's first value; the others may cross into later requests
    uint32_t j = e < len ? (local ? j0 + request_of(s_off, 0, cnt, b0 + e) : request_of(req_off, j0, nreq, b0 + e))
                         : 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      k[c] = 0;
      if (e + c < len) {
        for (;;) {  // advance past requests that end before this value (empty ones included)
          if (j + 1 >= nreq || (local && j + 1 - j0 > cnt)) break;
          const uint32_t next = local ? s_off[j + 1 - j0] : req_off[j + 1];
          if (b0 + e + c < next) break;
          ++j;
        }
        k[c] = op(v[c], j, over);
      }
    }
    if (vec) {
      u32x4 q;
      q.x = k[0], q.y = k[1], q.z = k[2], q.w = k[3];
      __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(out + b0 + e));
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (e + c < len) out[b0 + e + c] = k[c];
    }
  }
  if (over && bad) *bad = 1u;
}

// base[j] = scan[req_off[j]] for every non-empty request.
__global__ __launch_bounds__(kSplitBlock) void k_batch_bases(const uint32_t* __restrict__ scan, uint32_t n,
                                                             const uint32_t* __restrict__ req_off, uint32_t nreq,
                                                             uint32_t* __restrict__ base) {
  for (uint32_t j = blockIdx.x * kSplitBlock + threadIdx.x; j < nreq; j += gridDim.x * kSplitBlock)
    base[j] = req_off[j] < n ? scan[req_off[j]] : 0u;
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

// ---------------------------------------------------------------------------------
// Small requests: one persistent launch, one request at a time per work-group
// ---------------------------------------------------------------------------------
// When every request holds at most kSmallMax values and values fit in
// 32 - kSmallRowBits bits, the whole batch is one persistent launch,
// k_small_fused: each work-group takes the next request in order from a
// ticket counter and
//   * sorts value << kSmallRowBits | row in LDS (a bitonic sort; the row bits
//     make equal values keep their order) and marks value, group and fill
//     heads as the encoder does (Sec. 4.1 parts 3-5);
//   * publishes the request's word and value counts, and finds those of all
//     earlier requests by decoupled look-back over the requests' status words;
//   * writes its words, keys and offsets straight to their places and its
//     key_start / word_start entries.
// Tickets are taken in order by running work-groups only, so every request a
// work-group waits for is held by a running work-group that waits only for
// earlier ones: the look-back needs no fallback.  A request with a value at
// or above 2^value_bits (or above kSmallMax values) sets the batch's flag;
// the request that finishes the batch (the last ticket) writes the totals
// and, after the look-back has seen every earlier request, the lengths (all 0
// for a rejected batch).
constexpr int kSmallMax = 1024;
constexpr uint32_t kSmallRowBits = 10;
constexpr int kSmallBlock = 256;
constexpr int kSmallPer = kSmallMax / kSmallBlock;  // consecutive sorted elements per work-item
constexpr uint32_t kSmallRows = 31, kSmallFill = 0x80000000u;
constexpr uint32_t kSmallGrid = 2048;               // persistent work-groups (8 per CU)
static_assert((1 << kSmallRowBits) == kSmallMax, "row bits cover a request");

__global__ __launch_bounds__(kSmallBlock) void k_small_fused(
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ req_off, uint32_t nreq, uint32_t value_bits,
    uint32_t* __restrict__ ticket, uint64_t* __restrict__ status, uint32_t* __restrict__ bad_flag,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ offsets,
    uint32_t* __restrict__ words, uint32_t* __restrict__ key_start, uint32_t* __restrict__ word_start,
    uint64_t* __restrict__ len_keys, uint64_t* __restrict__ len_offsets, uint64_t* __restrict__ len_words,
    uint64_t* __restrict__ len_key_start, uint64_t* __restrict__ len_word_start) {
  __shared__ uint32_t s[kSmallMax];
  __shared__ uint32_t s_scan[kSmallBlock / 64];
  __shared__ uint32_t s_j, s_pre[2];
  const uint32_t tid = threadIdx.x;
  for (;;) {
    if (tid == 0) s_j = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t j = s_j;
    if (j >= nreq) break;  // uniform over the work-group
    const uint32_t b = req_off[j];
    // A request above kSmallMax (a wrong size hint) is rejected like an
    // out-of-range value; only its first kSmallMax values are touched.
    const uint32_t n_req = req_off[j + 1] - b;
    const uint32_t n = min(n_req, (uint32_t)kSmallMax);
    uint32_t over = n_req > (uint32_t)kSmallMax ? 1u : 0u;
#pragma unroll
    for (int q = 0; q < kSmallPer; ++q) {
      const uint32_t i = q * kSmallBlock + tid;
      uint32_t c = 0xFFFFFFFFu;  // padding sorts last
      if (i < n) {
        const uint32_t v = values[b + i];
        over |= v >> value_bits;  // value_bits <= 32 - kSmallRowBits here
        c = (v << kSmallRowBits) | i;
      }
      s[i] = c;
    }
    const bool bad = __syncthreads_or(over != 0u);
    // bitonic sort of the first m = 2^ceil(log2 n) entries, ascending
    uint32_t m = 1;
    while (m < n) m <<= 1;
    for (uint32_t k = 2; k <= m; k <<= 1) {
      for (uint32_t h = k >> 1; h > 0; h >>= 1) {
        for (uint32_t i = tid; i < m; i += kSmallBlock) {
          const uint32_t l = i ^ h;
          if (l > i) {
            const uint32_t x = s[i], y = s[l];
            if ((x > y) == ((i & k) == 0u)) {
              s[i] = y;
              s[l] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    // heads of values, groups and fills, as in the encoder
    const uint32_t e0 = tid * kSmallPer;
    uint32_t heads = 0, segs = 0, gaps = 0;
#pragma unroll
    for (int q = 0; q < kSmallPer; ++q) {
      const uint32_t i = e0 + q;
      if (i < n) {
        const uint32_t c = s[i], v = c >> kSmallRowBits, ch = (c & (kSmallMax - 1)) / kSmallRows;
        bool seg = true, grp = true, gap = ch != 0u;
        if (i > 0) {
          const uint32_t p = s[i - 1], pv = p >> kSmallRowBits, pch = (p & (kSmallMax - 1)) / kSmallRows;
          seg = v != pv;
          grp = seg || ch != pch;
          gap = grp && (seg ? ch != 0u : ch != pch + 1u);
        }
        heads |= (uint32_t)grp << q;
        segs |= (uint32_t)seg << q;
        gaps |= (uint32_t)gap << q;
      }
    }
    const uint32_t nw = (uint32_t)__popc(heads) + (uint32_t)__popc(gaps), ns = (uint32_t)__popc(segs);
    uint32_t total;
    const uint32_t pre = block_excl_scan<kSmallBlock>((ns << 16) | nw, s_scan, &total);
    const uint32_t W = total & 0xFFFFu, D = total >> 16;
    // publish this request's counts, then the look-back for the earlier ones
    if (tid == 0) {
      if (bad) {
        atomicOr(bad_flag, 1u);
        __threadfence();  // the flag is visible before the counts that follow it
      }
      lb_publish_raw(status + kLbSpread * j, lb_pack_pair(W, D, j == 0 ? kLbInclusive : kLbAggregate));
    }
    if (tid < 64) {
      LbPairSum p{0u, 0u};
      if (j > 0) {
        p = lb_lookback_ticket<kLbSpread>(status, j, LbPair{});
        if (tid == 0) lb_publish_raw(status + kLbSpread * j, lb_pack_pair(p.a + W, p.b + D, kLbInclusive));
      }
      if (tid == 0) {
        s_pre[0] = p.a;
        s_pre[1] = p.b;
      }
    }
    __syncthreads();
    const uint32_t wpre = s_pre[0], dpre = s_pre[1];
    uint32_t w = wpre + (pre & 0xFFFFu), d = dpre + (pre >> 16);
#pragma unroll
    for (int q = 0; q < kSmallPer; ++q) {
      if (!((heads >> q) & 1u)) continue;
      const uint32_t i = e0 + q;
      const uint32_t c = s[i], v = c >> kSmallRowBits, ch = (c & (kSmallMax - 1)) / kSmallRows;
      const bool seg = (segs >> q) & 1u;
      if (seg) {
        keys[d] = v;
        offsets[d + j] = w - wpre;  // relative to the request's own words
        ++d;
      }
      if ((gaps >> q) & 1u) {
        const uint32_t pch = seg ? 0u : (s[i - 1] & (kSmallMax - 1)) / kSmallRows;
        words[w++] = kSmallFill | (seg ? ch : ch - pch - 1u);
      }
      // the literal: the bits of the group's rows (at most 31 elements)
      uint32_t lit = 0;
      for (uint32_t t = i; t < n; ++t) {
        const uint32_t ct = s[t];
        const uint32_t rt = ct & (kSmallMax - 1);
        if ((ct >> kSmallRowBits) != v || rt / kSmallRows != ch) break;
        lit |= 1u << (rt - ch * kSmallRows);
      }
      words[w++] = lit;
    }
    if (tid == 0) {
      offsets[dpre + D + j] = W;
      key_start[j] = dpre;
      word_start[j] = wpre;
      if (j == nreq - 1) {  // every earlier request is accounted for
        key_start[nreq] = dpre + D;
        word_start[nreq] = wpre + W;
        __threadfence();
        const bool rejected = __hip_atomic_load(bad_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
        *len_keys = rejected ? 0u : dpre + D;
        *len_offsets = rejected ? 0u : (uint64_t)dpre + D + nreq;
        *len_words = rejected ? 0u : wpre + W;
        *len_key_start = rejected ? 0u : (uint64_t)nreq + 1;
        *len_word_start = rejected ? 0u : (uint64_t)nreq + 1;
      }
    }
    __syncthreads();  // s, s_j and s_pre are reused by the next request
  }
}

// The three-launch form of the small-request path:
//   k_small_index  the fused kernel's sort and heads for request j =
//                  blockIdx.x, its words, keys and offsets into slots bounded
//                  by its size (words at 2 req_off[j], keys at req_off[j],
//                  offsets at req_off[j] + j), and its counts and flag;
//   k_small_starts scans the counts into key_start and word_start and sets the
//                  output lengths (all 0 if a value was out of range);
//   k_small_place  copies each request's slots to their places.
// Every work-group is independent and the placement waits for a kernel
// boundary instead of a look-back, at the price of the slots' extra traffic.
__global__ __launch_bounds__(kSmallBlock) void k_small_index(const uint32_t* __restrict__ values,
                                                             const uint32_t* __restrict__ req_off,
                                                             uint32_t value_bits, uint32_t* __restrict__ wslot,
                                                             uint32_t* __restrict__ kslot,
                                                             uint32_t* __restrict__ oslot,
                                                             uint32_t* __restrict__ counts) {
  __shared__ uint32_t s[kSmallMax];
  __shared__ uint32_t s_scan[kSmallBlock / 64];
  const uint32_t j = blockIdx.x, tid = threadIdx.x;
  const uint32_t b = req_off[j];
  // A request above kSmallMax (a wrong size hint) fails the batch like an
  // out-of-range value; only its first kSmallMax values are touched.
  const uint32_t n_req = req_off[j + 1] - b;
  const uint32_t n = min(n_req, (uint32_t)kSmallMax);
  uint32_t over = n_req > (uint32_t)kSmallMax ? 1u : 0u;
#pragma unroll
  for (int q = 0; q < kSmallPer; ++q) {
    const uint32_t i = q * kSmallBlock + tid;
    uint32_t c = 0xFFFFFFFFu;  // padding sorts last
    if (i < n) {
      const uint32_t v = values[b + i];
      over |= v >> value_bits;  // value_bits <= 32 - kSmallRowBits here
      c = (v << kSmallRowBits) | i;
    }
    s[i] = c;
  }
  const bool bad = __syncthreads_or(over != 0u);
  // bitonic sort of the first m = 2^ceil(log2 n) entries, ascending
  uint32_t m = 1;
  while (m < n) m <<= 1;
  for (uint32_t k = 2; k <= m; k <<= 1) {
    for (uint32_t h = k >> 1; h > 0; h >>= 1) {
      for (uint32_t i = tid; i < m; i += kSmallBlock) {
        const uint32_t l = i ^ h;
        if (l > i) {
          const uint32_t x = s[i], y = s[l];
          if ((x > y) == ((i & k) == 0u)) {
            s[i] = y;
            s[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // heads of values, groups and fills, as in the encoder (Sec. 4.1 parts 3-5)
  const uint32_t e0 = tid * kSmallPer;
  uint32_t heads = 0, segs = 0, gaps = 0;
#pragma unroll
  for (int q = 0; q < kSmallPer; ++q) {
    const uint32_t i = e0 + q;
    if (i < n) {
      const uint32_t c = s[i], v = c >> kSmallRowBits, ch = (c & (kSmallMax - 1)) / kSmallRows;
      bool seg = true, grp = true, gap = ch != 0u;
      if (i > 0) {
        const uint32_t p = s[i - 1], pv = p >> kSmallRowBits, pch = (p & (kSmallMax - 1)) / kSmallRows;
        seg = v != pv;
        grp = seg || ch != pch;
        gap = grp && (seg ? ch != 0u : ch != pch + 1u);
      }
      heads |= (uint32_t)grp << q;
      segs |= (uint32_t)seg << q;
      gaps |= (uint32_t)gap << q;
    }
  }
  const uint32_t nw = (uint32_t)__popc(heads) + (uint32_t)__popc(gaps), ns = (uint32_t)__popc(segs);
  uint32_t total;
  const uint32_t pre = block_excl_scan<kSmallBlock>((ns << 16) | nw, s_scan, &total);
  const uint32_t W = total & 0xFFFFu, D = total >> 16;
  uint32_t w = pre & 0xFFFFu, d = pre >> 16;
  uint32_t* ws = wslot + 2ull * b;
  uint32_t* ks = kslot + b;
  uint32_t* os = oslot + b + j;
#pragma unroll
  for (int q = 0; q < kSmallPer; ++q) {
    if (!((heads >> q) & 1u)) continue;
    const uint32_t i = e0 + q;
    const uint32_t c = s[i], v = c >> kSmallRowBits, ch = (c & (kSmallMax - 1)) / kSmallRows;
    const bool seg = (segs >> q) & 1u;
    if (seg) {
      ks[d] = v;
      os[d] = w;
      ++d;
    }
    if ((gaps >> q) & 1u) {
      const uint32_t pch = seg ? 0u : (s[i - 1] & (kSmallMax - 1)) / kSmallRows;
      ws[w++] = kSmallFill | (seg ? ch : ch - pch - 1u);
    }
    // the literal: the bits of the group's rows (at most 31 elements)
    uint32_t lit = 0;
    for (uint32_t t = i; t < n; ++t) {
      const uint32_t ct = s[t];
      const uint32_t rt = ct & (kSmallMax - 1);
      if ((ct >> kSmallRowBits) != v || rt / kSmallRows != ch) break;
      lit |= 1u << (rt - ch * kSmallRows);
    }
    ws[w++] = lit;
  }
  if (tid == 0) {
    os[D] = W;
    counts[3 * j] = W;
    counts[3 * j + 1] = D;
    counts[3 * j + 2] = bad ? 1u : 0u;
  }
}

constexpr int kStartsBlock = 1024;
__global__ __launch_bounds__(kStartsBlock) void k_small_starts(const uint32_t* __restrict__ counts, uint32_t nreq,
                                                               uint32_t* __restrict__ key_start,
                                                               uint32_t* __restrict__ word_start,
                                                               uint64_t* __restrict__ len_keys,
                                                               uint64_t* __restrict__ len_offsets,
                                                               uint64_t* __restrict__ len_words,
                                                               uint64_t* __restrict__ len_key_start,
                                                               uint64_t* __restrict__ len_word_start,
                                                               uint32_t* __restrict__ req_bad) {
  __shared__ uint32_t s_a[kStartsBlock / 64], s_b[kStartsBlock / 64];
  uint32_t wbase = 0, dbase = 0, any_bad = 0;
  for (uint32_t c0 = 0; c0 < nreq; c0 += kStartsBlock) {
    const uint32_t j = c0 + threadIdx.x;
    const bool ok = j < nreq;
    const uint32_t wj = ok ? counts[3 * j] : 0u, dj = ok ? counts[3 * j + 1] : 0u;
    if (req_bad) {  // per-request rejection: the batch's lengths stand
      if (ok) req_bad[j] = counts[3 * j + 2];
    } else {
      any_bad |= ok ? counts[3 * j + 2] : 0u;
    }
    uint32_t wt, dt;
    const uint32_t wp = block_excl_scan<kStartsBlock>(wj, s_a, &wt);
    const uint32_t dp = block_excl_scan<kStartsBlock>(dj, s_b, &dt);
    if (ok) {
      word_start[j] = wbase + wp;
      key_start[j] = dbase + dp;
    }
    wbase += wt;
    dbase += dt;
    __syncthreads();  // s_a, s_b are reused by the next chunk
  }
  const bool bad = __syncthreads_or(any_bad != 0u);
  if (threadIdx.x == 0) {
    word_start[nreq] = wbase;
    key_start[nreq] = dbase;
    *len_keys = bad ? 0u : dbase;
    *len_offsets = bad ? 0u : (uint64_t)dbase + nreq;
    *len_words = bad ? 0u : wbase;
    *len_key_start = bad ? 0u : (uint64_t)nreq + 1;
    *len_word_start = bad ? 0u : (uint64_t)nreq + 1;
  }
}

__global__ __launch_bounds__(kSmallBlock) void k_small_place(const uint32_t* __restrict__ counts,
                                                             const uint32_t* __restrict__ req_off,
                                                             const uint32_t* __restrict__ wslot,
                                                             const uint32_t* __restrict__ kslot,
                                                             const uint32_t* __restrict__ oslot,
                                                             const uint32_t* __restrict__ key_start,
                                                             const uint32_t* __restrict__ word_start,
                                                             uint32_t* __restrict__ keys, uint32_t* __restrict__ offsets,
                                                             uint32_t* __restrict__ words) {
  const uint32_t j = blockIdx.x, tid = threadIdx.x;
  const uint32_t b = req_off[j], W = counts[3 * j], D = counts[3 * j + 1];
  const uint32_t wd = word_start[j], kd = key_start[j];
  for (uint32_t i = tid; i < W; i += kSmallBlock) words[wd + i] = wslot[2ull * b + i];
  for (uint32_t i = tid; i < D; i += kSmallBlock) keys[kd + i] = kslot[b + i];
  for (uint32_t i = tid; i <= D; i += kSmallBlock) offsets[kd + j + i] = oslot[b + j + i];
}

}  // namespace

int launch_wah_batch(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                     uint32_t value_bits, uint32_t* keys, uint32_t* offsets, uint32_t* words, uint32_t* key_start,
                     uint32_t* word_start, uint64_t* len_keys, uint64_t* len_offsets, uint64_t* len_words,
                     uint64_t* len_key_start, uint64_t* len_word_start, int sort_shape, uint32_t max_req,
                     uint32_t* req_bad, const uint64_t* d_n) {
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

  // Every request small: the three-launch form, or (sort variant 1, which the
  // autotuner times with the others; not with per-request rejection) the
  // persistent fused launch.
  const bool small = max_req <= (uint32_t)kSmallMax && value_bits <= 32 - kSmallRowBits;
  if (small && (sort_shape != 1 || req_bad)) {
    // every request is small, three launches: one work-group per request, then the placement
    uint32_t* wslot = static_cast<uint32_t*>(env.scratch(8 * (n ? n : 1)));
    uint32_t* kslot = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
    uint32_t* oslot = static_cast<uint32_t*>(env.scratch(4 * (n + nreq)));
    uint32_t* counts = static_cast<uint32_t*>(env.scratch(12ull * nreq));
    if (!wslot || !kslot || !oslot || !counts) return env.fail(kErrOom, "wah_index_batch: scratch");
    env.prof_begin("batch_small_index");
    k_small_index<<<dim3(nreq), dim3(kSmallBlock), 0, env.stream()>>>(values, req_off, value_bits, wslot, kslot,
                                                                       oslot, counts);
    env.prof_end("batch_small_index");
    int rc = check_launch(env, "batch_small_index launch");
    if (rc) return rc;
    env.prof_begin("batch_small_place");
    k_small_starts<<<dim3(1), dim3(kStartsBlock), 0, env.stream()>>>(counts, nreq, key_start, word_start, len_keys,
                                                                      len_offsets, len_words, len_key_start,
                                                                      len_word_start, req_bad);
    if ((rc = check_launch(env, "batch_small_starts launch"))) return rc;
    k_small_place<<<dim3(nreq), dim3(kSmallBlock), 0, env.stream()>>>(counts, req_off, wslot, kslot, oslot,
                                                                       key_start, word_start, keys, offsets, words);
    env.prof_end("batch_small_place");
    return check_launch(env, "batch_small_place launch");
  }

  if (small) {
    // every request is small, variant 1: one persistent launch (after clearing
    // its ticket, flag and status words)
    uint32_t* ticket = static_cast<uint32_t*>(env.scratch(8));
    uint64_t* status = static_cast<uint64_t*>(env.scratch(8ull * kLbSpread * nreq));
    if (!ticket || !status) return env.fail(kErrOom, "wah_index_batch: scratch");
    int rc = launch_fill_u32(env, ticket, 2, 0);  // ticket and batch flag
    if (!rc) rc = launch_fill_u64(env, status, (uint64_t)kLbSpread * nreq, 0);
    if (rc) return rc;
    env.prof_begin("batch_small_fused");
    k_small_fused<<<dim3(std::min<uint32_t>(nreq, kSmallGrid)), dim3(kSmallBlock), 0, env.stream()>>>(
        values, req_off, nreq, value_bits, ticket, status, ticket + 1, keys, offsets, words, key_start,
        word_start, len_keys, len_offsets, len_words, len_key_start, len_word_start);
    env.prof_end("batch_small_fused");
    return check_launch(env, "batch_small_fused launch");
  }

  const bool segmented = value_bits <= 16 && (sort_shape == 0 || sort_shape == 3);
  uint32_t* bad = static_cast<uint32_t*>(env.scratch(4));
  uint32_t* tkeys = segmented ? bad : static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* skeys = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* srows = static_cast<uint32_t*>(env.scratch(4 * (n ? n : 1)));
  uint32_t* g_off = static_cast<uint32_t*>(env.scratch(4 * (n + 1)));
  uint64_t* g_len = static_cast<uint64_t*>(env.scratch(8));
  if (!bad || !tkeys || !skeys || !srows || !g_off || !g_len) return env.fail(kErrOom, "wah_index_batch: scratch");
  int rc = launch_fill_u32(env, bad, 1, 0);
  if (rc) return rc;
  if (req_bad && (rc = launch_fill_u32(env, req_bad, nreq, 0))) return rc;
  // Values of at most 16 bits: the segmented sort orders each request by value
  // in ceil(value_bits / 8) passes over 16-bit keys and makes request-relative
  // rows; wider values: every value tagged with its request in the key's high
  // bits, one sort of the tagged keys over all requests (value_bits + the bits
  // of nreq - 1 passes' worth of digits), rows made relative by the encoder.
  if (n) {
    if (segmented) {
      if ((rc = launch_radix_sort_segments(env, values, n, req_off, nreq, value_bits, skeys, srows, bad, req_bad,
                                           sort_shape != 3)))
        return rc;
    } else {
      const uint64_t blocks = (n + kKeyTile - 1) / kKeyTile;
      env.prof_begin("batch_keys");
      k_batch_map<TagOp><<<dim3((uint32_t)blocks), dim3(kKeyBlock), 0, env.stream()>>>(
          values, tkeys, nn, req_off, nreq, TagOp{value_bits, req_bad}, bad, d_n);
      env.prof_end("batch_keys");
      if ((rc = check_launch(env, "batch_keys launch"))) return rc;
      if ((rc = launch_radix_sort_pairs(env, tkeys, nullptr, skeys, srows, n, sort_shape == 3 ? 0 : sort_shape, d_n)))
        return rc;
    }
  }
  // The tagged keys are the encoder's keys; rows are (or become) request-relative.
  if ((rc = launch_wah_encode(env, skeys, srows, n, keys, g_off, words, len_keys, g_len, len_words,
                              segmented ? nullptr : req_off, segmented ? 32u : value_bits, nullptr, 32u, d_n)))
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

// Exclusive scan of each of nreq requests concatenated in in[0..n): one scan
// of the whole batch, then every value minus the batch scan at its request's
// first position (mod 2^32 the difference is the request's own scan).
int launch_segmented_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* req_off,
                          uint32_t nreq) {
  if (n == 0) return kOk;
  if (!in || !out || !req_off || nreq == 0) return env.fail(kErrArg, "segmented scan: null buffer");
  if (n >= (1ull << 32)) return env.fail(kErrArg, "segmented scan: n must be below 2^32");
  uint32_t* base = static_cast<uint32_t*>(env.scratch(4ull * nreq));
  if (!base) return env.fail(kErrOom, "segmented scan: scratch");
  int rc = launch_exclusive_scan(env, in, out, n, nullptr);
  if (rc) return rc;
  const uint32_t nn = (uint32_t)n;
  const uint32_t sgrid = std::min<uint32_t>(kSplitGrid, (nreq + kSplitBlock - 1) / kSplitBlock);
  env.prof_begin("segment_rebase");
  k_batch_bases<<<dim3(sgrid), dim3(kSplitBlock), 0, env.stream()>>>(out, nn, req_off, nreq, base);
  if ((rc = check_launch(env, "batch_bases launch"))) return rc;
  const uint64_t blocks = (n + kKeyTile - 1) / kKeyTile;
  k_batch_map<RebaseOp><<<dim3((uint32_t)blocks), dim3(kKeyBlock), 0, env.stream()>>>(out, out, nn, req_off, nreq,
                                                                                     RebaseOp{base}, nullptr);
  env.prof_end("segment_rebase");
  return check_launch(env, "batch_map launch");
}

}  // namespace ka
