// Encoder formats over group lists, bitmap decoding, AND / OR of bitmaps and
// lookup by value -- the index in the two other word formats (the paper calls
// fills "homogeneous blocks" compressed into one word, Sec. 4.1, and names
// PLWAH as future work, Sec. 6) and the queries the index is built for (Sec.
// 4.1 keeps a lookup table from values to bitmaps; Sec. 4.2 names interactive
// searches and queries).
//
// A group is (key, chunk id, literal): the 31-row chunk of one value's bitmap
// and its rows as a literal.  Groups sorted by (key, chunk) define the index;
// the encoder turns them into words:
//   paper form  one 0-fill (gap > 0) and one literal per group;
//   canonical   the same, except that a run of full groups (all 31 rows, with
//               consecutive chunk ids, one value) is one 1-fill word (bits 31
//               and 30 set, run length in bits 29..0);
//   PLWAH       canonical with 25-bit fill lengths; a fill absorbs the group
//               right after it when that group differs from the fill's groups
//               in one bit only (one row after a 0-fill, one missing row after
//               a 1-fill): bits 29..25 = 1 + that bit's index.
// What group i emits depends on groups i-1 and i (flags), except for the
// length of a 1-fill (the run's end, found by binary search over the prefix
// count of full groups) and its PLWAH position (the group after the run).  So
// the encoding is: flags per group, prefix sums of words, values and full
// groups (the look-back scan), then each group writes its words.  Group lists
// come from sorted (key, row) pairs (k_group_heads, k_group_write) or from the
// non-empty groups of a dense bitmap (the AND / OR of two decoded bitmaps).
//
// Every count that depends on the data stays on the device; grids are sized
// by capacities and read the true counts there.
#include "common.hpp"

namespace ka {
namespace {

constexpr uint32_t kRows = 31;
constexpr uint32_t kFillBit = 0x80000000u;
constexpr uint32_t kOneBit = 0x40000000u;
constexpr uint32_t kFull = 0x7FFFFFFFu;
constexpr uint32_t kLen30 = 0x3FFFFFFFu;
constexpr uint32_t kPlwahShift = 25;
constexpr uint32_t kLen25 = 0x1FFFFFFu;
constexpr int kBlock = 256;
constexpr uint32_t kMaxGrid = 4096;

enum { kFmtPaper = 0, kFmtCanonical = 1, kFmtPlwah = 2 };

__device__ __forceinline__ uint32_t dev_count(uint64_t cap, const uint64_t* d_n) {
  return (uint32_t)device_count(cap, d_n);
}

uint32_t grid_for(uint64_t cap) {
  const uint64_t g = (cap + kBlock - 1) / kBlock;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, kMaxGrid));
}

// ---------------------------------------------------------------------------------
// groups of sorted (key, row) pairs
// ---------------------------------------------------------------------------------
// head[i] = 1 if pair i starts a group (first pair, new key or new chunk).
template <class KeyT>
__global__ __launch_bounds__(kBlock) void k_group_heads(const KeyT* __restrict__ skeys,
                                                        const uint32_t* __restrict__ srows, uint32_t n_cap,
                                                        const uint64_t* __restrict__ d_n, uint32_t* __restrict__ head) {
  const uint32_t n = dev_count(n_cap, d_n);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    bool h = i == 0;
    if (!h) h = skeys[i] != skeys[i - 1] || srows[i] / kRows != srows[i - 1] / kRows;
    head[i] = h ? 1u : 0u;
  }
}

// Every head writes its group at gpos[i] (the exclusive scan of the heads):
// key, chunk id and the literal of its rows (at most 31 pairs, read ahead).
// The last pair writes the group count.
template <class KeyT>
__global__ __launch_bounds__(kBlock) void k_group_write(const KeyT* __restrict__ skeys,
                                                        const uint32_t* __restrict__ srows, uint32_t n_cap,
                                                        const uint64_t* __restrict__ d_n,
                                                        const uint32_t* __restrict__ head,
                                                        const uint32_t* __restrict__ gpos,
                                                        uint32_t* __restrict__ gkey, uint32_t* __restrict__ gchunk,
                                                        uint32_t* __restrict__ glit, uint64_t* __restrict__ k_len) {
  const uint32_t n = dev_count(n_cap, d_n);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    if (i == n - 1) *k_len = (uint64_t)gpos[i] + head[i];
    if (!head[i]) continue;
    const uint32_t k = skeys[i], c = srows[i] / kRows;
    uint32_t lit = 0;
    for (uint32_t j = i; j < n && j < i + kRows; ++j) {
      const uint32_t r = srows[j];
      if (skeys[j] != k || r / kRows != c) break;
      lit |= 1u << (r - c * kRows);
    }
    const uint32_t g = gpos[i];
    gkey[g] = k;
    gchunk[g] = c;
    glit[g] = lit;
  }
}

// ---------------------------------------------------------------------------------
// the encoder over k groups (gkey null: one bitmap, key 0)
// ---------------------------------------------------------------------------------
struct Groups {
  const uint32_t* key;  // null: all 0
  const uint32_t* chunk;
  const uint32_t* lit;
  __device__ __forceinline__ uint32_t k_of(uint32_t i) const { return key ? key[i] : 0u; }
};

// What group i emits, from groups i-1 and i.
struct GroupFlags {
  bool seg;    // first group of its key
  bool full;   // all 31 rows
  bool fill;   // a 0-fill word precedes it (gap > 0), unless absorbed below
  bool main;   // its literal, or the 1-fill of the run it starts
  uint32_t gap;
  uint32_t words;
};

template <int kFmt>
__device__ __forceinline__ GroupFlags group_flags(const Groups& g, uint32_t i) {
  GroupFlags f;
  const uint32_t lit = g.lit[i], c = g.chunk[i];
  f.seg = i == 0 || g.k_of(i) != g.k_of(i - 1);
  const uint32_t pc = f.seg ? 0u : g.chunk[i - 1];
  f.gap = f.seg ? c : c - pc - 1u;
  f.full = lit == kFull;
  bool skip = false, fold1 = false;
  if (kFmt != kFmtPaper) {
    const bool pfull = !f.seg && pc + 1u == c && g.lit[i - 1] == kFull;  // the previous group ends a full run
    skip = f.full && pfull;                                                // inside the run's 1-fill
    if (kFmt == kFmtPlwah) {
      const uint32_t pop = (uint32_t)__popc(lit);
      skip = skip || (!f.full && pfull && pop == 30u);  // absorbed into the run's 1-fill
      fold1 = !f.full && f.gap > 0u && pop == 1u;       // absorbed into its 0-fill
    }
  }
  f.fill = !skip && f.gap > 0u;
  f.main = !skip && !fold1;
  f.words = (f.fill ? 1u : 0u) + (f.main ? 1u : 0u);
  return f;
}

// words[i], seg[i] and (formats with 1-fills) full[i] per group; a fill length
// beyond the format's field sets *reject.
template <int kFmt>
__global__ __launch_bounds__(kBlock) void k_groups_flags(Groups g, uint64_t cap, const uint64_t* __restrict__ k_len,
                                                         uint32_t* __restrict__ words, uint32_t* __restrict__ segs,
                                                         uint32_t* __restrict__ fulls, uint32_t* __restrict__ reject) {
  const uint32_t k = dev_count(cap, k_len);
  const uint32_t lim = kFmt == kFmtPlwah ? kLen25 : kLen30;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    const GroupFlags f = group_flags<kFmt>(g, i);
    words[i] = f.words;
    segs[i] = f.seg ? 1u : 0u;
    if (kFmt != kFmtPaper) fulls[i] = f.full ? 1u : 0u;
    if (f.fill && f.gap > lim) *reject = 1u;
  }
}

// Groups in the run of full groups that starts at i: the largest L with
// groups i .. i+L-1 of one key, consecutive chunk ids and all full.  The
// predicate is monotone in L (chunk ids increase within a key, so equal
// differences of ids and positions mean consecutive ids; the prefix count of
// full groups, fpos, tells whether all of them are full): exponential then
// binary search.
__device__ __forceinline__ uint32_t run_length(const Groups& g, const uint32_t* __restrict__ fpos,
                                               const uint32_t* __restrict__ fulls, uint32_t k, uint32_t i) {
  const uint32_t key = g.k_of(i), c = g.chunk[i], f0 = fpos[i];
  auto ok = [&](uint32_t L) {  // groups i .. i+L-1 form the run's first L groups
    const uint32_t e = i + L - 1u;
    return e < k && g.k_of(e) == key && g.chunk[e] - c == L - 1u && fpos[e] + fulls[e] - f0 == L;
  };
  uint32_t lo = 1, step = 1;  // ok(lo) holds
  while (ok(lo + step)) {
    lo += step;
    step <<= 1;
  }
  uint32_t hi = lo + step;  // ok(hi) fails
  while (hi - lo > 1u) {
    const uint32_t mid = lo + (hi - lo) / 2u;
    if (ok(mid))
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <int kFmt>
__global__ __launch_bounds__(kBlock) void k_groups_write(Groups g, uint64_t cap, const uint64_t* __restrict__ k_len,
                                                         const uint32_t* __restrict__ wpos,
                                                         const uint32_t* __restrict__ dpos,
                                                         const uint32_t* __restrict__ fpos,
                                                         const uint32_t* __restrict__ fulls,
                                                         const uint32_t* __restrict__ reject,
                                                         uint32_t* __restrict__ out_keys,
                                                         uint32_t* __restrict__ out_offsets,
                                                         uint32_t* __restrict__ out_words,
                                                         uint64_t* __restrict__ len_keys,
                                                         uint64_t* __restrict__ len_offsets,
                                                         uint64_t* __restrict__ len_words) {
  const uint32_t k = dev_count(cap, k_len);
  const uint32_t first = blockIdx.x * kBlock + threadIdx.x;
  if (k == 0) {
    if (first == 0) {
      if (out_offsets) out_offsets[0] = 0;
      if (len_keys) *len_keys = 0;
      if (len_offsets) *len_offsets = 1;
      *len_words = 0;
    }
    return;
  }
  for (uint32_t i = first; i < k; i += gridDim.x * kBlock) {
    const GroupFlags f = group_flags<kFmt>(g, i);
    uint32_t w = wpos[i];
    if (f.seg && out_keys) {
      const uint32_t d = dpos[i];
      out_keys[d] = g.k_of(i);
      out_offsets[d] = w;
    }
    const uint32_t lit = g.lit[i];
    if (f.fill) {
      uint32_t word = kFillBit | f.gap;
      if (kFmt == kFmtPlwah && !f.main) word |= (1u + (uint32_t)__builtin_ctz(lit)) << kPlwahShift;
      out_words[w++] = word;
    }
    if (f.main) {
      if (kFmt != kFmtPaper && f.full) {
        const uint32_t L = run_length(g, fpos, fulls, k, i);
        uint32_t word = kFillBit | kOneBit | L;
        const uint32_t nx = i + L;
        if (kFmt == kFmtPlwah && nx < k && g.k_of(nx) == g.k_of(i) && g.chunk[nx] == g.chunk[i] + L &&
            __popc(g.lit[nx]) == 30)
          word |= (1u + (uint32_t)__builtin_ctz(~g.lit[nx] & kFull)) << kPlwahShift;
        out_words[w] = word;
      } else {
        out_words[w] = lit;
      }
    }
    if (i == k - 1) {  // the last group: totals and lengths
      const uint32_t D = dpos[i] + (f.seg ? 1u : 0u), W = wpos[i] + f.words;
      const bool void_ = reject && *reject;
      if (out_offsets) out_offsets[D] = W;
      if (len_keys) *len_keys = void_ ? 0u : D;
      if (len_offsets) *len_offsets = void_ ? 0u : (uint64_t)D + 1;
      *len_words = void_ ? 0u : W;
    }
  }
}

// ---------------------------------------------------------------------------------
// decoding one bitmap into one 31-bit word per group
// ---------------------------------------------------------------------------------
template <int kFmt>
__device__ __forceinline__ uint32_t word_groups(uint32_t w) {
  if (!(w & kFillBit)) return 1u;
  if (kFmt == kFmtPlwah) return (w & kLen25) + (((w >> kPlwahShift) & 31u) ? 1u : 0u);
  return w & kLen30;
}

template <int kFmt>
__global__ __launch_bounds__(kBlock) void k_decode_counts(const uint32_t* __restrict__ words, uint64_t cap,
                                                          const uint64_t* __restrict__ m_len,
                                                          uint32_t* __restrict__ cnt) {
  const uint32_t m = dev_count(cap, m_len);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < m; i += gridDim.x * kBlock) cnt[i] = word_groups<kFmt>(words[i]);
}

// groups[g] for g < ngroups: the word covering g (binary search over the
// prefix counts), or 0 past the last word; more groups than ngroups sets
// *reject.
template <int kFmt>
__global__ __launch_bounds__(kBlock) void k_decode_expand(const uint32_t* __restrict__ words, uint64_t cap,
                                                          const uint64_t* __restrict__ m_len,
                                                          const uint32_t* __restrict__ start, uint32_t ngroups,
                                                          uint32_t* __restrict__ groups, uint32_t* __restrict__ reject) {
  const uint32_t m = dev_count(cap, m_len);
  const uint64_t total = m ? (uint64_t)start[m - 1] + word_groups<kFmt>(words[m - 1]) : 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0 && total > ngroups && reject) *reject = 1u;
  for (uint32_t gi = blockIdx.x * kBlock + threadIdx.x; gi < ngroups; gi += gridDim.x * kBlock) {
    uint32_t v = 0;
    if (gi < total) {
      uint32_t lo = 0, hi = m;  // the last word with start <= gi
      while (hi - lo > 1u) {
        const uint32_t mid = lo + (hi - lo) / 2u;
        if (start[mid] <= gi)
          lo = mid;
        else
          hi = mid;
      }
      const uint32_t w = words[lo];
      if (!(w & kFillBit)) {
        v = w;
      } else {
        const bool one = (w & kOneBit) != 0u;
        const uint32_t len = kFmt == kFmtPlwah ? (w & kLen25) : (w & kLen30);
        const uint32_t p = kFmt == kFmtPlwah ? (w >> kPlwahShift) & 31u : 0u;
        if (gi - start[lo] < len)
          v = one ? kFull : 0u;
        else  // the absorbed group after the fill
          v = one ? (kFull & ~(1u << (p - 1u))) : (1u << (p - 1u));
      }
    }
    groups[gi] = v;
  }
}

// ---------------------------------------------------------------------------------
// AND / OR of two decoded bitmaps, and the non-empty groups as a group list
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_combine(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                                    uint32_t ngroups, uint32_t op, uint32_t* __restrict__ lit,
                                                    uint32_t* __restrict__ tag) {
  for (uint32_t gi = blockIdx.x * kBlock + threadIdx.x; gi < ngroups; gi += gridDim.x * kBlock) {
    const uint32_t x = op ? (a[gi] | b[gi]) : (a[gi] & b[gi]);
    lit[gi] = x;
    tag[gi] = x ? gi + 1u : 0u;  // compacted below: the non-empty groups' ids + 1, in order
  }
}

__global__ __launch_bounds__(kBlock) void k_nonempty_groups(const uint32_t* __restrict__ tag, uint64_t cap,
                                                            const uint64_t* __restrict__ k_len,
                                                            const uint32_t* __restrict__ dense,
                                                            uint32_t* __restrict__ chunk, uint32_t* __restrict__ lit) {
  const uint32_t k = dev_count(cap, k_len);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    const uint32_t c = tag[i] - 1u;
    chunk[i] = c;
    lit[i] = dense[c];
  }
}

// ---------------------------------------------------------------------------------
// lookup of values in the table
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_lookup(const uint32_t* __restrict__ keys, uint64_t dcap,
                                                   const uint64_t* __restrict__ d_len,
                                                   const uint32_t* __restrict__ queries, uint32_t q_cap,
                                                   const uint64_t* __restrict__ q_len,
                                                   uint32_t* __restrict__ slots) {
  const uint32_t D = dev_count(dcap, d_len), q = dev_count(q_cap, q_len);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < q; i += gridDim.x * kBlock) {
    const uint32_t x = queries[i];
    uint32_t lo = 0, hi = D;  // first key >= x
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2u;
      if (keys[mid] < x)
        lo = mid + 1u;
      else
        hi = mid;
    }
    slots[i] = (lo < D && keys[lo] == x) ? lo : 0xFFFFFFFFu;
  }
}

__global__ void k_set_zero_u32(uint32_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0u;
}

// *reject = 1 if a key is at or above 2^bits (from the OR of all keys).
__global__ void k_reject_above(const uint32_t* __restrict__ keys_or, uint32_t bits, uint32_t* __restrict__ reject) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && bits < 32 && (*keys_or >> bits) != 0u) *reject = 1u;
}

// *len = *reject ? 0 : value.
__global__ void k_len_unless(uint64_t* __restrict__ len, uint64_t value, const uint32_t* __restrict__ reject) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *len = *reject ? 0u : value;
}

// ---- host side --------------------------------------------------------------------------
template <int kFmt>
int encode_groups_fmt(Env& env, const Groups& g, uint64_t cap, const uint64_t* k_len, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* len_keys, uint64_t* len_offsets,
                      uint64_t* len_words, uint32_t* reject) {
  const uint64_t c = std::max<uint64_t>(cap, 1);
  uint32_t* wc = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* sg = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* wp = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* dp = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* fl = kFmt != kFmtPaper ? static_cast<uint32_t*>(env.scratch(4 * c)) : nullptr;
  uint32_t* fp = kFmt != kFmtPaper ? static_cast<uint32_t*>(env.scratch(4 * c)) : nullptr;
  if (!wc || !sg || !wp || !dp || (kFmt != kFmtPaper && (!fl || !fp))) return env.fail(kErrOom, "group encoder: scratch");
  const uint32_t grid = grid_for(c);
  int rc;
  env.prof_begin("groups_flags");
  k_groups_flags<kFmt><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(g, c, k_len, wc, sg, fl, reject);
  env.prof_end("groups_flags");
  if ((rc = check_launch(env, "groups_flags launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, wc, wp, c, k_len))) return rc;
  if ((rc = launch_exclusive_scan(env, sg, dp, c, k_len))) return rc;
  if (kFmt != kFmtPaper && (rc = launch_exclusive_scan(env, fl, fp, c, k_len))) return rc;
  env.prof_begin("groups_write");
  k_groups_write<kFmt><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(g, c, k_len, wp, dp, fp, fl, reject, keys,
                                                                       offsets, words, len_keys, len_offsets,
                                                                       len_words);
  env.prof_end("groups_write");
  return check_launch(env, "groups_write launch");
}

int encode_groups(Env& env, uint32_t fmt, const Groups& g, uint64_t cap, const uint64_t* k_len, uint32_t* keys,
                  uint32_t* offsets, uint32_t* words, uint64_t* len_keys, uint64_t* len_offsets, uint64_t* len_words,
                  uint32_t* reject) {
  switch (fmt) {
    case kFmtPaper:
      return encode_groups_fmt<kFmtPaper>(env, g, cap, k_len, keys, offsets, words, len_keys, len_offsets, len_words,
                                          reject);
    case kFmtCanonical:
      return encode_groups_fmt<kFmtCanonical>(env, g, cap, k_len, keys, offsets, words, len_keys, len_offsets,
                                              len_words, reject);
    case kFmtPlwah:
      return encode_groups_fmt<kFmtPlwah>(env, g, cap, k_len, keys, offsets, words, len_keys, len_offsets, len_words,
                                          reject);
    default:
      return env.fail(kErrArg, "unknown WAH format");
  }
}

}  // namespace

template <class KeyT>
int encode_format_impl(Env& env, const KeyT* skeys, const uint32_t* srows, uint64_t n, uint32_t fmt, uint32_t* keys,
                       uint32_t* offsets, uint32_t* words, uint64_t* len_keys, uint64_t* len_offsets,
                       uint64_t* len_words, uint32_t* reject, const uint64_t* d_n) {
  if (fmt > kFmtPlwah) return env.fail(kErrArg, "unknown WAH format");
  if (!offsets || !len_keys || !len_offsets || !len_words || !reject)
    return env.fail(kErrArg, "wah encoder: null output");
  if (n >= (1ull << 30)) return env.fail(kErrArg, "wah encoder: n must be below 2^30");
  if (n && (!skeys || !srows || !keys || !words)) return env.fail(kErrArg, "wah encoder: null buffer");
  const uint64_t c = std::max<uint64_t>(n, 1);
  uint32_t* head = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* gpos = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* gkey = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* gchunk = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* glit = static_cast<uint32_t*>(env.scratch(4 * c));
  uint64_t* k_len = static_cast<uint64_t*>(env.scratch(8));
  if (!head || !gpos || !gkey || !gchunk || !glit || !k_len) return env.fail(kErrOom, "wah encoder: scratch");
  int rc;
  if ((rc = launch_set_len(env, k_len, 0))) return rc;
  if (n) {
    const uint32_t grid = grid_for(n), nn = (uint32_t)n;
    env.prof_begin("group_heads");
    k_group_heads<KeyT><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(skeys, srows, nn, d_n, head);
    env.prof_end("group_heads");
    if ((rc = check_launch(env, "group_heads launch"))) return rc;
    if ((rc = launch_exclusive_scan(env, head, gpos, n, d_n))) return rc;
    env.prof_begin("group_write");
    k_group_write<KeyT><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(skeys, srows, nn, d_n, head, gpos, gkey,
                                                                       gchunk, glit, k_len);
    env.prof_end("group_write");
    if ((rc = check_launch(env, "group_write launch"))) return rc;
  }
  return encode_groups(env, fmt, Groups{gkey, gchunk, glit}, c, k_len, keys, offsets, words, len_keys, len_offsets,
                       len_words, reject);
}

int launch_wah_encode_format(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t fmt,
                             uint32_t* keys, uint32_t* offsets, uint32_t* words, uint64_t* len_keys,
                             uint64_t* len_offsets, uint64_t* len_words, uint32_t* reject, const uint64_t* d_n) {
  return encode_format_impl(env, skeys, srows, n, fmt, keys, offsets, words, len_keys, len_offsets, len_words,
                            reject, d_n);
}

int launch_wah_encode_format16(Env& env, const uint16_t* skeys, const uint32_t* srows, uint64_t n, uint32_t fmt,
                               uint32_t* keys, uint32_t* offsets, uint32_t* words, uint64_t* len_keys,
                               uint64_t* len_offsets, uint64_t* len_words, uint32_t* reject, const uint64_t* d_n) {
  return encode_format_impl(env, skeys, srows, n, fmt, keys, offsets, words, len_keys, len_offsets, len_words,
                            reject, d_n);
}

int launch_reject_above(Env& env, const uint32_t* keys_or, uint32_t bits, uint32_t* reject) {
  k_reject_above<<<dim3(1), dim3(64), 0, env.stream()>>>(keys_or, bits, reject);
  return check_launch(env, "reject_above launch");
}

int launch_len_unless(Env& env, uint64_t* len, uint64_t value, const uint32_t* reject) {
  k_len_unless<<<dim3(1), dim3(64), 0, env.stream()>>>(len, value, reject);
  return check_launch(env, "len_unless launch");
}

int launch_wah_decode(Env& env, const uint32_t* words, uint64_t m_cap, const uint64_t* m_len, uint32_t fmt,
                      uint32_t ngroups, uint32_t* groups, uint32_t* reject) {
  if (fmt > kFmtPlwah) return env.fail(kErrArg, "unknown WAH format");
  if (!reject || (ngroups && !groups) || (m_cap && !words)) return env.fail(kErrArg, "wah decode: null buffer");
  const uint64_t c = std::max<uint64_t>(m_cap, 1);
  uint32_t* cnt = static_cast<uint32_t*>(env.scratch(4 * c));
  uint32_t* start = static_cast<uint32_t*>(env.scratch(4 * c));
  if (!cnt || !start) return env.fail(kErrOom, "wah decode: scratch");
  int rc;
  const uint32_t gw = grid_for(c), gg = grid_for(ngroups);
  env.prof_begin("wah_decode");
#define KA_DECODE(F)                                                                                              \
  k_decode_counts<F><<<dim3(gw), dim3(kBlock), 0, env.stream()>>>(words, m_cap, m_len, cnt);                      \
  if ((rc = check_launch(env, "decode_counts launch"))) return rc;                                                \
  if ((rc = launch_exclusive_scan(env, cnt, start, m_cap, m_len))) return rc;                                     \
  k_decode_expand<F><<<dim3(gg), dim3(kBlock), 0, env.stream()>>>(words, m_cap, m_len, start, ngroups, groups, \
                                                                  reject);
  if (fmt == kFmtPaper) {
    KA_DECODE(kFmtPaper)
  } else if (fmt == kFmtCanonical) {
    KA_DECODE(kFmtCanonical)
  } else {
    KA_DECODE(kFmtPlwah)
  }
#undef KA_DECODE
  env.prof_end("wah_decode");
  return check_launch(env, "decode_expand launch");
}

int launch_wah_combine(Env& env, const uint32_t* a, uint64_t a_cap, const uint64_t* a_len, const uint32_t* b,
                       uint64_t b_cap, const uint64_t* b_len, uint32_t in_fmt, uint32_t ngroups, uint32_t op,
                       uint32_t out_fmt, uint32_t* words, uint64_t* len_words, uint32_t* reject) {
  if (op > 1) return env.fail(kErrArg, "wah combine: op must be 0 (AND) or 1 (OR)");
  if (in_fmt > kFmtPlwah || out_fmt > kFmtPlwah) return env.fail(kErrArg, "unknown WAH format");
  if (!words || !len_words || !reject) return env.fail(kErrArg, "wah combine: null buffer");
  const uint64_t gc = std::max<uint64_t>(ngroups, 1);
  uint32_t* ga = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* gb = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* lit = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* tag = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* nz = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* chunk = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint32_t* glit = static_cast<uint32_t*>(env.scratch(4 * gc));
  uint64_t* k_len = static_cast<uint64_t*>(env.scratch(8));
  if (!ga || !gb || !lit || !tag || !nz || !chunk || !glit || !k_len) return env.fail(kErrOom, "wah combine: scratch");
  int rc;
  if ((rc = launch_wah_decode(env, a, a_cap, a_len, in_fmt, ngroups, ga, reject))) return rc;
  if ((rc = launch_wah_decode(env, b, b_cap, b_len, in_fmt, ngroups, gb, reject))) return rc;
  const uint32_t gg = grid_for(gc);
  env.prof_begin("wah_combine");
  k_combine<<<dim3(gg), dim3(kBlock), 0, env.stream()>>>(ga, gb, ngroups, op, lit, tag);
  env.prof_end("wah_combine");
  if ((rc = check_launch(env, "combine launch"))) return rc;
  if ((rc = launch_set_len(env, k_len, 0))) return rc;
  if (ngroups && (rc = launch_compact_nonzero(env, tag, nz, ngroups, nullptr, k_len))) return rc;
  k_nonempty_groups<<<dim3(gg), dim3(kBlock), 0, env.stream()>>>(nz, gc, k_len, lit, chunk, glit);
  if ((rc = check_launch(env, "nonempty_groups launch"))) return rc;
  return encode_groups(env, out_fmt, Groups{nullptr, chunk, glit}, gc, k_len, nullptr, nullptr, words, nullptr,
                       nullptr, len_words, reject);
}

int launch_wah_lookup(Env& env, const uint32_t* keys, uint64_t d_cap, const uint64_t* d_len, const uint32_t* queries,
                      uint64_t q, uint32_t* slots, const uint64_t* q_len) {
  if (q == 0) return kOk;
  if (!queries || !slots || (d_cap && !keys)) return env.fail(kErrArg, "wah lookup: null buffer");
  if (q >= (1ull << 32)) return env.fail(kErrArg, "wah lookup: too many queries");
  env.prof_begin("wah_lookup");
  k_lookup<<<dim3(grid_for(q)), dim3(kBlock), 0, env.stream()>>>(keys, d_cap, d_len, queries, (uint32_t)q, q_len,
                                                                         slots);
  env.prof_end("wah_lookup");
  return check_launch(env, "lookup launch");
}

int launch_zero_u32(Env& env, uint32_t* p) {
  k_set_zero_u32<<<dim3(1), dim3(64), 0, env.stream()>>>(p);
  return check_launch(env, "zero launch");
}

}  // namespace ka
