// Stable LSB radix sort of (uint32 key, uint32 row) pairs by key -- parts 1
// and 2 of the WAH index build (Sec. 4.1: tag every value with its input
// position, then sort by value; Sec. 4.2 sorts with a radix sort).
//
// 8-bit digits, up to four passes, each a reduce-then-scan over tiles of
// kTile keys -- no work-group ever waits for another one:
//  * k_radix_upsweep (one work-group per tile) counts the tile's digits into a
//    digit-major table; the pass-0 instance also records the OR and the AND of
//    the tile's keys, from which k_radix_plan forms the sort plan: a pass whose
//    digit is the same in every key (equal in the OR and the AND) is the
//    identity of a stable sort and is skipped, so 16-bit keys cost two passes.
//  * the exclusive scan of the table (the look-back scan kernel, into a
//    second table) turns every count into the output position of the tile's
//    first key with that digit.
//  * k_radix_scatter (one work-group per tile) ranks its keys by digit inside
//    each wave -- the lanes holding the same digit are found by OR-ing each
//    lane's bit into a per-digit mask in LDS (8-bit digits; digits 0 and 1 by a
//    ballot each) or with one ballot per digit bit (narrower digits), and a
//    key's rank is the number of such lanes below it plus the wave's earlier
//    count of that digit, so equal keys keep their order -- reorders the tile by
//    digit in LDS and writes each digit's run to its offset from the table,
//    consecutive work-items writing consecutive addresses.
// Tiles are taken in an XCD-aware order (see xcd_tile).
// The first active pass reads the input (and makes row ids 0..n-1 when no rows
// are given), later ones read the previous active pass's output, and the last
// active pass writes the caller's buffers.
#include <algorithm>
#include <cstddef>
#include <type_traits>

#include "common.hpp"

namespace ka {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kPasses = 32 / kRadixBits;

#ifndef KA_SORT_BLOCK
#define KA_SORT_BLOCK 1024
#endif
#ifndef KA_SORT_ITEMS
#define KA_SORT_ITEMS 8
#endif
#ifndef KA_XCD_MAP
#define KA_XCD_MAP 1
#endif
// Tile shapes (work-items x keys per work-item of the scatter), chosen per
// launch: variant 0 is the default, the others are candidates for autotuning.
// (Persistent scatters that load the next tile into a second register set
// while ranking the current one ran 35-60% slower at every shape: the extra
// registers cost more occupancy than the prefetch saves.)
struct SortShape {
  int block, items;
};
constexpr SortShape kShapes[] = {{KA_SORT_BLOCK, KA_SORT_ITEMS}, {512, 16}, {512, 8}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

}  // namespace

// The sort plan, written by the pass-0 count kernel.
struct SortPlan {
  uint32_t active;               // bit p: pass p moves data
  uint32_t keys_or;              // OR of all keys
  uint64_t scan_len[kPasses];    // entries of pass p's table scan (0 when skipped)
};
static_assert(sizeof(SortPlan) <= kSortPlanBytes, "plan storage");

namespace {

struct PassBuffers {
  const uint32_t* keys_in;
  const uint32_t* rows_in;  // null: rows are positions 0..n-1
  uint32_t* keys_a;         // caller's output (written by the last active pass)
  uint32_t* rows_a;
  uint32_t* keys_b;         // scratch ping-pong buffer
  uint32_t* rows_b;
};

// Source and destination of one pass; keys are uint32, or uint16 in the
// narrow-key sort.
template <class SK, class DK>
struct PassIoT {
  const SK* src_keys;
  const uint32_t* src_rows;
  DK* dst_keys;
  uint32_t* dst_rows;
  bool implicit_rows;
  uint32_t row_origin = 0;  // implicit rows: position - row_origin
  uint32_t key_or = 0;      // keys written as (key & key_and) | key_or (kTag scatters only)
  uint32_t key_and = ~0u;
};
using PassIo = PassIoT<uint32_t, uint32_t>;

// Source and destination of pass `pass` under the plan's active mask: the
// last active pass writes buffer a, the one before it b, and so on.
__device__ __forceinline__ PassIo pass_io(const PassBuffers& buf, uint32_t active, uint32_t pass) {
  const uint32_t later = (uint32_t)__popc(active >> pass);  // active passes from this one on
  const bool first = (active & ((1u << pass) - 1)) == 0;
  PassIo io;
  io.dst_keys = (later & 1u) ? buf.keys_a : buf.keys_b;
  io.dst_rows = (later & 1u) ? buf.rows_a : buf.rows_b;
  io.src_keys = first ? buf.keys_in : (((later + 1) & 1u) ? buf.keys_a : buf.keys_b);
  io.src_rows = first ? buf.rows_in : (((later + 1) & 1u) ? buf.rows_a : buf.rows_b);
  io.implicit_rows = first && buf.rows_in == nullptr;
  return io;
}

// LDS add of 1 to bin d by every active lane, aggregated over lanes that share
// a bin: in each of kRounds rounds the first remaining lane's bin takes the
// count of all remaining lanes with that bin in one add; the lanes left after
// the rounds add 1 each.  One round suits keys in input order (a second round
// in the first pass cost +9 us on Zipf keys); the later passes count in
// registers instead (upsweep_tile with kRounds < 0).
template <int kRounds>
__device__ __forceinline__ void lds_add_aggregated(uint32_t* bins, uint32_t d, bool valid) {
  uint64_t rest = __ballot(valid);
#pragma unroll
  for (int round = 0; round < kRounds; ++round) {
    if (!rest) return;
    const uint32_t first_lane = (uint32_t)__builtin_ctzll(rest);
    const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, (int)first_lane);
    const uint64_t same = __ballot(d == d0) & rest;
    if (lane_id() == first_lane) atomicAdd(&bins[d0], (uint32_t)__popcll(same));
    rest &= ~same;
  }
  if ((rest >> lane_id()) & 1ull) atomicAdd(&bins[d], 1u);
}

// Tile of work-group b under an XCD-aware order.  Work-groups are dispatched
// round-robin over the 8 XCDs (b mod 8), each with its own L2; this gives XCD x
// the contiguous tile range [x*q + min(x, r), ...) of q or q + 1 tiles (q =
// ntiles / 8, r = ntiles mod 8), so neighbouring tiles -- whose output runs meet
// in the same cache lines -- are handled by the same L2.  A bijection on
// [0, ntiles) for every ntiles.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t ntiles) {
#if KA_XCD_MAP
  const uint32_t x = b & 7u, i = b >> 3, q = ntiles >> 3, r = ntiles & 7u;
  return x * q + min(x, r) + i;
#else
  (void)ntiles;
  return b;
#endif
}

// Elements of tile `tile` (kTile each) out of n: n_cap, or the count *d_n
// written on the device by an earlier stage (grids are then sized by the
// capacity and the tiles past the count are empty).
__device__ __forceinline__ uint32_t tile_len(uint32_t tile, uint32_t kTile, uint32_t n_cap, const uint64_t* d_n) {
  const uint32_t n = (uint32_t)device_count(n_cap, d_n), base = tile * kTile;
  return base < n ? min(kTile, n - base) : 0u;
}

// ---------------------------------------------------------------------------------
// upsweep: digit counts of one tile into the digit-major table
// ---------------------------------------------------------------------------------
constexpr int kUpBlock = kRadix;                  // one work-item per digit when the counts are written
constexpr int kUpWaves = kUpBlock / 64;

// table[d * ntiles + tile] = number of keys of the tile with digit d.  The
// exclusive scan of the table in this digit-major order is, entry by entry,
// the position in the pass's output of the tile's first key with digit d.
// All of a work-item's loads are issued before the first key is counted; with
// kOrAnd the OR and the AND of the tile's keys are written too.
// The tile is keys[base, base + len); digit d's count goes to
// table[d * stride + col] (the plan-driven and fixed sorts: stride = tile
// count, col = tile; the segmented sort: its request's part of the table).
template <int kTile, int kRounds, bool kOrAnd, class SK>
__device__ __forceinline__ void upsweep_tile(const SK* __restrict__ keys, uint32_t shift, uint32_t base, uint32_t len,
                                             uint32_t* __restrict__ table, uint64_t col, uint64_t stride,
                                             uint32_t tile, uint32_t* __restrict__ orand,
                                             uint32_t mask = kRadix - 1) {
  constexpr int kUpVecs = kTile / 4 / kUpBlock;  // 4-key loads per work-item
  constexpr uintptr_t kAlign = 15;  // 16-byte loads
  __shared__ uint32_t s_hist[kUpWaves][kRadix];
  __shared__ uint32_t s_or[kUpWaves], s_and[kUpWaves];
  const uint32_t tid = threadIdx.x, w = tid / 64;

  // Key 4 (j * kUpBlock + tid) + c of the tile in k[j][c] (uint16 keys of a full
  // tile: key 8 (j/2 * kUpBlock + tid) + 4 (j mod 2) + c).
  uint32_t k[kUpVecs][4];
  if (len == (uint32_t)kTile && (reinterpret_cast<uintptr_t>(keys + base) & kAlign) == 0) {
    if (sizeof(SK) == 2) {
      // uint16 keys: 8 per 16-byte load (which keys a work-item holds does not
      // change the counts); half the loads of 8-byte ones: 40.5 -> 35.9 us for
      // the second pass over 2^26 keys
      static_assert(kUpVecs % 2 == 0, "pairs of 4-key groups");
#pragma unroll
      for (int j = 0; j < kUpVecs / 2; ++j) {
        const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(keys + base) + j * kUpBlock + tid);
        k[2 * j][0] = a.x & 0xFFFFu, k[2 * j][1] = a.x >> 16, k[2 * j][2] = a.y & 0xFFFFu, k[2 * j][3] = a.y >> 16;
        k[2 * j + 1][0] = a.z & 0xFFFFu, k[2 * j + 1][1] = a.z >> 16;
        k[2 * j + 1][2] = a.w & 0xFFFFu, k[2 * j + 1][3] = a.w >> 16;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kUpVecs; ++j) load_key4(keys + base, (uint64_t)j * kUpBlock + tid, k[j]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < kUpVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t e = 4 * (j * kUpBlock + tid) + c;
        k[j][c] = e < len ? (uint32_t)keys[base + e] : 0u;
      }
  }
  for (int i = tid; i < kUpWaves * kRadix; i += kUpBlock) (&s_hist[0][0])[i] = 0;
  __syncthreads();
  uint32_t kor = 0, kand = ~0u;
  // kRounds < 0: two digits are counted in registers -- 0 and the digit of the
  // wave's first key -- and every other key adds 1 in LDS.  After the first
  // pass of an LSD sort a tile's keys share their low digit and the next digit
  // is concentrated in few values, the most often 0 for small values or else
  // likely the first key's; the aggregated adds' ballots and lane reads cost
  // more there (measured on 16-bit Zipf keys: 62 -> 42 us; uniform keys 51 ->
  // 44 us).
  uint32_t c0 = 0, ch = 0;
  const uint32_t hot = (uint32_t)__builtin_amdgcn_readfirstlane((int)((k[0][0] >> shift) & mask));
#pragma unroll
  for (int j = 0; j < kUpVecs; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const bool valid = 4 * (j * kUpBlock + tid) + c < len;
      if (kRounds < 0) {
        const uint32_t d = (k[j][c] >> shift) & mask;
        if (valid) {
          if (d == hot)
            ++ch;
          else if (d == 0)
            ++c0;
          else
            atomicAdd(&s_hist[w][d], 1u);
        }
      } else {
        lds_add_aggregated<(kRounds < 0 ? 0 : kRounds)>(s_hist[w], (k[j][c] >> shift) & mask, valid);
      }
      if (kOrAnd && valid) {
        kor |= k[j][c];
        kand &= k[j][c];
      }
    }
  if (kRounds < 0) {
    const uint32_t z = wave_sum(c0), h = wave_sum(ch);
    if (lane_id() == 0) {
      if (z) atomicAdd(&s_hist[w][0], z);
      if (h) atomicAdd(&s_hist[w][hot], h);
    }
  }
  if (kOrAnd) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      kor |= (uint32_t)__shfl_xor((int)kor, off);
      kand &= (uint32_t)__shfl_xor((int)kand, off);
    }
    if (lane_id() == 0) {
      s_or[w] = kor;
      s_and[w] = kand;
    }
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int ww = 0; ww < kUpWaves; ++ww) c += s_hist[ww][tid];
  table[(uint64_t)tid * stride + col] = c;
  if (kOrAnd && tid == 0) {
    uint32_t o = 0, a = ~0u;
#pragma unroll
    for (int ww = 0; ww < kUpWaves; ++ww) {
      o |= s_or[ww];
      a &= s_and[ww];
    }
    orand[2 * tile] = o;
    orand[2 * tile + 1] = a;
  }
}

// Plan-driven upsweep of pass `pass`; the pass-0 instance also writes the OR
// and the AND of the tile's keys for the plan.
template <bool kFirst, int kTile>
__global__ __launch_bounds__(kUpBlock) void k_radix_upsweep(PassBuffers buf, const SortPlan* __restrict__ plan,
                                                            uint32_t* __restrict__ table, uint32_t* __restrict__ orand,
                                                            uint32_t pass, uint32_t n_cap, uint32_t ntiles,
                                                            const uint64_t* __restrict__ d_n) {
  const uint32_t* keys = buf.keys_in;
  if (!kFirst) {
    const uint32_t active = plan->active;
    if (!((active >> pass) & 1u)) return;  // uniform over the grid
    keys = pass_io(buf, active, pass).src_keys;
  }
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  upsweep_tile<kTile, kFirst ? 1 : -1, kFirst>(keys, pass * kRadixBits, tile * kTile, tile_len(tile, kTile, n_cap, d_n),
                                              table, tile, ntiles, tile, orand);
}

// Upsweep of a fixed pass (no plan) over uint32 or uint16 keys.  Work-group 0
// of the first pass clears *reject.
template <int kTile, int kRounds, class SK>
__global__ __launch_bounds__(kUpBlock) void k_radix_count(const SK* __restrict__ keys, uint32_t* __restrict__ table,
                                                          uint32_t shift, uint32_t mask, uint32_t n_cap,
                                                          uint32_t ntiles, uint32_t* __restrict__ reject,
                                                          const uint64_t* __restrict__ d_n) {
  if (reject && blockIdx.x == 0 && threadIdx.x == 0) *reject = 0u;
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  upsweep_tile<kTile, kRounds, false>(keys, shift, tile * kTile, tile_len(tile, kTile, n_cap, d_n), table, tile,
                                      ntiles, tile, nullptr, mask);
}

// The sort plan from the OR and the AND of every tile's keys: a pass moves
// data unless its digit is the same in every key, i.e. the same in the OR and
// the AND.  Also the length of each pass's table scan: the full table for an
// active pass, 0 (nothing to scan) for a skipped one.  One work-group.
constexpr int kPlanBlock = 1024;
__global__ __launch_bounds__(kPlanBlock) void k_radix_plan(const uint32_t* __restrict__ orand, uint32_t ntiles,
                                                           SortPlan* __restrict__ plan) {
  __shared__ uint32_t s_or[kPlanBlock / 64], s_and[kPlanBlock / 64];
  uint32_t o = 0, a = ~0u;
  for (uint32_t t = threadIdx.x; t < ntiles; t += kPlanBlock) {
    o |= orand[2 * t];
    a &= orand[2 * t + 1];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    o |= (uint32_t)__shfl_xor((int)o, off);
    a &= (uint32_t)__shfl_xor((int)a, off);
  }
  if (lane_id() == 0) {
    s_or[threadIdx.x / 64] = o;
    s_and[threadIdx.x / 64] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int ww = 1; ww < kPlanBlock / 64; ++ww) {
      o |= s_or[ww];
      a &= s_and[ww];
    }
    const uint32_t diff = o ^ a;
    uint32_t act = 0;
    for (int p = 0; p < kPasses; ++p)
      if ((diff >> (p * kRadixBits)) & (kRadix - 1)) act |= 1u << p;
    if (act == 0) act = 1u << (kPasses - 1);  // all keys equal: one pass still moves them
    plan->active = act;
    plan->keys_or = o;
    for (int p = 0; p < kPasses; ++p) plan->scan_len[p] = ((act >> p) & 1u) ? (uint64_t)ntiles * kRadix : 0u;
  }
}

// ---------------------------------------------------------------------------------
// scatter: one tile, ranked in LDS, written to its offsets
// ---------------------------------------------------------------------------------
// Bit B of d spread over the word: 0 or ~0 (one v_bfe_i32; the compiler
// otherwise emits a shift pair).
template <int B>
__device__ __forceinline__ uint32_t spread_bit(uint32_t d) {
  uint32_t s;
  asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(s) : "v"(d), "n"(B));
  return s;
}

// Adds to (lo, hi) the lanes whose digit differs from this lane's in bit B or
// B+1: for each bit, the ballot of the bit XOR this lane's bit spread over the
// word.  One v_bitop3_b32 per bit and half computes lo | (m ^ s) (truth table
// 0xF6 with operands in the order lo, m, s); together with the ballot's
// compare and the extract that is 4 instructions per digit bit, which matters
// because the scatter is bound by instruction issue, not by HBM.
template <int B>
__device__ __forceinline__ void differing_lanes(uint32_t d, uint32_t& lo, uint32_t& hi) {
  const uint32_t s0 = spread_bit<B>(d), s1 = spread_bit<B + 1>(d);
  const uint64_t m0 = __ballot(s0 != 0), m1 = __ballot(s1 != 0);
  lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m0, s0, 0xF6);
  hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m0 >> 32), s0, 0xF6);
  lo = __builtin_amdgcn_bitop3_b32(lo, (uint32_t)m1, s1, 0xF6);
  hi = __builtin_amdgcn_bitop3_b32(hi, (uint32_t)(m1 >> 32), s1, 0xF6);
}

template <int kBlock, int kItems>
struct ScatterLds {
  static constexpr int kWaves = kBlock / 64;
  static constexpr int kTile = kBlock * kItems;
  uint2 kr[kTile];  // reorder buffer: key and row of each element (the rank masks before)
  uint16_t wcnt[kWaves][kRadix];  // per-wave digit counts, then each wave's start of each digit in the tile
  uint32_t dbase[kRadix];         // global start minus tile-local start
  uint32_t scan[kWaves];
};

// The tile's keys and rows: wave w owns 64*kItems consecutive elements, lane
// l the elements w*64*kItems + i*64 + l.
template <int kBlock, int kItems, class IO>
__device__ __forceinline__ void scatter_load(const IO& io, uint32_t base, uint32_t tile_n,
                                             uint32_t (&key)[kItems], uint32_t (&row)[kItems]) {
  constexpr int kTile = kBlock * kItems;
  const uint32_t w = threadIdx.x / 64, lane = lane_id();
  const uint32_t wbase = w * 64 * kItems;
  if (tile_n == (uint32_t)kTile) {  // uniform: every load of a full tile is issued unconditionally
#pragma unroll
    for (int i = 0; i < kItems; ++i) key[i] = __builtin_nontemporal_load(io.src_keys + base + wbase + i * 64 + lane);
    if (io.implicit_rows) {
#pragma unroll
      for (int i = 0; i < kItems; ++i) row[i] = base + wbase + i * 64 + lane - io.row_origin;
    } else {
#pragma unroll
      for (int i = 0; i < kItems; ++i)
        row[i] = __builtin_nontemporal_load(io.src_rows + base + wbase + i * 64 + lane);
    }
  } else {
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      const uint32_t local = wbase + i * 64 + lane;
      const uint32_t g = base + local;
      const bool valid = local < tile_n;
      key[i] = valid ? (uint32_t)io.src_keys[g] : 0u;
      row[i] = valid ? (io.implicit_rows ? g - io.row_origin : io.src_rows[g]) : 0u;
    }
  }
}

// Ranks, reorders and writes one tile whose keys and rows are in registers
// (their loads may still be in flight); dstart = the table entry of digit
// threadIdx.x for this tile.  Starts and ends with a barrier.  With kCheck a
// key at or above 2^check_shift sets *reject to 1.  With kFull the tile is
// full (tile_n = kBlock * kItems) and no element is checked against tile_n.
template <int kBlock, int kItems, bool kCheck = false, bool kTag = false, int kBits = kRadixBits, bool kFull = false,
          class IO>
__device__ __forceinline__ void scatter_tile(ScatterLds<kBlock, kItems>& L, const IO& io, uint32_t shift,
                                             uint32_t tile_n, uint32_t dstart, const uint32_t (&key)[kItems],
                                             const uint32_t (&row)[kItems], uint32_t check_shift = 32,
                                             uint32_t* reject = nullptr) {
  constexpr int kWaves = kBlock / 64;
  static_assert(kBits >= 2 && kBits <= kRadixBits && kBits % 2 == 0, "digit widths 2, 4, 6, 8");
  constexpr uint32_t kMask = (1u << kBits) - 1u;
  const uint32_t tid = threadIdx.x, w = tid / 64, lane = lane_id();
  const uint32_t wbase = w * 64 * kItems;
  for (int i = tid; i < kWaves * kRadix; i += kBlock) (&L.wcnt[0][0])[i] = 0;
  // 8-bit digits: per-wave digit masks, in the reorder buffer (unused until
  // the reorder).
  constexpr bool kMaskRank = kBits == kRadixBits;
  static_assert(kBlock * kItems >= kWaves * kRadix, "digit masks fit the reorder buffer");
  uint64_t* dmask = reinterpret_cast<uint64_t*>(&L.kr[0]) + w * kRadix;
  if (kMaskRank)
    for (int j = lane; j < kRadix; j += 64) dmask[j] = 0ull;
  __syncthreads();

  // ---- rank inside the wave: peers = lanes with the same digit ----------------
  // 8-bit digits: digits 0 and 1, the most frequent ones on small values, by
  // one ballot each; every other digit by its mask: the lanes holding it OR
  // their bits into it, read it back and clear it (three LDS operations of the
  // one wave, executed in order; OR commutes, so the mask is exact whatever
  // order the lanes are served in).  That costs fewer instructions than a
  // ballot per digit bit (≈30 per key), and the scatter is bound by
  // instruction issue: 347 -> 330 us per 2^26 pair sort over 16-bit Zipf keys,
  // the same on uniform ones (ballots for digit 0 alone: 334 us; for 0..3:
  // 340 us).  Narrower digits take the ballots (3 rounds for 6 bits), which are
  // cheaper there: the batched build's 6-bit passes ran 1.3% slower with the
  // masks.
  const uint64_t mybit = 1ull << lane;
  uint32_t rank[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = (kFull || wbase + i * 64 + lane < tile_n);
    const uint32_t d = (key[i] >> shift) & kMask;
    uint32_t r = 0;
    uint64_t peers;
    if (kMaskRank) {
      const uint64_t b0 = __builtin_amdgcn_ballot_w64(valid && d == 0u);
      const uint64_t b1 = __builtin_amdgcn_ballot_w64(valid && d == 1u);
      peers = d == 0u ? b0 : b1;
      if (valid && d > 1u) {
        __hip_atomic_fetch_or(&dmask[d], mybit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        peers = __hip_atomic_load(&dmask[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __hip_atomic_store(&dmask[d], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      }
    } else {
      // the valid lanes whose digit equals this lane's, i.e. that differ from
      // it in no digit bit (kBits / 2 bit pairs)
      uint32_t diff_lo = 0, diff_hi = 0;
      differing_lanes<0>(d, diff_lo, diff_hi);
      if (kBits > 2) differing_lanes<2>(d, diff_lo, diff_hi);
      if (kBits > 4) differing_lanes<4>(d, diff_lo, diff_hi);
      peers = __builtin_amdgcn_ballot_w64(valid) & ~(((uint64_t)diff_hi << 32) | diff_lo);
    }
    if (valid) {
      const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
      const uint32_t old = L.wcnt[w][d];
      if (below == 0) L.wcnt[w][d] = (uint16_t)(old + (uint32_t)__popcll(peers));
      r = old + below;
    }
    rank[i] = r;
  }
  if (kCheck) {
    uint32_t over = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i)
      over |= ((kFull || wbase + i * 64 + lane < tile_n)) ? key[i] >> check_shift : 0u;
    if (__ballot(over != 0u) && lane == 0) *reject = 1u;
  }
  __syncthreads();

  // ---- per digit: tile-local offsets and global destinations ------------------
  uint32_t tile_count = 0;
  if (tid < kRadix) {
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      const uint32_t c = L.wcnt[ww][tid];
      L.wcnt[ww][tid] = (uint16_t)tile_count;
      tile_count += c;
    }
  }
  uint32_t total;
  const uint32_t loff = block_excl_scan<kBlock>(tid < kRadix ? tile_count : 0u, L.scan, &total);
  // Each wave's start of each digit in the tile: the digit's tile-local start
  // added to its per-wave offsets here, once per (wave, digit), so the reorder
  // reads one LDS word per key instead of two (2^26 Zipf sort: -5 us).
  if (tid < kRadix) {
    L.dbase[tid] = dstart - loff;
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) L.wcnt[ww][tid] = (uint16_t)(L.wcnt[ww][tid] + loff);
  }
  __syncthreads();

  // ---- reorder the tile by digit in LDS ---------------------------------------
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if ((kFull || wbase + i * 64 + lane < tile_n)) {
      const uint32_t d = (key[i] >> shift) & kMask;
      const uint32_t pos = L.wcnt[w][d] + rank[i];
      L.kr[pos] = make_uint2(key[i], row[i]);
    }
  }
  __syncthreads();

  // ---- write each digit's run to its global place ------------------------------
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t p = i * kBlock + tid;
    if (kFull || p < tile_n) {
      const uint2 v = L.kr[p];
      const uint32_t k = v.x;
      const uint32_t g = L.dbase[(k >> shift) & kMask] + p;
      io.dst_keys[g] = (std::remove_pointer_t<decltype(io.dst_keys)>)(kTag ? (k & io.key_and) | io.key_or : k);
      io.dst_rows[g] = v.y;
    }
  }
  __syncthreads();  // the LDS buffers are free again
}

// One work-group per tile.
template <int kBlock, int kItems>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(PassBuffers buf, const SortPlan* __restrict__ plan,
                                                          const uint32_t* __restrict__ table, uint32_t pass,
                                                          uint32_t n_cap, uint32_t ntiles,
                                                          const uint64_t* __restrict__ d_n) {
  constexpr int kTile = kBlock * kItems;
  __shared__ ScatterLds<kBlock, kItems> L;
  const uint32_t active = plan->active;
  if (!((active >> pass) & 1u)) return;
  const PassIo io = pass_io(buf, active, pass);
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  const uint32_t base = tile * kTile;
  const uint32_t tile_n = tile_len(tile, kTile, n_cap, d_n);
  if (tile_n == 0) return;  // past a device-resident count
  // This tile's output position for each digit: loaded first, used last.
  const uint32_t dstart = threadIdx.x < kRadix ? table[(uint64_t)threadIdx.x * ntiles + tile] : 0u;
  uint32_t key[kItems], row[kItems];
  scatter_load<kBlock, kItems>(io, base, tile_n, key, row);
  if (tile_n == (uint32_t)kTile)  // uniform: a full tile checks no element against its length
    scatter_tile<kBlock, kItems, false, false, kRadixBits, true>(L, io, pass * kRadixBits, tile_n, dstart, key, row);
  else
    scatter_tile<kBlock, kItems>(L, io, pass * kRadixBits, tile_n, dstart, key, row);
}

// Scatter of a fixed pass (no plan): keys uint32 or uint16 on either side.
// With kCheck (the first pass of the narrow-key sort) a key at or above
// 2^check_shift sets *reject.
template <int kBlock, int kItems, bool kCheck, int kBits, class SK, class DK>
__global__ __launch_bounds__(kBlock) void k_radix_scatter_fixed(PassIoT<SK, DK> io, const uint32_t* __restrict__ table,
                                                                uint32_t shift, uint32_t n_cap, uint32_t ntiles,
                                                                uint32_t check_shift, uint32_t* __restrict__ reject,
                                                                const uint64_t* __restrict__ d_n) {
  constexpr int kTile = kBlock * kItems;
  __shared__ ScatterLds<kBlock, kItems> L;
  const uint32_t tile = xcd_tile(blockIdx.x, ntiles);
  const uint32_t base = tile * kTile;
  const uint32_t tile_n = tile_len(tile, kTile, n_cap, d_n);
  if (tile_n == 0) return;  // past a device-resident count
  const uint32_t dstart = threadIdx.x < kRadix ? table[(uint64_t)threadIdx.x * ntiles + tile] : 0u;
  uint32_t key[kItems], row[kItems];
  scatter_load<kBlock, kItems>(io, base, tile_n, key, row);
  if (tile_n == (uint32_t)kTile)  // uniform: a full tile checks no element against its length
    scatter_tile<kBlock, kItems, kCheck, false, kBits, true>(L, io, shift, tile_n, dstart, key, row, check_shift,
                                                             reject);
  else
    scatter_tile<kBlock, kItems, kCheck, false, kBits, false>(L, io, shift, tile_n, dstart, key, row, check_shift,
                                                              reject);
}

}  // namespace

namespace {

template <int kBlock, int kItems>
int sort_with_shape(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys, uint32_t* srows,
                    uint64_t n, const uint64_t* d_n) {
  constexpr int kTile = kBlock * kItems;
  SortPlan* plan = reinterpret_cast<SortPlan*>(env.arena()->plan);
  const uint32_t ntiles = (uint32_t)((n + kTile - 1) / kTile);
  const uint32_t nn = (uint32_t)n;

  PassBuffers buf;
  buf.keys_in = keys;
  buf.rows_in = rows;
  buf.keys_a = skeys;
  buf.rows_a = srows;
  buf.keys_b = static_cast<uint32_t*>(env.scratch(n * 4));
  buf.rows_b = static_cast<uint32_t*>(env.scratch(n * 4));
  uint32_t* table = static_cast<uint32_t*>(env.scratch((uint64_t)ntiles * kRadix * 4));
  uint32_t* offs = static_cast<uint32_t*>(env.scratch((uint64_t)ntiles * kRadix * 4));
  uint32_t* orand = static_cast<uint32_t*>(env.scratch((uint64_t)ntiles * 2 * 4));
  if (!buf.keys_b || !buf.rows_b || !table || !offs || !orand)
    return env.fail(kErrOom, "radix_sort: scratch buffers");
  // One work-group per tile.  (Grid-stride versions with occupancy-sized
  // grids made skipped passes cheaper but active scatters 50% slower: the two
  // work-groups of a CU then run their phases in step instead of interleaved.)
  const uint32_t g_up0 = ntiles, g_up = ntiles, g_sc = ntiles;
  for (uint32_t pass = 0; pass < (uint32_t)kPasses; ++pass) {
    if (pass == 0) {
      env.prof_begin("radix_upsweep0");
      k_radix_upsweep<true, kTile><<<dim3(g_up0), dim3(kUpBlock), 0, env.stream()>>>(buf, plan, table, orand, pass,
                                                                                      nn, ntiles, d_n);
      env.prof_end("radix_upsweep0");
      int rc = check_launch(env, "radix_upsweep launch");
      if (rc) return rc;
      env.prof_begin("radix_plan");
      k_radix_plan<<<dim3(1), dim3(kPlanBlock), 0, env.stream()>>>(orand, ntiles, plan);
      env.prof_end("radix_plan");
      rc = check_launch(env, "radix_plan launch");
      if (rc) return rc;
    } else {
      env.prof_begin("radix_upsweep");
      k_radix_upsweep<false, kTile><<<dim3(g_up), dim3(kUpBlock), 0, env.stream()>>>(buf, plan, table, orand,
                                                                                       pass, nn, ntiles, d_n);
      env.prof_end("radix_upsweep");
      int rc = check_launch(env, "radix_upsweep launch");
      if (rc) return rc;
    }
    // Offsets: exclusive scan of the digit-major table into offs (the scan's
    // input and output must not overlap); the plan gives a skipped pass a
    // scan of length 0.
    int rc = launch_exclusive_scan(env, table, offs, (uint64_t)ntiles * kRadix, &plan->scan_len[pass]);
    if (rc) return rc;
    env.prof_begin("radix_scatter");
    k_radix_scatter<kBlock, kItems><<<dim3(g_sc), dim3(kBlock), 0, env.stream()>>>(
        buf, static_cast<const SortPlan*>(plan), offs, pass, nn, ntiles, d_n);
    env.prof_end("radix_scatter");
    rc = check_launch(env, "radix_scatter launch");
    if (rc) return rc;
  }
  return kOk;
}

// ---------------------------------------------------------------------------------
// the segmented sort: a batch of requests, keys sorted inside each request
// ---------------------------------------------------------------------------------
// Request j owns positions [req_off[j], req_off[j+1]); its tiles are its
// positions cut at the multiples of kTile, so tile l of request j covers
// [max(req_off[j], (c0 + l) kTile), min(req_off[j+1], (c0 + l + 1) kTile)) with
// c0 = req_off[j] / kTile (whole tiles stay aligned).  tile_base[j] is the
// number of tiles of the requests before j.  The digit table holds request j's
// counts at 256 tile_base[j] + d ntiles_j + l: scanned in that order, each
// entry is the position in the batch of the tile's first key with digit d, and
// no key leaves its request.  Rows are made relative to the request's first
// position; the last pass writes the key tagged with its request (j <<
// value_bits | key), which is what the encoder and the per-request split read.
template <int kTile>
__global__ __launch_bounds__(256) void k_seg_tiles(const uint32_t* __restrict__ req_off, uint32_t nreq,
                                                   uint32_t* __restrict__ ntiles) {
  for (uint32_t j = blockIdx.x * 256 + threadIdx.x; j <= nreq; j += gridDim.x * 256) {
    uint32_t nt = 0;
    if (j < nreq && req_off[j + 1] > req_off[j])
      nt = (req_off[j + 1] + (uint32_t)kTile - 1u) / (uint32_t)kTile - req_off[j] / (uint32_t)kTile;
    ntiles[j] = nt;
  }
}

// The table's length for its scan: 256 entries per tile of the batch.
__global__ void k_seg_table_len(const uint32_t* __restrict__ tile_base, uint32_t nreq, uint64_t* __restrict__ len) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *len = (uint64_t)kRadix * tile_base[nreq];
}

struct SegTile {
  uint32_t j, l, base, len, nt;
};

// Request and place of tile t < tile_base[nreq]: the last request j with
// tile_base[j] <= t (empty requests share their successor's base).
template <int kTile>
__device__ __forceinline__ SegTile seg_tile(const uint32_t* __restrict__ req_off, const uint32_t* __restrict__ tile_base,
                                            uint32_t nreq, uint32_t t) {
  uint32_t lo = 0, hi = nreq;
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) / 2u;
    if (tile_base[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  SegTile s;
  s.j = lo;
  s.l = t - tile_base[lo];
  s.nt = tile_base[lo + 1] - tile_base[lo];
  const uint32_t r0 = req_off[lo], r1 = req_off[lo + 1], c0 = r0 / (uint32_t)kTile;
  s.base = max(r0, (c0 + s.l) * (uint32_t)kTile);
  s.len = min(r1, (c0 + s.l + 1u) * (uint32_t)kTile) - s.base;
  return s;
}

template <int kTile, int kRounds, class SK>
__global__ __launch_bounds__(kUpBlock) void k_seg_count(const SK* __restrict__ keys, uint32_t* __restrict__ table,
                                                        uint32_t shift, uint32_t mask,
                                                        const uint32_t* __restrict__ req_off,
                                                        const uint32_t* __restrict__ tile_base, uint32_t nreq,
                                                        uint32_t ub) {
  const uint32_t t = xcd_tile(blockIdx.x, ub);
  if (t >= tile_base[nreq]) return;  // uniform over the work-group
  const SegTile s = seg_tile<kTile>(req_off, tile_base, nreq, t);
  upsweep_tile<kTile, kRounds, false>(keys, shift, s.base, s.len, table, (uint64_t)kRadix * tile_base[s.j] + s.l, s.nt,
                                      t, nullptr, mask);
}

// kCheck (the first pass): a key at or above 2^value_bits flags its request
// (req_bad[j]) or, without req_bad, the batch (*bad).  kTag (the last pass):
// keys are written as j << value_bits | key.
template <int kBlock, int kItems, bool kCheck, bool kTag, int kBits, class SK, class DK>
__global__ __launch_bounds__(kBlock) void k_seg_scatter(PassIoT<SK, DK> io, const uint32_t* __restrict__ table,
                                                        uint32_t shift, const uint32_t* __restrict__ req_off,
                                                        const uint32_t* __restrict__ tile_base, uint32_t nreq,
                                                        uint32_t ub, uint32_t value_bits, uint32_t* __restrict__ bad,
                                                        uint32_t* __restrict__ req_bad) {
  constexpr int kTile = kBlock * kItems;
  __shared__ ScatterLds<kBlock, kItems> L;
  const uint32_t t = xcd_tile(blockIdx.x, ub);
  if (t >= tile_base[nreq]) return;  // uniform over the work-group
  const SegTile s = seg_tile<kTile>(req_off, tile_base, nreq, t);
  const uint32_t dstart =
      threadIdx.x < kRadix ? table[(uint64_t)kRadix * tile_base[s.j] + (uint64_t)threadIdx.x * s.nt + s.l] : 0u;
  io.row_origin = req_off[s.j];
  if (kTag) {
    io.key_and = value_bits < 32 ? (1u << value_bits) - 1u : ~0u;
    io.key_or = value_bits < 32 ? s.j << value_bits : 0u;
  }
  uint32_t key[kItems], row[kItems];
  scatter_load<kBlock, kItems>(io, s.base, s.len, key, row);
  uint32_t* const flag = req_bad ? req_bad + s.j : bad;
  if (s.len == (uint32_t)kTile)  // uniform: a full tile checks no element against its length
    scatter_tile<kBlock, kItems, kCheck, kTag, kBits, true>(L, io, shift, s.len, dstart, key, row, value_bits, flag);
  else
    scatter_tile<kBlock, kItems, kCheck, kTag, kBits, false>(L, io, shift, s.len, dstart, key, row, value_bits, flag);
}

// Digits of a fixed-pass sort of values below 2^value_bits (value_bits 1..16):
// pass p ranks `bits` bits from `shift` on.  The byte split takes 8 bits, then
// the rest; the even split halves value_bits.  Widths are rounded up to even
// (the ranking takes the bits in pairs): bits above value_bits are 0 in every
// key that passes the range check, and a key that fails it is flagged and its
// result discarded, so masking them only keeps its ranks in range.
struct DigitSplit {
  uint32_t passes;
  uint32_t shift[2], bits[2];
};

DigitSplit digit_split(uint32_t value_bits, bool even) {
  auto up2 = [](uint32_t b) { return (b + 1u) & ~1u; };
  DigitSplit d{};
  d.passes = (value_bits + kRadixBits - 1) / kRadixBits;
  if (d.passes == 1) {
    d.shift[0] = 0;
    d.bits[0] = up2(value_bits);
    return d;
  }
  const uint32_t b0 = even ? up2((value_bits + 1) / 2) : (uint32_t)kRadixBits;
  d.shift[0] = 0;
  d.bits[0] = b0;
  d.shift[1] = b0;
  d.bits[1] = up2(value_bits - b0);
  return d;
}

// Launch of a fixed-pass scatter for a digit width known at run time.
template <int kBits, int kBlock, int kItems, bool kCheck, class SK, class DK>
void scatter_fixed_bits(Env& env, uint32_t grid, const PassIoT<SK, DK>& io, const uint32_t* offs, uint32_t shift,
                        uint32_t nn, uint32_t ntiles, uint32_t check_shift, uint32_t* reject, const uint64_t* d_n) {
  k_radix_scatter_fixed<kBlock, kItems, kCheck, kBits><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(
      io, offs, shift, nn, ntiles, check_shift, reject, d_n);
}

template <int kBlock, int kItems, bool kCheck, class SK, class DK>
void scatter_fixed(Env& env, uint32_t bits, uint32_t grid, const PassIoT<SK, DK>& io, const uint32_t* offs,
                   uint32_t shift, uint32_t nn, uint32_t ntiles, uint32_t check_shift, uint32_t* reject,
                   const uint64_t* d_n) {
  switch (bits) {
    case 2:
      return scatter_fixed_bits<2, kBlock, kItems, kCheck>(env, grid, io, offs, shift, nn, ntiles, check_shift, reject,
                                                            d_n);
    case 4:
      return scatter_fixed_bits<4, kBlock, kItems, kCheck>(env, grid, io, offs, shift, nn, ntiles, check_shift, reject,
                                                            d_n);
    case 6:
      return scatter_fixed_bits<6, kBlock, kItems, kCheck>(env, grid, io, offs, shift, nn, ntiles, check_shift, reject,
                                                            d_n);
    default:
      return scatter_fixed_bits<8, kBlock, kItems, kCheck>(env, grid, io, offs, shift, nn, ntiles, check_shift, reject,
                                                            d_n);
  }
}

// The narrow-key sort: keys below 2^value_bits, value_bits <= 16, rows
// 0..n-1.  ceil(value_bits / 8) fixed passes (no plan, no skipped launches)
// with the even split of digit_split; from the first pass on the keys are
// stored as uint16 (6 bytes per pair instead of 8).  The first pass flags a
// key at or above 2^value_bits in *reject (cleared by its upsweep); the sort's
// output is then unspecified.
template <int kBlock, int kItems>
int sort16_with_shape(Env& env, const uint32_t* keys, uint16_t* skeys, uint32_t* srows, uint64_t n,
                      uint32_t value_bits, uint32_t* reject, const uint64_t* d_n) {
  constexpr int kTile = kBlock * kItems;
  const uint32_t ntiles = (uint32_t)((n + kTile - 1) / kTile);
  const uint32_t nn = (uint32_t)n;
  const DigitSplit ds = digit_split(value_bits, true);
  const uint32_t passes = ds.passes;
  uint16_t* kb = nullptr;
  uint32_t* rb = nullptr;
  if (passes > 1) {
    kb = static_cast<uint16_t*>(env.scratch(n * 2));
    rb = static_cast<uint32_t*>(env.scratch(n * 4));
    if (!kb || !rb) return env.fail(kErrOom, "radix_sort16: scratch buffers");
  }
  uint32_t* table = static_cast<uint32_t*>(env.scratch((uint64_t)ntiles * kRadix * 4));
  uint32_t* offs = static_cast<uint32_t*>(env.scratch((uint64_t)ntiles * kRadix * 4));
  if (!table || !offs) return env.fail(kErrOom, "radix_sort16: digit tables");
  const uint64_t tlen = (uint64_t)ntiles * kRadix;
  int rc;
  // pass 0: uint32 values in, uint16 keys out
  env.prof_begin("radix_upsweep0");
  k_radix_count<kTile, 1, uint32_t><<<dim3(ntiles), dim3(kUpBlock), 0, env.stream()>>>(
      keys, table, ds.shift[0], (1u << ds.bits[0]) - 1u, nn, ntiles, reject, d_n);
  env.prof_end("radix_upsweep0");
  if ((rc = check_launch(env, "radix_count launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, table, offs, tlen, nullptr))) return rc;
  PassIoT<uint32_t, uint16_t> io0{keys, nullptr, passes > 1 ? kb : skeys, passes > 1 ? rb : srows, true};
  env.prof_begin("radix_scatter");
  scatter_fixed<kBlock, kItems, true>(env, ds.bits[0], ntiles, io0, offs, ds.shift[0], nn, ntiles, value_bits, reject,
                                      d_n);
  env.prof_end("radix_scatter");
  if ((rc = check_launch(env, "radix_scatter launch"))) return rc;
  if (passes == 1) return kOk;
  // pass 1: uint16 keys in and out
  env.prof_begin("radix_upsweep");
  k_radix_count<kTile, -1, uint16_t><<<dim3(ntiles), dim3(kUpBlock), 0, env.stream()>>>(
      kb, table, ds.shift[1], (1u << ds.bits[1]) - 1u, nn, ntiles, nullptr, d_n);
  env.prof_end("radix_upsweep");
  if ((rc = check_launch(env, "radix_count launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, table, offs, tlen, nullptr))) return rc;
  PassIoT<uint16_t, uint16_t> io1{kb, rb, skeys, srows, false};
  env.prof_begin("radix_scatter");
  scatter_fixed<kBlock, kItems, false>(env, ds.bits[1], ntiles, io1, offs, ds.shift[1], nn, ntiles, 32u, nullptr,
                                       d_n);
  env.prof_end("radix_scatter");
  return check_launch(env, "radix_scatter launch");
}

// Launch of a segmented scatter for a digit width known at run time.
template <int kBlock, int kItems, bool kCheck, bool kTag, class SK, class DK>
void seg_scatter(Env& env, uint32_t bits, uint32_t grid, const PassIoT<SK, DK>& io, const uint32_t* offs,
                 uint32_t shift, const uint32_t* req_off, const uint32_t* tile_base, uint32_t nreq, uint32_t ub,
                 uint32_t value_bits, uint32_t* bad, uint32_t* req_bad) {
#define KA_SEG_SCATTER(B)                                                                                   \
  k_seg_scatter<kBlock, kItems, kCheck, kTag, B><<<dim3(grid), dim3(kBlock), 0, env.stream()>>>(          \
      io, offs, shift, req_off, tile_base, nreq, ub, value_bits, bad, req_bad)
  switch (bits) {
    case 2:
      KA_SEG_SCATTER(2);
      break;
    case 4:
      KA_SEG_SCATTER(4);
      break;
    case 6:
      KA_SEG_SCATTER(6);
      break;
    default:
      KA_SEG_SCATTER(8);
      break;
  }
#undef KA_SEG_SCATTER
}

// The segmented sort of a batch (values below 2^value_bits, value_bits <= 16):
// uint16 keys between passes, request-relative rows, tagged uint32 keys out;
// the byte or the even digit split.
int seg_sort(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
             uint32_t value_bits, uint32_t* skeys, uint32_t* srows, uint32_t* bad, uint32_t* req_bad, bool even) {
  constexpr int kBlock = kShapes[0].block, kItems = kShapes[0].items, kTile = kBlock * kItems;
  const DigitSplit ds = digit_split(value_bits, even);
  const uint32_t passes = ds.passes;
  const uint64_t ub64 = (n + kTile - 1) / kTile + nreq;  // tiles: at most one more per request
  if (ub64 >= (1ull << 31)) return env.fail(kErrArg, "segmented sort: too many tiles");
  const uint32_t ub = (uint32_t)ub64;
  uint32_t* ntiles = static_cast<uint32_t*>(env.scratch(4ull * (nreq + 1)));
  uint32_t* tile_base = static_cast<uint32_t*>(env.scratch(4ull * (nreq + 1)));
  uint64_t* tlen = static_cast<uint64_t*>(env.scratch(8));
  uint32_t* table = static_cast<uint32_t*>(env.scratch((uint64_t)kRadix * ub * 4));
  uint32_t* offs = static_cast<uint32_t*>(env.scratch((uint64_t)kRadix * ub * 4));
  uint16_t* kb = passes > 1 ? static_cast<uint16_t*>(env.scratch(2 * n)) : nullptr;
  uint32_t* rb = passes > 1 ? static_cast<uint32_t*>(env.scratch(4 * n)) : nullptr;
  if (!ntiles || !tile_base || !tlen || !table || !offs || (passes > 1 && (!kb || !rb)))
    return env.fail(kErrOom, "segmented sort: scratch");
  int rc;
  env.prof_begin("seg_tiles");
  k_seg_tiles<kTile><<<dim3(std::min<uint32_t>((nreq + 256) / 256, 1024)), dim3(256), 0, env.stream()>>>(req_off, nreq,
                                                                                                      ntiles);
  env.prof_end("seg_tiles");
  if ((rc = check_launch(env, "seg_tiles launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, ntiles, tile_base, nreq + 1ull, nullptr))) return rc;
  k_seg_table_len<<<dim3(1), dim3(64), 0, env.stream()>>>(tile_base, nreq, tlen);
  if ((rc = check_launch(env, "seg_table_len launch"))) return rc;
  const uint64_t tcap = (uint64_t)kRadix * ub;
  // pass 0: uint32 values in (checked), uint16 keys out -- or tagged keys if it is the only pass
  env.prof_begin("radix_upsweep0");
  k_seg_count<kTile, 1, uint32_t><<<dim3(ub), dim3(kUpBlock), 0, env.stream()>>>(
      values, table, ds.shift[0], (1u << ds.bits[0]) - 1u, req_off, tile_base, nreq, ub);
  env.prof_end("radix_upsweep0");
  if ((rc = check_launch(env, "seg_count launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, table, offs, tcap, tlen))) return rc;
  env.prof_begin("radix_scatter");
  if (passes == 1) {
    PassIoT<uint32_t, uint32_t> io{values, nullptr, skeys, srows, true};
    seg_scatter<kBlock, kItems, true, true>(env, ds.bits[0], ub, io, offs, ds.shift[0], req_off, tile_base, nreq, ub,
                                            value_bits, bad, req_bad);
  } else {
    PassIoT<uint32_t, uint16_t> io{values, nullptr, kb, rb, true};
    seg_scatter<kBlock, kItems, true, false>(env, ds.bits[0], ub, io, offs, ds.shift[0], req_off, tile_base, nreq, ub,
                                             value_bits, bad, req_bad);
  }
  env.prof_end("radix_scatter");
  if ((rc = check_launch(env, "seg_scatter launch"))) return rc;
  if (passes == 1) return kOk;
  // pass 1: uint16 keys in, tagged uint32 keys out
  env.prof_begin("radix_upsweep");
  k_seg_count<kTile, -1, uint16_t><<<dim3(ub), dim3(kUpBlock), 0, env.stream()>>>(
      kb, table, ds.shift[1], (1u << ds.bits[1]) - 1u, req_off, tile_base, nreq, ub);
  env.prof_end("radix_upsweep");
  if ((rc = check_launch(env, "seg_count launch"))) return rc;
  if ((rc = launch_exclusive_scan(env, table, offs, tcap, tlen))) return rc;
  PassIoT<uint16_t, uint32_t> io1{kb, rb, skeys, srows, false};
  env.prof_begin("radix_scatter");
  seg_scatter<kBlock, kItems, false, true>(env, ds.bits[1], ub, io1, offs, ds.shift[1], req_off, tile_base, nreq, ub,
                                           value_bits, bad, req_bad);
  env.prof_end("radix_scatter");
  return check_launch(env, "seg_scatter launch");
}

}  // namespace

int sort_shape_count() { return kNumShapes; }
int batch_variant_count() { return kNumShapes + 1; }

int launch_radix_sort_segments(Env& env, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                               uint32_t value_bits, uint32_t* skeys, uint32_t* srows, uint32_t* bad,
                               uint32_t* req_bad, bool even_split) {
  if (n == 0) return kOk;
  if (!values || !req_off || !skeys || !srows || !bad || nreq == 0)
    return env.fail(kErrArg, "segmented sort: null buffer");
  if (value_bits == 0 || value_bits > 16) return env.fail(kErrArg, "segmented sort: value_bits must be 1..16");
  if (n >= (1ull << 31)) return env.fail(kErrArg, "segmented sort: n must be below 2^31");
  return seg_sort(env, values, n, req_off, nreq, value_bits, skeys, srows, bad, req_bad, even_split);
}

const uint32_t* sort_plan_keys_or(Env& env) {
  return reinterpret_cast<const uint32_t*>(static_cast<const char*>(env.arena()->plan) + offsetof(SortPlan, keys_or));
}

int launch_radix_sort_rows16(Env& env, const uint32_t* keys, uint16_t* skeys, uint32_t* srows, uint64_t n,
                             uint32_t value_bits, uint32_t* reject, int shape, const uint64_t* d_n) {
  if (!reject) return env.fail(kErrArg, "radix_sort16: null reject flag");
  if (value_bits == 0 || value_bits > 16) return env.fail(kErrArg, "radix_sort16: value_bits must be 1..16");
  if (n == 0) return launch_fill_u32(env, reject, 1, 0);
  if (!keys || !skeys || !srows) return env.fail(kErrArg, "radix_sort16: null buffer");
  if (n >= (1ull << 31)) return env.fail(kErrArg, "radix_sort16: n must be below 2^31");
  switch (shape) {
    case 0:
      return sort16_with_shape<kShapes[0].block, kShapes[0].items>(env, keys, skeys, srows, n, value_bits, reject,
                                                                      d_n);
    case 1:
      return sort16_with_shape<kShapes[1].block, kShapes[1].items>(env, keys, skeys, srows, n, value_bits, reject,
                                                                      d_n);
    case 2:
      return sort16_with_shape<kShapes[2].block, kShapes[2].items>(env, keys, skeys, srows, n, value_bits, reject,
                                                                      d_n);
    default:
      return env.fail(kErrArg, "radix_sort16: unknown tile shape");
  }
}

int launch_radix_sort_pairs(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys,
                            uint32_t* srows, uint64_t n, int shape, const uint64_t* d_n) {
  if (n == 0) return kOk;
  if (!keys || !skeys || !srows) return env.fail(kErrArg, "radix_sort: null buffer");
  if (n >= (1ull << 31)) return env.fail(kErrArg, "radix_sort: n must be below 2^31");
  switch (shape) {
    case 0:
      return sort_with_shape<kShapes[0].block, kShapes[0].items>(env, keys, rows, skeys, srows, n, d_n);
    case 1:
      return sort_with_shape<kShapes[1].block, kShapes[1].items>(env, keys, rows, skeys, srows, n, d_n);
    case 2:
      return sort_with_shape<kShapes[2].block, kShapes[2].items>(env, keys, rows, skeys, srows, n, d_n);
    default:
      return env.fail(kErrArg, "radix_sort: unknown tile shape");
  }
}

}  // namespace ka
