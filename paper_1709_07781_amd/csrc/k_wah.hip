// WAH encoding of sorted (value, row) pairs -- parts 3 to 6 of the index build
// of Sec. 4.1 in one pass over the sorted pairs:
//   part 3  chunk ids and literals: a group is a maximal run of equal value
//           and equal chunk id row / 31; its literal ORs 1 << (row % 31);
//   part 4  fills: the gap of empty chunks since the previous group of the
//           same value (or since chunk -1 for the value's first group);
//   part 5  fuseFillsLiterals: the fill and literal words of every group in
//           order, zero fills dropped (a stream compaction, fused here: each
//           group emits 1 or 2 words and the word positions are a prefix sum);
//   part 6  lookup table: keys[d] and offsets[d] for the first group of each
//           value, offsets[D] = W.
//
// A group spans at most 31 sorted elements (rows are distinct), so a tile
// finishes a group that runs past its end by reading at most 30 elements ahead
// (kLook); the only dependency between tiles is the pair (words, values)
// emitted by earlier tiles, found by decoupled look-back on two channels, each
// covering 256 predecessors per round trip.  A tile publishes its totals as
// soon as it has counted, before it builds its literals.  Words are staged in
// LDS (over the staged input, which is no longer needed by then) and written
// out by consecutive work-items.
#include "common.hpp"

namespace ka {
namespace {

constexpr int kEncBlock = 256;
#ifndef KA_ENC_ITEMS
#define KA_ENC_ITEMS 16
#endif
constexpr int kEncItems = KA_ENC_ITEMS;
constexpr int kEncTile = kEncBlock * kEncItems;  // 4096 pairs
constexpr int kLook = 32;                        // >= 30 elements of look-ahead
constexpr int kStage = kEncTile + 1 + kLook;     // one element of look-behind
constexpr uint32_t kGroupRows = 31;
constexpr uint32_t kFill = 0x80000000u;

// Padded LDS index: one spare word every 16 so that a work-item reading its
// kEncItems consecutive elements does not collide on banks with its neighbours.
__device__ __forceinline__ uint32_t pidx(uint32_t i) { return i + (i >> 4); }
constexpr int kStagePadded = kStage + kStage / 16 + 1;
static_assert(2 * kEncTile <= 2 * kStagePadded, "word staging fits over the input staging");

template <bool kVec>
__global__ __launch_bounds__(kEncBlock) void k_wah_encode(const uint32_t* __restrict__ skeys,
                                                          const uint32_t* __restrict__ srows, uint32_t n,
                                                          uint32_t* __restrict__ out_keys,
                                                          uint32_t* __restrict__ out_offsets,
                                                          uint32_t* __restrict__ out_words,
                                                          uint64_t* __restrict__ len_keys,
                                                          uint64_t* __restrict__ len_offsets,
                                                          uint64_t* __restrict__ len_words, LbArgs lb) {
  __shared__ __align__(16) uint32_t s_mem[2 * kStagePadded];
  __shared__ uint32_t s_scan[kEncBlock / 64];
  __shared__ uint32_t s_wpre, s_dpre;
  uint32_t* s_k = s_mem;
  uint32_t* s_r = s_mem + kStagePadded;
  uint32_t* s_words = s_mem;  // after the literals are built

  const uint32_t tid = threadIdx.x;
  if (n == 0) {  // empty input: D = 0, W = 0, offsets = [0]
    if (blockIdx.x == 0 && tid == 0) {
      out_offsets[0] = 0;
      *len_keys = 0;
      *len_offsets = 1;
      *len_words = 0;
    }
    return;
  }
  const uint32_t ntiles = (n + kEncTile - 1) / kEncTile;
  uint32_t tile = blockIdx.x;
  if (tile >= ntiles) return;

  // A tile's elements in registers: slot (j, c) of work-item tid holds element
  // 4 (j * kEncBlock + tid) + c; work-items 64..96 also hold the look-behind
  // element (slot 0) and the look-ahead (slots kEncTile+1 ..).
  constexpr int kVecs = kEncTile / 4 / kEncBlock;
  uint32_t vk[kVecs][4], vr[kVecs][4], xk = 0, xr = 0;
  const bool extra = tid >= 64 && tid < 64 + 1 + kLook;
  const uint32_t xslot = tid == 64 ? 0u : (uint32_t)(kEncTile + (tid - 64));
  auto fetch = [&](uint32_t t, uint32_t tid) {
    const uint32_t b = t * kEncTile;
    const uint32_t len = t < ntiles ? min((uint32_t)kEncTile, n - b) : 0u;
    if (kVec && len == (uint32_t)kEncTile) {
#pragma unroll
      for (int j = 0; j < kVecs; ++j) {
        const uint32_t q = j * kEncBlock + tid;
        const u32x4 a = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(skeys + b) + q);
        const u32x4 c = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(srows + b) + q);
        vk[j][0] = a.x, vk[j][1] = a.y, vk[j][2] = a.z, vk[j][3] = a.w;
        vr[j][0] = c.x, vr[j][1] = c.y, vr[j][2] = c.z, vr[j][3] = c.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kVecs; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t i = 4 * (j * kEncBlock + tid) + c;
          vk[j][c] = i < len ? skeys[b + i] : 0u;
          vr[j][c] = i < len ? srows[b + i] : 0u;
        }
    }
    if (extra) {
      const int64_t g = (int64_t)b - 1 + xslot;
      const bool ok = t < ntiles && g >= 0 && g < (int64_t)n;
      xk = ok ? skeys[g] : 0u;
      xr = ok ? srows[g] : 0u;
    }
  };
  for (;;) {
    // The work-item index is made opaque per tile so that the compiler
    // recomputes the addresses derived from it instead of keeping them all
    // live across the persistent loop (that would cost occupancy).
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    fetch(tile, tid);
    const uint32_t base = tile * kEncTile;
    const uint32_t tile_n = min((uint32_t)kEncTile, n - base);
    const uint32_t avail = min((uint32_t)(kEncTile + kLook), n - base);  // readable from base on

    // ---- stage elements base-1 .. base+kEncTile+kLook-1 into slots 0.. ------
#pragma unroll
    for (int j = 0; j < kVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t sl = 1 + 4 * (j * kEncBlock + tid) + c;
        s_k[pidx(sl)] = vk[j][c];
        s_r[pidx(sl)] = vr[j][c];
      }
    if (extra) {
      s_k[pidx(xslot)] = xk;
      s_r[pidx(xslot)] = xr;
    }
    __syncthreads();
    const uint32_t next = tile + gridDim.x;

    // ---- this work-item's elements, once, in registers -------------------------
    const uint32_t e0 = tid * kEncItems;
    uint32_t key[kEncItems], row[kEncItems];
#pragma unroll
    for (int i = 0; i < kEncItems; ++i) {
      key[i] = s_k[pidx(e0 + i + 1)];
      row[i] = s_r[pidx(e0 + i + 1)];
    }
    const uint32_t kprev = s_k[pidx(e0)];
    const uint32_t cprev = s_r[pidx(e0)] / kGroupRows;

    // ---- group and value heads, words and values emitted ---------------------
    uint32_t heads = 0, segs = 0, gaps = 0;  // bit i: element i starts a group / a value / has a fill
    uint32_t nw = 0, ns = 0;
#pragma unroll
    for (int i = 0; i < kEncItems; ++i) {
      if (e0 + i < tile_n) {
        const uint32_t c = row[i] / kGroupRows;
        const uint32_t kp = i ? key[i - 1] : kprev;
        const uint32_t cp = i ? row[i - 1] / kGroupRows : cprev;
        const bool seg = (base + e0 + i) == 0 || key[i] != kp;
        const bool grp = seg || c != cp;
        if (grp) {
          const bool gap = seg ? c != 0u : c != cp + 1u;
          heads |= 1u << i;
          segs |= (seg ? 1u : 0u) << i;
          gaps |= (gap ? 1u : 0u) << i;
          nw += gap ? 2u : 1u;
          ns += seg ? 1u : 0u;
        }
      }
    }
    // Both counts in one scan: words in the low half, values in the high half
    // (a tile emits at most 2*kEncTile words and kEncTile values).
    uint32_t packed_total;
    const uint32_t packed_pre = block_excl_scan<kEncBlock>((ns << 16) | nw, s_scan, &packed_total);
    const uint32_t tile_words = packed_total & 0xFFFFu, tile_segs = packed_total >> 16;
    if (tid < 2) {  // channel 0 = words, channel 1 = values
      const uint32_t agg = tid == 0 ? tile_words : tile_segs;
      lb_publish(lb.status + 2ull * tile + tid, agg, lb.epoch, tile == 0 ? kLbInclusive : kLbAggregate);
    }

    // ---- the last group may run past this work-item's elements (at most 30
    // further elements, into the look-ahead): collect its bits now ------------
    uint32_t tail = 0;
    if (e0 + kEncItems <= tile_n) {
      const uint32_t kl = key[kEncItems - 1], cl = row[kEncItems - 1] / kGroupRows;
      for (uint32_t j = e0 + kEncItems; j < avail; ++j) {
        const uint32_t kj = s_k[pidx(j + 1)];
        const uint32_t rj = s_r[pidx(j + 1)];
        const uint32_t cj = rj / kGroupRows;
        if (kj != kl || cj != cl) break;
        tail |= 1u << (rj - cj * kGroupRows);
      }
    }

    // ---- look-back: wave 0 for words, wave 1 for values --------------------
    const uint32_t wave = tid / 64;
    if (wave < 2) {
      const uint32_t agg = wave == 0 ? tile_words : tile_segs;
      uint32_t prefix = 0;
      if (tile != 0) {
        prefix = lb_lookback_wave<4>(lb.status + wave, 2, tile, lb.epoch);
        if (lane_id() == 0) lb_publish(lb.status + 2ull * tile + wave, prefix + agg, lb.epoch, kLbInclusive);
      }
      if (lane_id() == 0) {
        if (wave == 0)
          s_wpre = prefix;
        else
          s_dpre = prefix;
      }
    }
    __syncthreads();  // the staged input is dead from here on
    const uint32_t wpre = s_wpre, dpre = s_dpre;

    // ---- one backward sweep: literals (OR of the group's bits), fills and
    // lookup-table entries, placed from the end of this work-item's words --------
    {
      uint32_t w = (packed_pre & 0xFFFFu) + nw;  // one past this work-item's last word
      const uint32_t ls = packed_pre >> 16;      // tile-local index of its first value
      uint32_t acc = tail;
#pragma unroll
      for (int i = kEncItems - 1; i >= 0; --i) {
        if (e0 + i < tile_n) {
          const uint32_t c = row[i] / kGroupRows;
          acc |= 1u << (row[i] - c * kGroupRows);
          if ((heads >> i) & 1u) {
            s_words[--w] = acc;
            acc = 0;
            const bool seg = (segs >> i) & 1u;
            if ((gaps >> i) & 1u) {
              const uint32_t cp = i ? row[i - 1] / kGroupRows : cprev;
              s_words[--w] = kFill | (seg ? c : c - cp - 1u);
            }
            if (seg) {
              const uint32_t d = dpre + ls + (uint32_t)__popc(segs & ((1u << i) - 1u));
              out_keys[d] = key[i];
              out_offsets[d] = wpre + w;
            }
          }
        }
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < tile_words; i += kEncBlock) out_words[wpre + i] = s_words[i];

    if (tile == ntiles - 1 && tid == 0) {
      const uint32_t D = dpre + tile_segs, W = wpre + tile_words;
      out_offsets[D] = W;
      *len_keys = D;
      *len_offsets = (uint64_t)D + 1;
      *len_words = W;
    }
    if (next >= ntiles) break;
    __syncthreads();  // the word staging is reused by the next tile
    tile = next;
  }
}

}  // namespace

int launch_wah_encode(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                      uint64_t* d_len_words) {
  if (!offsets || !d_len_keys || !d_len_offsets || !d_len_words)
    return env.fail(kErrArg, "wah_encode_sorted: null output");
  if (n >= (1ull << 30)) return env.fail(kErrArg, "wah_encode_sorted: n must be below 2^30");
  if (n && (!skeys || !srows || !keys || !words)) return env.fail(kErrArg, "wah_encode_sorted: null buffer");
  const uint32_t tiles = n ? (uint32_t)((n + kEncTile - 1) / kEncTile) : 1u;
  LbArgs lb;
  if (!env.lookback(2ull * tiles, 0, &lb)) return env.fail(kErrOom, "wah_encode_sorted: look-back");
  const bool vec = ((reinterpret_cast<uintptr_t>(skeys) | reinterpret_cast<uintptr_t>(srows)) & 15u) == 0;
  const uint32_t nn = (uint32_t)n;
  if (vec)
    return launch_persistent(env, "wah_encode", k_wah_encode<true>, tiles, (uint32_t)kEncBlock, skeys, srows, nn,
                             keys, offsets, words, d_len_keys, d_len_offsets, d_len_words, lb);
  return launch_persistent(env, "wah_encode", k_wah_encode<false>, tiles, (uint32_t)kEncBlock, skeys, srows, nn, keys,
                           offsets, words, d_len_keys, d_len_offsets, d_len_words, lb);
}

}  // namespace ka
