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
// emitted by earlier tiles, found by decoupled look-back on two channels.
// Words are staged in LDS and written out by consecutive work-items.
#include "common.hpp"

namespace ka {
namespace {

constexpr int kEncBlock = 256;
constexpr int kEncItems = 8;
constexpr int kEncTile = kEncBlock * kEncItems;  // 2048 pairs
constexpr int kLook = 32;                        // >= 30 elements of look-ahead
constexpr int kStage = kEncTile + 1 + kLook;     // one element of look-behind
constexpr uint32_t kGroupRows = 31;
constexpr uint32_t kFill = 0x80000000u;

// Padded LDS index: one spare word every 16 so that a work-item reading its
// kEncItems consecutive elements does not collide on banks with its neighbours.
__device__ __forceinline__ uint32_t pidx(uint32_t i) { return i + (i >> 4); }
constexpr int kStagePadded = kStage + kStage / 16 + 1;

__global__ __launch_bounds__(kEncBlock) void k_wah_encode(const uint32_t* __restrict__ skeys,
                                                          const uint32_t* __restrict__ srows, uint32_t n,
                                                          uint32_t* __restrict__ out_keys,
                                                          uint32_t* __restrict__ out_offsets,
                                                          uint32_t* __restrict__ out_words,
                                                          uint64_t* __restrict__ len_keys,
                                                          uint64_t* __restrict__ len_offsets,
                                                          uint64_t* __restrict__ len_words, LbArgs lb) {
  __shared__ uint32_t s_k[kStagePadded];
  __shared__ uint32_t s_r[kStagePadded];
  __shared__ uint32_t s_words[2 * kEncTile];
  __shared__ uint32_t s_scan[kEncBlock / 64];
  __shared__ uint32_t s_tile, s_wpre, s_dpre;

  const uint32_t tile = lb_take_tile(lb, &s_tile);
  const uint32_t tid = threadIdx.x;
  const uint32_t base = tile * kEncTile;
  if (base >= n) {
    if (tile == 0 && tid == 0) {  // empty input: D = 0, W = 0, offsets = [0]
      out_offsets[0] = 0;
      *len_keys = 0;
      *len_offsets = 1;
      *len_words = 0;
    }
    return;
  }
  const uint32_t tile_n = min((uint32_t)kEncTile, n - base);
  // Elements base-1 .. base+kEncTile+kLook-1 go to LDS slots 0 .. kStage-1.
  const uint32_t avail = min((uint32_t)(kEncTile + kLook), n - base);  // readable ahead of base
  for (uint32_t i = tid; i < (uint32_t)kStage; i += kEncBlock) {
    const int64_t g = (int64_t)base - 1 + i;
    const bool ok = g >= 0 && g < (int64_t)n;
    s_k[pidx(i)] = ok ? skeys[g] : 0u;
    s_r[pidx(i)] = ok ? srows[g] : 0u;
  }
  __syncthreads();

  // ---- count words and values emitted by this work-item's elements ---------
  const uint32_t e0 = tid * kEncItems;
  uint32_t fill[kEncItems];
  uint32_t heads = 0, segs = 0;  // bit i: element i starts a group / a value
  uint32_t nw = 0, ns = 0;
#pragma unroll
  for (int i = 0; i < kEncItems; ++i) {
    fill[i] = 0;
    const uint32_t e = e0 + i;
    if (e < tile_n) {
      const uint32_t k = s_k[pidx(e + 1)];
      const uint32_t c = s_r[pidx(e + 1)] / kGroupRows;
      const bool has_prev = (base + e) > 0;
      const uint32_t kp = s_k[pidx(e)];
      const uint32_t cp = s_r[pidx(e)] / kGroupRows;
      const bool seg = !has_prev || k != kp;
      const bool grp = seg || c != cp;
      if (grp) {
        const uint32_t gap = seg ? c : c - cp - 1u;
        fill[i] = gap ? (kFill | gap) : 0u;
        heads |= 1u << i;
        segs |= (seg ? 1u : 0u) << i;
        nw += 1u + (gap ? 1u : 0u);
        ns += seg ? 1u : 0u;
      }
    }
  }
  // Both counts in one scan: words in the low half, values in the high half
  // (a tile emits at most 2*kEncTile words and kEncTile values).
  uint32_t packed_total;
  const uint32_t packed_pre = block_excl_scan<kEncBlock>((ns << 16) | nw, s_scan, &packed_total);
  const uint32_t tile_words = packed_total & 0xFFFFu, tile_segs = packed_total >> 16;

  // ---- look-back: channel 0 = words (wave 0), channel 1 = values (wave 1) ---
  const uint32_t wave = tid / 64;
  if (wave < 2) {
    const uint32_t agg = wave == 0 ? tile_words : tile_segs;
    uint64_t* st = lb.status + 2ull * tile + wave;
    uint32_t prefix = 0;
    if (tile == 0) {
      if (lane_id() == 0) lb_publish(st, agg, lb.epoch, kLbInclusive);
    } else {
      if (lane_id() == 0) lb_publish(st, agg, lb.epoch, kLbAggregate);
      prefix = lb_lookback_wave(lb.status + wave, 2, tile, lb.epoch);
      if (lane_id() == 0) lb_publish(st, prefix + agg, lb.epoch, kLbInclusive);
    }
    if (lane_id() == 0) {
      if (wave == 0)
        s_wpre = prefix;
      else
        s_dpre = prefix;
    }
  }
  __syncthreads();
  const uint32_t wpre = s_wpre, dpre = s_dpre;

  // ---- emit words (to LDS) and lookup-table entries (to HBM) ---------------
  uint32_t lw = packed_pre & 0xFFFFu;  // tile-local word index
  uint32_t ls = packed_pre >> 16;      // tile-local value index
  const uint32_t lim = avail;          // elements base .. base+lim-1 are readable
#pragma unroll
  for (int i = 0; i < kEncItems; ++i) {
    if ((heads >> i) & 1u) {
      const uint32_t e = e0 + i;
      const uint32_t k = s_k[pidx(e + 1)];
      const uint32_t r = s_r[pidx(e + 1)];
      const uint32_t c = r / kGroupRows;
      uint32_t lit = 1u << (r - c * kGroupRows);
      for (uint32_t j = e + 1; j < lim; ++j) {
        const uint32_t kj = s_k[pidx(j + 1)];
        const uint32_t rj = s_r[pidx(j + 1)];
        const uint32_t cj = rj / kGroupRows;
        if (kj != k || cj != c) break;
        lit |= 1u << (rj - cj * kGroupRows);
      }
      if ((segs >> i) & 1u) {
        const uint32_t d = dpre + ls++;
        out_keys[d] = k;
        out_offsets[d] = wpre + lw;
      }
      if (fill[i]) s_words[lw++] = fill[i];
      s_words[lw++] = lit;
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < tile_words; i += kEncBlock) out_words[wpre + i] = s_words[i];

  const uint32_t ntiles = (n + kEncTile - 1) / kEncTile;
  if (tile == ntiles - 1 && tid == 0) {
    const uint32_t D = dpre + tile_segs, W = wpre + tile_words;
    out_offsets[D] = W;
    *len_keys = D;
    *len_offsets = (uint64_t)D + 1;
    *len_words = W;
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
  const uint32_t grid = n ? (uint32_t)((n + kEncTile - 1) / kEncTile) : 1u;
  LbArgs lb;
  if (!env.lookback(2ull * grid, grid, &lb)) return env.fail(kErrOom, "wah_encode_sorted: look-back");
  env.prof_begin("wah_encode");
  k_wah_encode<<<dim3(grid), dim3(kEncBlock), 0, env.stream()>>>(skeys, srows, (uint32_t)n, keys, offsets, words,
                                                                d_len_keys, d_len_offsets, d_len_words, lb);
  env.prof_end("wah_encode");
  return check_launch(env, "wah_encode launch");
}

}  // namespace ka
