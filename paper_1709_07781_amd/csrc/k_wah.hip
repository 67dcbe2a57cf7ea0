// WAH encoding of sorted (value, row) pairs -- parts 3 to 6 of the index build
// of Sec. 4.1:
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
// What element e contributes depends only on e and its predecessor e - 1:
//   seg(e) = e is the first element of its value,
//   grp(e) = seg(e) or chunk(e) != chunk(e - 1)   (e starts a group),
//   gap(e) = grp(e) and the fill before e is non-zero (chunk(e) != 0 for a
//            value's first group, chunk(e) != chunk(e - 1) + 1 otherwise),
// and e emits grp(e) + gap(e) words and seg(e) values.  So the encoding is a
// reduce-then-scan over tiles of kEncTile pairs, with no wait between tiles:
//   k_wah_count    counts each tile's words and values,
//   k_wah_groups   scans the tile counts inside groups of 1024 tiles and
//                  writes the group totals,
//   k_wah_write    adds the totals of the earlier groups to its tile's offset,
//                  re-derives the tile's groups and writes its words and
//                  lookup-table entries; the last tile writes W, D, offsets[D]
//                  and the three output lengths.
// A group spans at most 31 sorted elements (rows are distinct), so the write
// kernel finishes a group that runs past its tile by reading at most 30
// elements ahead (kLook).  Words are staged in LDS (over the staged input,
// which is dead by then) and written out by consecutive work-items.
#include "common.hpp"

namespace ka {
namespace {

constexpr int kEncBlock = 256;
#ifndef KA_ENC_ITEMS
#define KA_ENC_ITEMS 16
#endif
constexpr int kEncItems = KA_ENC_ITEMS;
constexpr int kEncTile = kEncBlock * kEncItems;  // 4096 pairs
constexpr int kVecs = kEncTile / 4 / kEncBlock;  // 16-byte loads per work-item and array
constexpr int kLook = 32;                        // >= 30 elements of look-ahead
constexpr int kStage = kEncTile + kLook;         // staged elements (the look-behind is kept apart)
constexpr uint32_t kGroupRows = 31;
constexpr uint32_t kFill = 0x80000000u;

// Padded LDS index: four spare words after every 64 elements.  Groups of 4
// elements stay 16-byte aligned, so the tile is staged with conflict-free
// 16-byte writes (work-item t writes elements 4t..4t+3); a work-item reads its
// 16 consecutive elements with 16-byte reads, and the 16 work-items served
// together (starting 64 bytes apart, plus 16 after every fourth) cover all 64
// banks once.
__device__ __forceinline__ uint32_t pidx(uint32_t i) { return i + 4 * (i >> 6); }
constexpr int kStagePadded = kStage + 4 * (kStage / 64) + 4;
static_assert(kEncItems == 16, "one padded run of 16 elements per work-item");
static_assert(2 * kEncTile <= 2 * kStagePadded, "word staging fits over the input staging");

// Words and values emitted by an element with key k and row r whose
// predecessor has key kp and row rp (first: no predecessor).
__device__ __forceinline__ void element_counts(uint32_t k, uint32_t r, uint32_t kp, uint32_t rp, bool first,
                                               uint32_t& nw, uint32_t& ns) {
  const uint32_t c = r / kGroupRows, cp = rp / kGroupRows;
  const bool seg = first || k != kp;
  const bool grp = seg || c != cp;
  const bool gap = grp && (seg ? c != 0u : c != cp + 1u);
  nw += (grp ? 1u : 0u) + (gap ? 1u : 0u);
  ns += seg ? 1u : 0u;
}

// Tile elements in registers: slot (j, c) of work-item tid holds element
// b + 4 (j * kEncBlock + tid) + c (0 beyond len).
template <bool kVec>
__device__ __forceinline__ void load_pairs(const uint32_t* __restrict__ skeys, const uint32_t* __restrict__ srows,
                                           uint32_t b, uint32_t len, uint32_t tid, uint32_t (&vk)[kVecs][4],
                                           uint32_t (&vr)[kVecs][4]) {
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
}

// ---------------------------------------------------------------------------------
// count: words and values emitted by each tile
// ---------------------------------------------------------------------------------
// Rows of a batch of requests sorted together are batch positions; the row
// inside the request is the position minus the request's first position,
// found from the request id in the key's high bits (key >> req_shift).
struct BatchRows {
  const uint32_t* req_base;  // null: rows are used as they are
  uint32_t req_shift;
  __device__ __forceinline__ uint32_t local(uint32_t key, uint32_t row) const {
    return req_base ? row - req_base[req_shift < 32 ? key >> req_shift : 0u] : row;
  }
};

template <bool kVec>
__global__ __launch_bounds__(kEncBlock) void k_wah_count(const uint32_t* __restrict__ skeys,
                                                         const uint32_t* __restrict__ srows, uint32_t n,
                                                         uint32_t* __restrict__ tile_words,
                                                         uint32_t* __restrict__ tile_values, BatchRows br) {
  __shared__ uint32_t s_w[kEncBlock / 64], s_s[kEncBlock / 64];
  const uint32_t tid = threadIdx.x, tile = blockIdx.x;
  const uint32_t b = tile * kEncTile;
  const uint32_t len = min((uint32_t)kEncTile, n - b);
  uint32_t vk[kVecs][4], vr[kVecs][4], pk[kVecs], pr[kVecs];
  load_pairs<kVec>(skeys, srows, b, len, tid, vk, vr);
  if (br.req_base) {
#pragma unroll
    for (int j = 0; j < kVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) vr[j][c] = br.local(vk[j][c], vr[j][c]);
  }
  // The predecessor of each vector's first element is the last element of the
  // lane before (a wave shuffle); lane 0 reads it from memory (it belongs to
  // another wave's vector or to the previous tile, and is served from cache).
  const uint32_t lane = lane_id();
#pragma unroll
  for (int j = 0; j < kVecs; ++j) {
    const uint32_t i = 4 * (j * kEncBlock + tid);
    pk[j] = (uint32_t)__shfl_up((int)vk[j][3], 1);
    pr[j] = (uint32_t)__shfl_up((int)vr[j][3], 1);
    if (lane == 0 && b + i > 0 && i < len) {
      pk[j] = skeys[b + i - 1];
      pr[j] = br.local(pk[j], srows[b + i - 1]);
    }
  }
  uint32_t nw = 0, ns = 0;
#pragma unroll
  for (int j = 0; j < kVecs; ++j)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t i = 4 * (j * kEncBlock + tid) + c;
      if (i < len)
        element_counts(vk[j][c], vr[j][c], c ? vk[j][c - 1] : pk[j], c ? vr[j][c - 1] : pr[j], b + i == 0, nw,
                       ns);
    }
  nw = wave_sum(nw);
  ns = wave_sum(ns);
  if (lane_id() == 0) {
    s_w[tid / 64] = nw;
    s_s[tid / 64] = ns;
  }
  __syncthreads();
  if (tid == 0) {
    uint32_t w = 0, s = 0;
#pragma unroll
    for (int i = 0; i < kEncBlock / 64; ++i) {
      w += s_w[i];
      s += s_s[i];
    }
    tile_words[tile] = w;
    tile_values[tile] = s;
  }
}

// ---------------------------------------------------------------------------------
// groups: tile counts -> offsets inside groups of kGroupTiles tiles, group totals
// ---------------------------------------------------------------------------------
constexpr int kGroupTiles = 1024;  // one work-item per tile of the group

// The write kernel adds the totals of the groups before its own (at most
// ntiles / kGroupTiles values), so no single work-group scans every tile.
__global__ __launch_bounds__(kGroupTiles) void k_wah_groups(uint32_t* __restrict__ tile_words,
                                                            uint32_t* __restrict__ tile_values, uint32_t ntiles,
                                                            uint32_t* __restrict__ group_words,
                                                            uint32_t* __restrict__ group_values) {
  __shared__ uint32_t s_a[kGroupTiles / 64], s_b[kGroupTiles / 64];
  const uint32_t t = blockIdx.x * kGroupTiles + threadIdx.x;
  const uint32_t w = t < ntiles ? tile_words[t] : 0u, v = t < ntiles ? tile_values[t] : 0u;
  uint32_t tw, tv;
  const uint32_t pw = block_excl_scan<kGroupTiles>(w, s_a, &tw);
  const uint32_t pv = block_excl_scan<kGroupTiles>(v, s_b, &tv);
  if (t < ntiles) {
    tile_words[t] = pw;
    tile_values[t] = pv;
  }
  if (threadIdx.x == 0) {
    group_words[blockIdx.x] = tw;
    group_values[blockIdx.x] = tv;
  }
}

// An empty input: D = 0, W = 0, offsets = [0].
__global__ void k_wah_empty(uint32_t* __restrict__ out_offsets, uint64_t* __restrict__ len_keys,
                            uint64_t* __restrict__ len_offsets, uint64_t* __restrict__ len_words) {
  if (threadIdx.x == 0) {
    out_offsets[0] = 0;
    *len_keys = 0;
    *len_offsets = 1;
    *len_words = 0;
  }
}

// ---------------------------------------------------------------------------------
// write: literals, fills and lookup-table entries of one tile
// ---------------------------------------------------------------------------------
template <bool kVec>
__global__ __launch_bounds__(kEncBlock, 4) void k_wah_write(const uint32_t* __restrict__ skeys,
                                                         const uint32_t* __restrict__ srows, uint32_t n,
                                                         const uint32_t* __restrict__ tile_words,
                                                         const uint32_t* __restrict__ tile_values,
                                                         const uint32_t* __restrict__ group_words,
                                                         const uint32_t* __restrict__ group_values,
                                                         uint32_t* __restrict__ out_keys,
                                                         uint32_t* __restrict__ out_offsets,
                                                         uint32_t* __restrict__ out_words, BatchRows br,
                                                         uint64_t* __restrict__ len_keys,
                                                         uint64_t* __restrict__ len_offsets,
                                                         uint64_t* __restrict__ len_words) {
  __shared__ __align__(16) uint32_t s_mem[2 * kStagePadded];
  __shared__ uint32_t s_scan[kEncBlock / 64];
  __shared__ uint32_t s_pre[2];
  __shared__ uint32_t s_behind[2];  // key and row of element base - 1
  uint32_t* s_k = s_mem;
  uint32_t* s_r = s_mem + kStagePadded;
  uint32_t* s_words = s_mem;  // after the literals are built

  const uint32_t tid = threadIdx.x, tile = blockIdx.x;
  const uint32_t base = tile * kEncTile;
  const uint32_t tile_n = min((uint32_t)kEncTile, n - base);
  const uint32_t avail = min((uint32_t)(kEncTile + kLook), n - base);  // readable from base on

  // ---- stage elements base .. base+kEncTile+kLook-1 into slots 0.. ---------------
  // Work-items 64..95 also load the look-ahead (slots kEncTile ..) and
  // work-item 96 the look-behind element base - 1.
  {
    uint32_t vk[kVecs][4], vr[kVecs][4];
    load_pairs<kVec>(skeys, srows, base, tile_n, tid, vk, vr);
    const bool extra = tid >= 64 && tid < 64 + kLook + 1;
    const int64_t g = tid == 64 + kLook ? (int64_t)base - 1 : (int64_t)base + kEncTile + (tid - 64);
    uint32_t xk = 0, xr = 0;
    if (extra) {
      const bool ok = g >= 0 && g < (int64_t)n;
      xk = ok ? skeys[g] : 0u;
      xr = ok ? br.local(xk, srows[g]) : 0u;
    }
    // This tile's first word and value: its offset inside its group plus the
    // totals of the groups before (wave 0, once the tile's loads are issued;
    // read after the next barrier).
    if (tid < 64) {
      const uint32_t grp = tile / kGroupTiles;
      uint32_t gw = 0, gv = 0;
      for (uint32_t j = tid; j < grp; j += 64) {
        gw += group_words[j];
        gv += group_values[j];
      }
      gw = wave_sum(gw);
      gv = wave_sum(gv);
      if (tid == 0) {
        s_pre[0] = gw + tile_words[tile];
        s_pre[1] = gv + tile_values[tile];
      }
    }
#pragma unroll
    for (int j = 0; j < kVecs; ++j) {
      const uint32_t sl = pidx(4 * (j * kEncBlock + tid));
      u32x4 k4, r4;
      k4.x = vk[j][0], k4.y = vk[j][1], k4.z = vk[j][2], k4.w = vk[j][3];
      r4.x = br.local(vk[j][0], vr[j][0]), r4.y = br.local(vk[j][1], vr[j][1]);
      r4.z = br.local(vk[j][2], vr[j][2]), r4.w = br.local(vk[j][3], vr[j][3]);
      *reinterpret_cast<u32x4*>(s_k + sl) = k4;
      *reinterpret_cast<u32x4*>(s_r + sl) = r4;
    }
    if (extra) {
      if (tid == 64 + kLook) {
        s_behind[0] = xk;
        s_behind[1] = xr;
      } else {
        const uint32_t sl = pidx((uint32_t)(kEncTile + (tid - 64)));
        s_k[sl] = xk;
        s_r[sl] = xr;
      }
    }
  }
  __syncthreads();
  const uint32_t wpre = s_pre[0], dpre = s_pre[1];

  // ---- this work-item's kEncItems consecutive elements, in registers: key, the
  // row's group (row / 31) and its bit inside the group; elements past the
  // tile's end get bit 31, which no literal keeps --------------------------------
  const uint32_t e0 = tid * kEncItems;
  const uint32_t nvalid = e0 < tile_n ? min(tile_n - e0, (uint32_t)kEncItems) : 0u;
  const uint32_t valid = nvalid >= 32u ? ~0u : (1u << nvalid) - 1u;  // bit i: element i exists
  uint32_t key[kEncItems], grp_of[kEncItems], bit_of[kEncItems];
#pragma unroll
  for (int q = 0; q < kEncItems / 4; ++q) {
    const u32x4 k4 = *reinterpret_cast<const u32x4*>(s_k + pidx(e0) + 4 * q);
    const u32x4 r4 = *reinterpret_cast<const u32x4*>(s_r + pidx(e0) + 4 * q);
    const uint32_t kk[4] = {k4.x, k4.y, k4.z, k4.w}, rr[4] = {r4.x, r4.y, r4.z, r4.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = 4 * q + c;
      key[i] = kk[c];
      grp_of[i] = rr[c] / kGroupRows;
      bit_of[i] = (valid >> i) & 1u ? rr[c] - grp_of[i] * kGroupRows : 31u;
    }
  }
  const uint32_t kprev = tid ? s_k[pidx(e0 - 1)] : s_behind[0];
  const uint32_t cprev = (tid ? s_r[pidx(e0 - 1)] : s_behind[1]) / kGroupRows;

  // ---- group and value heads, words and values emitted ------------------------------
  uint32_t heads = 0, segs = 0, gaps = 0;  // bit i: element i starts a group / a value / has a fill
#pragma unroll
  for (int i = 0; i < kEncItems; ++i) {
    const uint32_t c = grp_of[i];
    const uint32_t kp = i ? key[i - 1] : kprev;
    const uint32_t cp = i ? grp_of[i - 1] : cprev;
    const bool seg = key[i] != kp || (base + e0 + i) == 0;
    const bool grp = seg || c != cp;
    const bool gap = grp && (seg ? c != 0u : c != cp + 1u);
    heads |= (uint32_t)grp << i;
    segs |= (uint32_t)seg << i;
    gaps |= (uint32_t)gap << i;
  }
  heads &= valid;
  segs &= valid;
  gaps &= valid;
  const uint32_t nw = (uint32_t)__popc(heads) + (uint32_t)__popc(gaps);
  const uint32_t ns = (uint32_t)__popc(segs);
  // Both counts in one scan: words in the low half, values in the high half
  // (a tile emits at most 2*kEncTile words and kEncTile values).
  uint32_t packed_total;
  const uint32_t packed_pre = block_excl_scan<kEncBlock>((ns << 16) | nw, s_scan, &packed_total);
  const uint32_t tile_nw = packed_total & 0xFFFFu;

  // ---- the last group may run past this work-item's elements (at most 30
  // further elements, into the look-ahead): collect its bits now -------------------
  uint32_t tail = 0;
  if (e0 + kEncItems <= tile_n) {
    const uint32_t kl = key[kEncItems - 1], cl = grp_of[kEncItems - 1];
    for (uint32_t j = e0 + kEncItems; j < avail; ++j) {
      const uint32_t kj = s_k[pidx(j)];
      const uint32_t rj = s_r[pidx(j)];
      const uint32_t cj = rj / kGroupRows;
      if (kj != kl || cj != cl) break;
      tail |= 1u << (rj - cj * kGroupRows);
    }
  }
  __syncthreads();  // the staged input is dead from here on

  // ---- one backward sweep: literals (OR of the group's bits), fills and lookup-table
  // entries, placed from the end of this work-item's words --------------------------
  {
    uint32_t w = (packed_pre & 0xFFFFu) + nw;  // one past this work-item's last word
    const uint32_t ls = packed_pre >> 16;      // tile-local index of its first value
    uint32_t acc = tail;
#pragma unroll
    for (int i = kEncItems - 1; i >= 0; --i) {
      acc |= 1u << bit_of[i];
      if ((heads >> i) & 1u) {
        s_words[--w] = acc & ~kFill;  // drops the bit 31 of elements past the tile's end
        acc = 0;
        const bool seg = (segs >> i) & 1u;
        if ((gaps >> i) & 1u) {
          const uint32_t cp = i ? grp_of[i - 1] : cprev;
          s_words[--w] = kFill | (seg ? grp_of[i] : grp_of[i] - cp - 1u);
        }
        if (seg) {
          const uint32_t d = dpre + ls + (uint32_t)__popc(segs & ((1u << i) - 1u));
          out_keys[d] = key[i];
          out_offsets[d] = wpre + w;
        }
      }
    }
  }
  __syncthreads();
  for (uint32_t i = tid; i < tile_nw; i += kEncBlock) out_words[wpre + i] = s_words[i];
  if (base + tile_n == n && tid == 0) {  // the last tile: totals and lengths
    const uint32_t D = dpre + (packed_total >> 16), W = wpre + tile_nw;
    out_offsets[D] = W;
    *len_keys = D;
    *len_offsets = (uint64_t)D + 1;
    *len_words = W;
  }
}

}  // namespace

int launch_wah_encode(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                      uint64_t* d_len_words, const uint32_t* req_base, uint32_t req_shift) {
  if (!offsets || !d_len_keys || !d_len_offsets || !d_len_words)
    return env.fail(kErrArg, "wah_encode_sorted: null output");
  if (n >= (1ull << 30)) return env.fail(kErrArg, "wah_encode_sorted: n must be below 2^30");
  if (n && (!skeys || !srows || !keys || !words)) return env.fail(kErrArg, "wah_encode_sorted: null buffer");
  const uint32_t ntiles = (uint32_t)((n + kEncTile - 1) / kEncTile);
  const uint32_t nn = (uint32_t)n;
  uint32_t* tw = static_cast<uint32_t*>(env.scratch(4ull * (ntiles ? ntiles : 1)));
  uint32_t* tv = static_cast<uint32_t*>(env.scratch(4ull * (ntiles ? ntiles : 1)));
  const uint64_t ng = (ntiles + kGroupTiles - 1) / kGroupTiles;
  uint32_t* gw = static_cast<uint32_t*>(env.scratch(4ull * (ng ? ng : 1)));
  uint32_t* gv = static_cast<uint32_t*>(env.scratch(4ull * (ng ? ng : 1)));
  if (!tw || !tv || !gw || !gv) return env.fail(kErrOom, "wah_encode_sorted: tile counts");
  const bool vec = ((reinterpret_cast<uintptr_t>(skeys) | reinterpret_cast<uintptr_t>(srows)) & 15u) == 0;
  const BatchRows br{req_base, req_shift};
  int rc;
  if (ntiles) {
    env.prof_begin("wah_count");
    if (vec)
      k_wah_count<true><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(skeys, srows, nn, tw, tv, br);
    else
      k_wah_count<false><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(skeys, srows, nn, tw, tv, br);
    env.prof_end("wah_count");
    if ((rc = check_launch(env, "wah_count launch"))) return rc;
  }
  if (!ntiles) {
    k_wah_empty<<<dim3(1), dim3(64), 0, env.stream()>>>(offsets, d_len_keys, d_len_offsets, d_len_words);
    return check_launch(env, "wah_empty launch");
  }
  const uint32_t ngroups = (ntiles + kGroupTiles - 1) / kGroupTiles;
  env.prof_begin("wah_offsets");
  k_wah_groups<<<dim3(ngroups), dim3(kGroupTiles), 0, env.stream()>>>(tw, tv, ntiles, gw, gv);
  env.prof_end("wah_offsets");
  if ((rc = check_launch(env, "wah_groups launch"))) return rc;
  env.prof_begin("wah_write");
  if (vec)
    k_wah_write<true><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(
        skeys, srows, nn, tw, tv, gw, gv, keys, offsets, words, br, d_len_keys, d_len_offsets, d_len_words);
  else
    k_wah_write<false><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(
        skeys, srows, nn, tw, tv, gw, gv, keys, offsets, words, br, d_len_keys, d_len_offsets, d_len_words);
  env.prof_end("wah_write");
  if ((rc = check_launch(env, "wah_write launch"))) return rc;
  return kOk;
}

}  // namespace ka
