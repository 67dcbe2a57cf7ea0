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
// and e emits grp(e) + gap(e) words and seg(e) values.  So the encoding is one
// single-pass kernel over tiles of kEncTile pairs, k_wah_write: each tile
// counts its words and values, publishes both counts, finds the counts of all
// earlier tiles by decoupled look-back (one status chain for words, one for
// values; a silent predecessor is counted from its input by the waiting wave)
// and writes its words and lookup-table entries; the last tile writes W, D,
// offsets[D] and the three output lengths.  The sorted pairs are read once.
// A group spans at most 31 sorted elements (rows are distinct), so a tile
// finishes a group that runs past its end by reading at most 30 elements
// ahead (kLook).  Words are staged in LDS (over the staged input, which is
// dead by then) and written out by consecutive work-items.  Sorted keys are
// uint32, or uint16 when every value is below 2^16 (the index build's
// narrow-key sort).
#include "common.hpp"

namespace ka {
namespace {

// 1024 work-items x 8 elements: a tile of 8192 pairs, two work-groups of 16
// waves per CU (bound by LDS; 63 VGPRs).  The look-back's latency (a few
// device-coherent round trips, about 0.75 us each) is paid once per tile while
// the tile's work-group waits, and the LDS sweeps stall on bank conflicts:
// twice the waves of 512 x 16 hide both better, 206 -> 181 us on 2^26 Zipf
// pairs and 324 -> 225 us on uniform 16-bit ones (the batched build of 4096
// requests: +0.8%).  Tiles of 4096 pairs paid the look-back twice as often
// (244 against 228 us at 512 x 16); 16384-pair tiles (one work-group per CU)
// took 308 us.
constexpr int kEncBlock = 1024;
#ifndef KA_ENC_ITEMS
#define KA_ENC_ITEMS 8
#endif
constexpr int kEncItems = KA_ENC_ITEMS;
constexpr int kEncTile = kEncBlock * kEncItems;  // 8192 pairs
constexpr int kVecs = kEncTile / 4 / kEncBlock;  // 16-byte loads per work-item and array
constexpr int kLook = 32;                        // >= 30 elements of look-ahead
constexpr int kStage = kEncTile + kLook;         // staged elements (the look-behind is kept apart)
constexpr uint32_t kGroupRows = 31;
constexpr uint32_t kFill = 0x80000000u;

// Padded LDS index: four spare words after every 64 elements.  Groups of 4
// elements stay 16-byte aligned, so the tile is staged with conflict-free
// 16-byte writes (work-item t writes elements 4t..4t+3); a work-item reads its
// 8 consecutive elements with two 16-byte reads, and the 16 work-items served
// together (starting 32 bytes apart, plus 16 after every eighth) cover all 64
// banks once.
__device__ __forceinline__ uint32_t pidx(uint32_t i) { return i + 4 * (i >> 6); }
constexpr int kStagePadded = kStage + 4 * (kStage / 64) + 4;
static_assert(kEncItems == 8, "one padded run of 8 elements per work-item");
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
template <bool kVec, class KeyT>
__device__ __forceinline__ void load_pairs(const KeyT* __restrict__ skeys, const uint32_t* __restrict__ srows,
                                           uint32_t b, uint32_t len, uint32_t tid, uint32_t (&vk)[kVecs][4],
                                           uint32_t (&vr)[kVecs][4]) {
  if (kVec && len == (uint32_t)kEncTile) {
#pragma unroll
    for (int j = 0; j < kVecs; ++j) {
      const uint32_t q = j * kEncBlock + tid;
      load_key4(skeys + b, q, vk[j]);
      const u32x4 c = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(srows + b) + q);
      vr[j][0] = c.x, vr[j][1] = c.y, vr[j][2] = c.z, vr[j][3] = c.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < kVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t i = 4 * (j * kEncBlock + tid) + c;
        vk[j][c] = i < len ? (uint32_t)skeys[b + i] : 0u;
        vr[j][c] = i < len ? srows[b + i] : 0u;
      }
  }
}

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

// Words and values that tile u emits, counted from its input by one wave --
// the look-back's fallback for a predecessor that has not published yet.  Lane
// l takes 64 consecutive elements.
template <class KeyT>
__device__ LbPairSum wave_tile_count(const KeyT* __restrict__ skeys, const uint32_t* __restrict__ srows, uint32_t n,
                                     uint32_t u, BatchRows br) {
  constexpr uint32_t kPer = kEncTile / 64;
  const uint32_t b = u * kEncTile;
  const uint32_t end = min(b + (uint32_t)kEncTile, n);
  const uint32_t e0 = b + lane_id() * kPer;
  uint32_t nw = 0, ns = 0;
  if (e0 < end) {
    uint32_t kp = 0, rp = 0;
    if (e0 > 0) {
      kp = skeys[e0 - 1];
      rp = br.local(kp, srows[e0 - 1]);
    }
    const uint32_t e1 = min(e0 + kPer, end);
    for (uint32_t e = e0; e < e1; ++e) {
      const uint32_t k = skeys[e], r = br.local(k, srows[e]);
      element_counts(k, r, kp, rp, e == 0, nw, ns);
      kp = k;
      rp = r;
    }
  }
  return {wave_sum(nw), wave_sum(ns)};
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

// Rejection of the whole input, decided by earlier kernels: the encoding is
// void when (*flag >> shift) != 0 (a value at or above 2^shift), and every
// output length is then 0.
struct Reject {
  const uint32_t* flag;  // null: never
  uint32_t shift;
  __device__ __forceinline__ bool operator()() const { return flag && shift < 32 && (*flag >> shift) != 0u; }
};

// ---------------------------------------------------------------------------------
// write: literals, fills and lookup-table entries of one tile
// ---------------------------------------------------------------------------------
// status[kLbSpread * tile]: the tile's (words, values) look-back word, zeroed
// before the launch.
template <bool kVec, class KeyT>
__global__ __launch_bounds__(kEncBlock, 8) void k_wah_write(const KeyT* __restrict__ skeys,
                                                         const uint32_t* __restrict__ srows, uint32_t n_cap,
                                                         const uint64_t* __restrict__ d_n,
                                                         uint64_t* __restrict__ status, uint32_t spin_limit,
                                                         uint32_t* __restrict__ out_keys,
                                                         uint32_t* __restrict__ out_offsets,
                                                         uint32_t* __restrict__ out_words, BatchRows br, Reject rej,
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
  // n_cap pairs, or the count written on the device by an earlier stage: the
  // grid then covers the capacity and the tiles past the count leave at once
  // (tile 0 of an empty input writes the empty index).
  const uint32_t n = (uint32_t)device_count(n_cap, d_n);
  if (base >= n) {
    if (tile == 0 && tid == 0) {
      out_offsets[0] = 0;
      *len_keys = 0;
      *len_offsets = 1;
      *len_words = 0;
    }
    return;
  }
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
      xk = ok ? (uint32_t)skeys[g] : 0u;
      xr = ok ? br.local(xk, srows[g]) : 0u;
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
  // The element before this work-item's first: the previous work-item's last
  // (a shuffle; lane 0 reads it from LDS: the wave before, or the look-behind).
  const uint32_t lane = lane_id();
  uint32_t kprev = (uint32_t)__shfl_up((int)key[kEncItems - 1], 1);
  uint32_t cprev = (uint32_t)__shfl_up((int)grp_of[kEncItems - 1], 1);
  if (lane == 0) {
    kprev = tid ? s_k[pidx(e0 - 1)] : s_behind[0];
    cprev = (tid ? s_r[pidx(e0 - 1)] : s_behind[1]) / kGroupRows;
  }

  // ---- group and value heads, words and values emitted ------------------------------
  uint32_t heads = 0, segs = 0, gaps = 0;  // bit i: element i starts a group / a value / has a fill
  const bool first_of_input = base + e0 == 0u;  // this work-item's element 0 is the input's first
#pragma unroll
  for (int i = 0; i < kEncItems; ++i) {
    const uint32_t c = grp_of[i];
    const uint32_t kp = i ? key[i - 1] : kprev;
    const uint32_t cp = i ? grp_of[i - 1] : cprev;
    const bool seg = key[i] != kp || (i == 0 && first_of_input);
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
  const uint32_t tile_nw = packed_total & 0xFFFFu, tile_ns = packed_total >> 16;

  // ---- publish the tile's counts at once: successors find them while this
  // tile builds its words --------------------------------------------------------------
  if (tid == 0)
    lb_publish_raw(status + kLbSpread * tile,
                   lb_pack_pair(tile_nw, tile_ns, tile == 0 ? kLbInclusive : kLbAggregate));

  // ---- the last group may run past this work-item's elements (at most 30
  // further elements): collect its bits now.  They are the elements of the next
  // work-items before their first group head ("lead"): a group holds at most 31
  // elements, so it reaches at most four work-items further, and the fourth
  // one has a head.  Shuffles within the wave; the wave's last four lanes read
  // ahead in LDS (the next wave's elements, or the look-ahead).  Lanes with
  // invalid elements have no head and no lead bits, which ends a group at the
  // tile's (and the input's) end.
  const uint32_t lead_n = heads ? (uint32_t)__builtin_ctz(heads) : (uint32_t)kEncItems;
  uint32_t lead = 0;
#pragma unroll
  for (int i = 0; i < kEncItems; ++i)
    if ((uint32_t)i < lead_n) lead |= (1u << bit_of[i]) & ~kFill;  // bit 31 marks invalid elements
  const uint32_t lead1 = (uint32_t)__shfl_down((int)lead, 1), lead2 = (uint32_t)__shfl_down((int)lead, 2);
  const uint32_t lead3 = (uint32_t)__shfl_down((int)lead, 3), lead4 = (uint32_t)__shfl_down((int)lead, 4);
  const uint32_t nh = heads == 0u ? 1u : 0u;
  const uint32_t nohead1 = (uint32_t)__shfl_down((int)nh, 1), nohead2 = (uint32_t)__shfl_down((int)nh, 2);
  const uint32_t nohead3 = (uint32_t)__shfl_down((int)nh, 3);
  uint32_t tail = 0;
  if (e0 + kEncItems <= tile_n) {
    if (lane < 60) {
      tail = lead1 | (nohead1 ? (lead2 | (nohead2 ? (lead3 | (nohead3 ? lead4 : 0u)) : 0u)) : 0u);
    } else {
      const uint32_t kl = key[kEncItems - 1], cl = grp_of[kEncItems - 1];
      for (uint32_t j = e0 + kEncItems; j < avail; ++j) {
        const uint32_t kj = s_k[pidx(j)];
        const uint32_t rj = s_r[pidx(j)];
        const uint32_t cj = rj / kGroupRows;
        if (kj != kl || cj != cl) break;
        tail |= 1u << (rj - cj * kGroupRows);
      }
    }
  }
  __syncthreads();  // the staged input is dead from here on

  // ---- one backward sweep: literals (OR of the group's bits) and fills, placed in
  // LDS from the end of this work-item's words --------------------------------------
  const uint32_t wbeg = packed_pre & 0xFFFFu;  // this work-item's first word in the tile
  {
    uint32_t w = wbeg + nw;  // one past this work-item's last word
    uint32_t acc = tail;
#pragma unroll
    for (int i = kEncItems - 1; i >= 0; --i) {
      acc |= 1u << bit_of[i];
      if ((heads >> i) & 1u) {
        s_words[--w] = acc & ~kFill;  // drops the bit 31 of elements past the tile's end
        acc = 0;
        if ((gaps >> i) & 1u) {
          const uint32_t cp = i ? grp_of[i - 1] : cprev;
          s_words[--w] = kFill | (((segs >> i) & 1u) ? grp_of[i] : grp_of[i] - cp - 1u);
        }
      }
    }
  }

  // ---- the tile's first word and value: look back over the earlier tiles (wave 0)
  if (tid < 64) {
    LbPairSum pre{0u, 0u};
    if (tile > 0) {
      pre = lb_lookback_st<kLbSpread>(status, tile, LbPair{}, spin_limit,
                                      [&](uint32_t u) { return wave_tile_count(skeys, srows, n, u, br); });
      if (tid == 0)
        lb_publish_raw(status + kLbSpread * tile, lb_pack_pair(pre.a + tile_nw, pre.b + tile_ns, kLbInclusive));
    }
    if (tid == 0) {
      s_pre[0] = pre.a;
      s_pre[1] = pre.b;
    }
  }
  __syncthreads();
  const uint32_t wpre = s_pre[0], dpre = s_pre[1];

  // ---- words, then the lookup-table entries of the values starting here ----------------
  // Four words per work-item and step: an aligned 16-byte LDS read and a
  // 16-byte global store at word alignment (wpre is any word): a quarter of the
  // store instructions of word-sized stores (204 against 215 us per 2^26
  // Zipf pairs).
  {
    const uint32_t nv = tile_nw / 4;
    for (uint32_t v = tid; v < nv; v += kEncBlock)
      *reinterpret_cast<u32x4w*>(out_words + wpre + 4 * v) = *reinterpret_cast<const u32x4*>(s_words + 4 * v);
    if (tid < tile_nw - 4 * nv) out_words[wpre + 4 * nv + tid] = s_words[4 * nv + tid];
  }
  if (segs) {
    const uint32_t ls = packed_pre >> 16;  // tile-local index of this work-item's first value
#pragma unroll
    for (int i = 0; i < kEncItems; ++i) {
      if ((segs >> i) & 1u) {
        const uint32_t below = (1u << i) - 1u;
        const uint32_t d = dpre + ls + (uint32_t)__popc(segs & below);
        out_keys[d] = key[i];
        out_offsets[d] = wpre + wbeg + (uint32_t)__popc(heads & below) + (uint32_t)__popc(gaps & below);
      }
    }
  }
  if (base + tile_n == n && tid == 0) {  // the last tile: totals and lengths
    const uint32_t D = dpre + tile_ns, W = wpre + tile_nw;
    out_offsets[D] = W;
    const bool void_ = rej();
    *len_keys = void_ ? 0u : D;
    *len_offsets = void_ ? 0u : (uint64_t)D + 1;
    *len_words = void_ ? 0u : W;
  }
}

// Zeroes the encoder's status words (ntiles of them, kLbSpread apart) before
// the write kernel.
__global__ void k_wah_clear(uint64_t* __restrict__ status, uint32_t ntiles) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntiles) status[kLbSpread * i] = 0ull;
}

template <class KeyT>
int encode_impl(Env& env, const KeyT* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys, uint32_t* offsets,
                uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets, uint64_t* d_len_words,
                const uint32_t* req_base, uint32_t req_shift, const uint32_t* reject_flag, uint32_t reject_shift,
                const uint64_t* d_n) {
  if (!offsets || !d_len_keys || !d_len_offsets || !d_len_words)
    return env.fail(kErrArg, "wah_encode_sorted: null output");
  if (n >= (1ull << 30)) return env.fail(kErrArg, "wah_encode_sorted: n must be below 2^30");
  if (n && (!skeys || !srows || !keys || !words)) return env.fail(kErrArg, "wah_encode_sorted: null buffer");
  const uint32_t ntiles = (uint32_t)((n + kEncTile - 1) / kEncTile);
  if (!ntiles) {
    k_wah_empty<<<dim3(1), dim3(64), 0, env.stream()>>>(offsets, d_len_keys, d_len_offsets, d_len_words);
    return check_launch(env, "wah_empty launch");
  }
  // The (words, values) chain has no epoch: its own status words, zeroed here.
  uint64_t* status = static_cast<uint64_t*>(env.scratch(8ull * kLbSpread * ntiles));
  if (!status) return env.fail(kErrOom, "wah_encode_sorted: look-back status words");
  int rc;
  k_wah_clear<<<dim3((ntiles + 255) / 256), dim3(256), 0, env.stream()>>>(status, ntiles);
  if ((rc = check_launch(env, "wah_clear launch"))) return rc;
  constexpr uintptr_t kKeyAlign = sizeof(KeyT) == 4 ? 15u : 7u;
  const bool vec = ((reinterpret_cast<uintptr_t>(skeys) & kKeyAlign) | (reinterpret_cast<uintptr_t>(srows) & 15u)) == 0;
  const BatchRows br{req_base, req_shift};
  const Reject rej{reject_flag, reject_shift};
  const uint32_t nn = (uint32_t)n;
  env.prof_begin("wah_write");
  if (vec)
    k_wah_write<true, KeyT><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(
        skeys, srows, nn, d_n, status, env.spin_limit(), keys, offsets, words, br, rej, d_len_keys, d_len_offsets,
        d_len_words);
  else
    k_wah_write<false, KeyT><<<dim3(ntiles), dim3(kEncBlock), 0, env.stream()>>>(
        skeys, srows, nn, d_n, status, env.spin_limit(), keys, offsets, words, br, rej, d_len_keys, d_len_offsets,
        d_len_words);
  env.prof_end("wah_write");
  return check_launch(env, "wah_write launch");
}

}  // namespace

int launch_wah_encode(Env& env, const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                      uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                      uint64_t* d_len_words, const uint32_t* req_base, uint32_t req_shift,
                      const uint32_t* reject_flag, uint32_t reject_shift, const uint64_t* d_n) {
  return encode_impl(env, skeys, srows, n, keys, offsets, words, d_len_keys, d_len_offsets, d_len_words, req_base,
                     req_shift, reject_flag, reject_shift, d_n);
}

int launch_wah_encode16(Env& env, const uint16_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                        uint32_t* offsets, uint32_t* words, uint64_t* d_len_keys, uint64_t* d_len_offsets,
                        uint64_t* d_len_words, const uint32_t* reject_flag, uint32_t reject_shift,
                        const uint64_t* d_n) {
  return encode_impl(env, skeys, srows, n, keys, offsets, words, d_len_keys, d_len_offsets, d_len_words, nullptr, 32u,
                     reject_flag, reject_shift, d_n);
}

}  // namespace ka
