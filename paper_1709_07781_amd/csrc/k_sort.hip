// Stable LSB radix sort of (uint32 key, uint32 row) pairs by key -- parts 1
// and 2 of the WAH index build (Sec. 4.1: tag every value with its input
// position, then sort by value; Sec. 4.2 sorts with a radix sort).
//
// 8-bit digits, up to four passes, each a reduce-then-scan over tiles of
// kTile keys -- no work-group ever waits for another one's tile:
//  * k_radix_count (cooperative launch, a few hundred work-groups, each owning
//    a contiguous range of tiles) counts every tile's digits into a table and
//    sums its range; after one grid barrier each work-group turns its tiles'
//    counts into global offsets: the digit's start (exclusive prefix over
//    digits of the digit totals) plus the counts of all earlier tiles.  The
//    pass-0 instance also forms the OR and the AND of all keys for the sort
//    plan: a pass whose digit is the same in every key (equal in the OR and
//    the AND) is the identity of a stable sort and is skipped, so 16-bit keys
//    cost two passes.
//  * k_radix_scatter (one work-group per tile) ranks its keys by digit inside
//    each wave with an LDS match (every lane ORs its lane bit into a 64-bit
//    mask per digit and reads back the mask of its digit, so equal keys keep
//    their order), reorders the tile by digit in LDS and writes each digit's
//    run to its offset from the table, consecutive work-items writing
//    consecutive addresses.
// The first active pass reads the input (and makes row ids 0..n-1 when no rows
// are given), later ones read the previous active pass's output, and the last
// active pass writes the caller's buffers.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

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
constexpr int kBlock = KA_SORT_BLOCK;
constexpr int kWaves = kBlock / 64;
constexpr int kItems = KA_SORT_ITEMS;
constexpr int kTile = kBlock * kItems;  // 8192 keys per tile
constexpr int kCountVecs = kTile / 4 / kBlock;

}  // namespace

// The sort plan, written by the pass-0 count kernel.
struct SortPlan {
  uint32_t active;  // bit p: pass p moves data
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

struct PassIo {
  const uint32_t* src_keys;
  const uint32_t* src_rows;
  uint32_t* dst_keys;
  uint32_t* dst_rows;
  bool implicit_rows;
};

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
// the first active lane's bin (the common case for skewed or high digits).
__device__ __forceinline__ void lds_add_aggregated(uint32_t* bins, uint32_t d, bool valid) {
  const uint64_t active = __ballot(valid);
  if (!active) return;
  const uint32_t first_lane = (uint32_t)__builtin_ctzll(active);
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, (int)first_lane);
  const uint64_t same = __ballot(valid && d == d0);
  if (lane_id() == first_lane) atomicAdd(&bins[d0], (uint32_t)__popcll(same));
  if (valid && d != d0) atomicAdd(&bins[d], 1u);
}

// ---------------------------------------------------------------------------------
// count: per-tile digit counts -> per-tile digit offsets
// ---------------------------------------------------------------------------------
constexpr int kPartStride = kRadix + 2;  // per work-group: digit counts, then OR and AND of its keys

template <bool kFirst>
__global__ __launch_bounds__(kBlock) void k_radix_count(PassBuffers buf, SortPlan* __restrict__ plan,
                                                        uint32_t* __restrict__ table, uint32_t* __restrict__ part,
                                                        uint32_t pass, uint32_t n) {
  __shared__ uint32_t s_tile[kWaves][kRadix];  // per-wave counts of the current tile
  __shared__ uint32_t s_acc[kRadix];           // this work-group's counts over its tiles
  __shared__ uint32_t s_scan[kWaves];
  __shared__ uint32_t s_or[kWaves], s_and[kWaves];
  const uint32_t tid = threadIdx.x, w = tid / 64;

  uint32_t active = 1u;
  if (!kFirst) {
    active = plan->active;
    if (!((active >> pass) & 1u)) return;  // uniform: no work-group reaches the grid barrier
  }
  const uint32_t* keys = kFirst ? buf.keys_in : pass_io(buf, active, pass).src_keys;
  const uint32_t shift = pass * kRadixBits;
  const uint32_t ntiles = (n + kTile - 1) / kTile;
  const uint32_t G = gridDim.x, b = blockIdx.x;
  const uint32_t t0 = (uint32_t)((uint64_t)b * ntiles / G), t1 = (uint32_t)((uint64_t)(b + 1) * ntiles / G);
  const bool vec = (reinterpret_cast<uintptr_t>(keys) & 15u) == 0;

  // Keys of a tile: element 4 (j * kBlock + tid) + c in slot (j, c).
  auto fetch = [&](uint32_t t, uint32_t (&k)[kCountVecs][4]) {
    const uint32_t base = t * kTile;
    const uint32_t len = t < t1 ? min((uint32_t)kTile, n - base) : 0u;
#pragma unroll
    for (int j = 0; j < kCountVecs; ++j) {
      const uint32_t e = 4 * (j * kBlock + tid);
      if (vec && e + 4 <= len) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(keys + base + e));
        k[j][0] = v.x, k[j][1] = v.y, k[j][2] = v.z, k[j][3] = v.w;
      } else {
#pragma unroll
        for (int c = 0; c < 4; ++c) k[j][c] = e + c < len ? keys[base + e + c] : 0u;
      }
    }
  };

  if (tid < kRadix) s_acc[tid] = 0;
  uint32_t kor = 0, kand = ~0u;
  // Two tiles of keys are in flight while one is counted.
  uint32_t cur[kCountVecs][4], nxt[kCountVecs][4];
  fetch(t0, cur);
  fetch(t0 + 1, nxt);
  for (uint32_t t = t0; t < t1; ++t) {
    for (int i = tid; i < kWaves * kRadix; i += kBlock) (&s_tile[0][0])[i] = 0;
    uint32_t nxt2[kCountVecs][4];
    fetch(t + 2, nxt2);
    __syncthreads();
    const uint32_t len = min((uint32_t)kTile, n - t * kTile);
#pragma unroll
    for (int j = 0; j < kCountVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool valid = 4 * (j * kBlock + tid) + c < len;
        lds_add_aggregated(s_tile[w], (cur[j][c] >> shift) & (kRadix - 1), valid);
        if (kFirst && valid) {
          kor |= cur[j][c];
          kand &= cur[j][c];
        }
      }
    __syncthreads();
    if (tid < kRadix) {
      uint32_t c = 0;
#pragma unroll
      for (int ww = 0; ww < kWaves; ++ww) c += s_tile[ww][tid];
      table[(uint64_t)t * kRadix + tid] = c;
      s_acc[tid] += c;
    }
#pragma unroll
    for (int j = 0; j < kCountVecs; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        cur[j][c] = nxt[j][c];
        nxt[j][c] = nxt2[j][c];
      }
    __syncthreads();  // s_tile is cleared again for the next tile
  }
  uint32_t* mine = part + (uint64_t)b * kPartStride;
  if (tid < kRadix) mine[tid] = s_acc[tid];
  if (kFirst) {
    // OR and AND of this work-group's keys: a pass moves data unless its digit
    // is the same in every key, i.e. the same in the OR and the AND.
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      kor |= (uint32_t)__shfl_xor((int)kor, off);
      kand &= (uint32_t)__shfl_xor((int)kand, off);
    }
    if (lane_id() == 0) {
      s_or[w] = kor;
      s_and[w] = kand;
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t o = 0, a = ~0u;
      for (int ww = 0; ww < kWaves; ++ww) {
        o |= s_or[ww];
        a &= s_and[ww];
      }
      mine[kRadix] = o;
      mine[kRadix + 1] = a;
    }
  }
  cooperative_groups::this_grid().sync();

  // ---- every work-group: the start of its range for each digit ------------------
  // Work-item (q, d) sums the partials of every fourth work-group for digit d;
  // the loads are independent and unrolled so that many are in flight.
  uint32_t tot = 0, carry = 0;
  {
    constexpr uint32_t kQ = kBlock / kRadix;  // work-items per digit
    static_assert(2 * kQ <= kWaves, "quarter sums fit in s_tile");
    const uint32_t d = tid & (kRadix - 1), q = tid / kRadix;
#pragma unroll 8
    for (uint32_t bb = q; bb < G; bb += kQ) {
      const uint32_t c = part[(uint64_t)bb * kPartStride + d];
      tot += c;
      carry += bb < b ? c : 0u;
    }
    __syncthreads();
    s_tile[q][d] = tot;  // s_tile is free again: reuse it for the partial sums
    s_tile[kQ + q][d] = carry;
    __syncthreads();
    if (tid < kRadix) {
      tot = 0;
      carry = 0;
#pragma unroll
      for (uint32_t k = 0; k < kQ; ++k) {
        tot += s_tile[k][tid];
        carry += s_tile[kQ + k][tid];
      }
    }
  }
  uint32_t total;
  const uint32_t start = block_excl_scan<kBlock>(tid < kRadix ? tot : 0u, s_scan, &total);
  if (kFirst && b == 0 && tid == 0) {
    uint32_t o = 0, a = ~0u;
    for (uint32_t bb = 0; bb < G; ++bb) {
      o |= part[(uint64_t)bb * kPartStride + kRadix];
      a &= part[(uint64_t)bb * kPartStride + kRadix + 1];
    }
    const uint32_t diff = o ^ a;
    uint32_t act = 0;
    for (int p = 0; p < kPasses; ++p)
      if ((diff >> (p * kRadixBits)) & (kRadix - 1)) act |= 1u << p;
    if (act == 0) act = 1u << (kPasses - 1);  // all keys equal: one pass still moves them
    plan->active = act;
  }
  // ---- counts of this work-group's tiles -> offsets (16 tiles per round) -----------
  if (tid < kRadix) {
    uint32_t run = start + carry;
    for (uint32_t t = t0; t < t1; t += 16) {
      uint32_t c[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) c[j] = t + j < t1 ? table[(uint64_t)(t + j) * kRadix + tid] : 0u;
#pragma unroll
      for (int j = 0; j < 16; ++j)
        if (t + j < t1) {
          table[(uint64_t)(t + j) * kRadix + tid] = run;
          run += c[j];
        }
    }
  }
}

// ---------------------------------------------------------------------------------
// scatter: one tile, ranked in LDS, written to its offsets
// ---------------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_radix_scatter(PassBuffers buf, const SortPlan* __restrict__ plan,
                                                          const uint32_t* __restrict__ table, uint32_t pass,
                                                          uint32_t n) {
  // Reorder buffers; during ranking the key buffer holds the match masks.
  __shared__ __align__(16) uint32_t s_keys[kTile];
  __shared__ uint32_t s_rows[kTile];
  __shared__ uint16_t s_wcnt[kWaves][kRadix];  // per-wave digit counts, then per-wave offsets
  __shared__ uint32_t s_loff[kRadix];          // tile-local start of each digit
  __shared__ uint32_t s_dbase[kRadix];         // global start minus tile-local start
  __shared__ uint32_t s_scan[kWaves];
  static_assert(kWaves * kRadix * 2 <= kTile, "match masks fit in the key buffer");
  unsigned long long(*s_match)[kRadix] = reinterpret_cast<unsigned long long(*)[kRadix]>(&s_keys[0]);

  const uint32_t tid = threadIdx.x;
  const uint32_t active = plan->active;
  if (!((active >> pass) & 1u)) return;
  const PassIo io = pass_io(buf, active, pass);
  const uint32_t shift = pass * kRadixBits;
  const uint32_t tile = blockIdx.x;
  const uint32_t base = tile * kTile;
  const uint32_t tile_n = min((uint32_t)kTile, n - base);

  for (int i = tid; i < kWaves * kRadix; i += kBlock) {
    (&s_wcnt[0][0])[i] = 0;
    (&s_match[0][0])[i] = 0ull;
  }
  // ---- load: wave w owns 64*kItems consecutive elements -----------------------
  const uint32_t w = tid / 64, lane = lane_id();
  const uint32_t wbase = w * 64 * kItems;
  uint32_t key[kItems], row[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t local = wbase + i * 64 + lane;
    const uint32_t g = base + local;
    const bool valid = local < tile_n;
    key[i] = valid ? __builtin_nontemporal_load(io.src_keys + g) : 0u;
    row[i] = valid ? (io.implicit_rows ? g : __builtin_nontemporal_load(io.src_rows + g)) : 0u;
  }
  __syncthreads();

  // ---- rank inside the wave: peers = lanes with the same digit ----------------
  const uint64_t lt = lanemask_lt();
  uint32_t rank[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool valid = wbase + i * 64 + lane < tile_n;
    const uint32_t d = (key[i] >> shift) & (kRadix - 1);
    uint32_t r = 0;
    if (valid) {
      atomicOr(&s_match[w][d], 1ull << lane);
      const uint64_t peers = s_match[w][d];
      const uint32_t below = (uint32_t)__popcll(peers & lt);
      const uint32_t old = s_wcnt[w][d];
      if (below == 0) {
        s_wcnt[w][d] = (uint16_t)(old + (uint32_t)__popcll(peers));
        s_match[w][d] = 0ull;
      }
      r = old + below;
    }
    rank[i] = r;
  }
  __syncthreads();

  // ---- per digit: tile-local offsets and global destinations ------------------
  uint32_t tile_count = 0;
  if (tid < kRadix) {
#pragma unroll
    for (int ww = 0; ww < kWaves; ++ww) {
      const uint32_t c = s_wcnt[ww][tid];
      s_wcnt[ww][tid] = (uint16_t)tile_count;
      tile_count += c;
    }
  }
  uint32_t total;
  const uint32_t loff = block_excl_scan<kBlock>(tid < kRadix ? tile_count : 0u, s_scan, &total);
  if (tid < kRadix) {
    s_loff[tid] = loff;
    s_dbase[tid] = table[(uint64_t)tile * kRadix + tid] - loff;
  }
  __syncthreads();

  // ---- reorder the tile by digit in LDS ---------------------------------------
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (wbase + i * 64 + lane < tile_n) {
      const uint32_t d = (key[i] >> shift) & (kRadix - 1);
      const uint32_t pos = s_loff[d] + s_wcnt[w][d] + rank[i];
      s_keys[pos] = key[i];
      s_rows[pos] = row[i];
    }
  }
  __syncthreads();

  // ---- write each digit's run to its global place ------------------------------
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t p = i * kBlock + tid;
    if (p < tile_n) {
      const uint32_t k = s_keys[p];
      const uint32_t g = s_dbase[(k >> shift) & (kRadix - 1)] + p;
      io.dst_keys[g] = k;
      io.dst_rows[g] = s_rows[p];
    }
  }
}

}  // namespace

int launch_radix_sort_pairs(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys,
                            uint32_t* srows, uint64_t n) {
  if (n == 0) return kOk;
  if (!keys || !skeys || !srows) return env.fail(kErrArg, "radix_sort: null buffer");
  if (n >= (1ull << 31)) return env.fail(kErrArg, "radix_sort: n must be below 2^31");
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
  const int cap = coresident_blocks(reinterpret_cast<const void*>(&k_radix_count<true>), kBlock);
  if (cap <= 0) return env.fail(kErrLaunch, "radix_sort: cooperative launch not available");
  const uint32_t G = (uint32_t)std::min<int>(cap, (int)ntiles);
  uint32_t* part = static_cast<uint32_t*>(env.scratch((uint64_t)G * kPartStride * 4));
  if (!buf.keys_b || !buf.rows_b || !table || !part) return env.fail(kErrOom, "radix_sort: scratch buffers");

  for (uint32_t pass = 0; pass < (uint32_t)kPasses; ++pass) {
    int rc;
    if (pass == 0)
      rc = launch_persistent(env, "radix_count0", k_radix_count<true>, G, (uint32_t)kBlock, buf, plan, table, part,
                             pass, nn);
    else
      rc = launch_persistent(env, "radix_count", k_radix_count<false>, G, (uint32_t)kBlock, buf, plan, table, part,
                             pass, nn);
    if (rc) return rc;
    env.prof_begin("radix_scatter");
    k_radix_scatter<<<dim3(ntiles), dim3(kBlock), 0, env.stream()>>>(buf, static_cast<const SortPlan*>(plan), table,
                                                                     pass, nn);
    env.prof_end("radix_scatter");
    rc = check_launch(env, "radix_scatter launch");
    if (rc) return rc;
  }
  return kOk;
}

}  // namespace ka
