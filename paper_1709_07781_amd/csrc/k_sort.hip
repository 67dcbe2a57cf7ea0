// Stable LSB radix sort of (uint32 key, uint32 row) pairs by key -- parts 1
// and 2 of the WAH index build (Sec. 4.1: tag every value with its input
// position, then sort by value; Sec. 4.2 sorts with a radix sort).
//
// Structure (8-bit digits, up to 4 passes):
//  * k_radix_hist reads the keys once and builds the digit histograms of all
//    four passes (LDS sub-histograms per wave, wave-aggregated LDS atomics for
//    runs of equal digits, one global atomic per non-empty bin and work-group).
//  * k_radix_pass, once per digit position.  Every work-group derives the same
//    plan from the histograms: a pass whose digit is the same for all keys is
//    the identity of a stable sort and is skipped (so 16-bit keys cost two
//    passes), the first active pass reads the input (and makes row ids
//    0..n-1 when no rows are given), later ones read the previous active
//    pass's output, and the last active pass writes the caller's buffers.
//    Inside a pass a tile is ranked with wave64 ballots (peers with the same
//    digit within the wave, counted against lanes of lower index, so equal
//    keys keep their order), per-digit global offsets come from the upfront
//    histogram plus a decoupled look-back over the tile counts of earlier
//    tiles, and the tile is reordered through LDS so that consecutive
//    work-items write consecutive addresses of each digit's run.
#include "common.hpp"

namespace ka {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kPasses = 32 / kRadixBits;

constexpr int kHistBlock = 256;
constexpr int kHistWaves = kHistBlock / 64;

constexpr int kPassBlock = 512;
constexpr int kPassItems = 16;
constexpr int kPassWaves = kPassBlock / 64;
constexpr int kPassTile = kPassBlock * kPassItems;  // 8192 pairs
constexpr uint32_t kNoDigit = kRadix;               // marks elements past the end

// LDS add of 1 to bin d by every active lane, aggregated over lanes that share
// the first active lane's bin (the common case for skewed or high digits).
__device__ __forceinline__ void lds_add_aggregated(uint32_t* bins, uint32_t d, bool valid) {
  uint64_t active = __ballot(valid);
  if (!active) return;
  const uint32_t first_lane = (uint32_t)__builtin_ctzll(active);
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, (int)first_lane);
  const uint64_t same = __ballot(valid && d == d0);
  if (lane_id() == first_lane) atomicAdd(&bins[d0], (uint32_t)__popcll(same));
  if (valid && d != d0) atomicAdd(&bins[d], 1u);
}

__global__ __launch_bounds__(kHistBlock) void k_radix_hist(const uint32_t* __restrict__ keys, uint64_t n,
                                                           uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ hist_next) {
  __shared__ uint32_t s_bins[kHistWaves][kPasses][kRadix];
  uint32_t* flat = &s_bins[0][0][0];
  for (int i = threadIdx.x; i < kHistWaves * kPasses * kRadix; i += kHistBlock) flat[i] = 0;
  // The other histogram buffer is cleared here for the next sort on this
  // stream; the previous sort, which used it, has completed (stream order).
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kPasses * kRadix; i += kHistBlock) hist_next[i] = 0;
  __syncthreads();
  const uint32_t w = threadIdx.x / 64;
  const bool vec = (reinterpret_cast<uintptr_t>(keys) & 15u) == 0;
  const uint64_t nvec = (n + 3) / 4;
  for (uint64_t q = (uint64_t)blockIdx.x * kHistBlock + threadIdx.x; q - threadIdx.x < nvec;
       q += (uint64_t)gridDim.x * kHistBlock) {
    uint32_t k[4];
    bool valid[4];
    const uint64_t e = q * 4;
    if (vec && e + 4 <= n) {
      const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(keys + e));
      k[0] = v.x;
      k[1] = v.y;
      k[2] = v.z;
      k[3] = v.w;
#pragma unroll
      for (int j = 0; j < 4; ++j) valid[j] = true;
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        valid[j] = (q < nvec) && (e + j < n);
        k[j] = valid[j] ? keys[e + j] : 0u;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int p = 0; p < kPasses; ++p)
        lds_add_aggregated(s_bins[w][p], (k[j] >> (p * kRadixBits)) & (kRadix - 1), valid[j]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kPasses * kRadix; i += kHistBlock) {
    uint32_t sum = 0;
#pragma unroll
    for (int ww = 0; ww < kHistWaves; ++ww) sum += (&s_bins[ww][0][0])[i];
    if (sum) atomicAdd(&hist[i], sum);
  }
}

struct PassBuffers {
  const uint32_t* keys_in;
  const uint32_t* rows_in;  // null: rows are positions 0..n-1
  uint32_t* keys_a;         // caller's output (written by the last active pass)
  uint32_t* rows_a;
  uint32_t* keys_b;         // scratch ping-pong buffer
  uint32_t* rows_b;
};

__global__ __launch_bounds__(kPassBlock) void k_radix_pass(PassBuffers buf, const uint32_t* __restrict__ hist,
                                                           uint32_t pass, uint32_t n, LbArgs lb) {
  __shared__ uint32_t s_keys[kPassTile];
  __shared__ uint32_t s_rows[kPassTile];
  __shared__ uint32_t s_wcnt[kPassWaves][kRadix];  // per-wave digit counts, then per-wave offsets
  __shared__ uint32_t s_loff[kRadix];              // tile-local start of each digit
  __shared__ uint32_t s_dbase[kRadix];             // global start minus tile-local start
  __shared__ uint32_t s_scan[kPassBlock / 64];
  __shared__ uint32_t s_tile, s_full;

  const uint32_t tile = lb_take_tile(lb, &s_tile);
  const uint32_t tid = threadIdx.x;

  // ---- plan: a pass is active unless one digit holds all n keys -------------
  if (tid == 0) s_full = 0;
  __syncthreads();
  if (tid < kRadix) {
#pragma unroll
    for (int p = 0; p < kPasses; ++p)
      if (hist[p * kRadix + tid] == n) atomicOr(&s_full, 1u << p);
  }
  __syncthreads();
  uint32_t active = ~s_full & ((1u << kPasses) - 1);
  if (active == 0) active = 1u << (kPasses - 1);  // all keys equal: one pass still moves them
  if (!((active >> pass) & 1u)) return;
  const uint32_t later = (uint32_t)__popc(active >> pass);  // active passes from this one on
  const bool first = (active & ((1u << pass) - 1)) == 0;
  uint32_t* dst_keys = (later & 1u) ? buf.keys_a : buf.keys_b;
  uint32_t* dst_rows = (later & 1u) ? buf.rows_a : buf.rows_b;
  const uint32_t* src_keys = first ? buf.keys_in : (((later + 1) & 1u) ? buf.keys_a : buf.keys_b);
  const uint32_t* src_rows = first ? buf.rows_in : (((later + 1) & 1u) ? buf.rows_a : buf.rows_b);
  const bool implicit_rows = first && buf.rows_in == nullptr;
  const uint32_t shift = pass * kRadixBits;

  const uint32_t base = tile * kPassTile;
  if (base >= n) return;
  const uint32_t tile_n = min((uint32_t)kPassTile, n - base);

  for (int i = tid; i < kPassWaves * kRadix; i += kPassBlock) (&s_wcnt[0][0])[i] = 0;

  // ---- load: wave w owns 64*kPassItems consecutive elements ---------------
  const uint32_t w = tid / 64, lane = lane_id();
  const uint32_t wbase = w * 64 * kPassItems;
  uint32_t key[kPassItems], row[kPassItems], dig[kPassItems];
#pragma unroll
  for (int i = 0; i < kPassItems; ++i) {
    const uint32_t local = wbase + i * 64 + lane;
    const bool valid = local < tile_n;
    const uint32_t g = base + local;
    key[i] = valid ? src_keys[g] : 0u;
    row[i] = valid ? (implicit_rows ? g : src_rows[g]) : 0u;
    dig[i] = valid ? ((key[i] >> shift) & (kRadix - 1)) : kNoDigit;
  }
  __syncthreads();

  // ---- rank inside the wave: peers = lanes with the same digit -------------
  uint32_t rank[kPassItems];
#pragma unroll
  for (int i = 0; i < kPassItems; ++i) {
    const bool valid = dig[i] != kNoDigit;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint64_t bal = __ballot((dig[i] >> b) & 1u);
      peers &= ((dig[i] >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lanemask_lt());
    uint32_t old = 0;
    if (valid) old = s_wcnt[w][dig[i]];
    if (valid && below == 0) s_wcnt[w][dig[i]] = old + (uint32_t)__popcll(peers);
    rank[i] = old + below;
  }
  __syncthreads();

  // ---- per digit: counts, tile-local offsets, global offsets ---------------
  uint32_t tile_count = 0;
  if (tid < kRadix) {
#pragma unroll
    for (int ww = 0; ww < kPassWaves; ++ww) {
      const uint32_t c = s_wcnt[ww][tid];
      s_wcnt[ww][tid] = tile_count;
      tile_count += c;
    }
    uint64_t* st = lb.status + (uint64_t)tile * kRadix + tid;
    lb_publish(st, tile_count, lb.epoch, tile == 0 ? kLbInclusive : kLbAggregate);
  }
  uint32_t total;
  const uint32_t loff = block_excl_scan<kPassBlock>(tid < kRadix ? tile_count : 0u, s_scan, &total);
  __syncthreads();
  const uint32_t hcount = tid < kRadix ? hist[pass * kRadix + tid] : 0u;
  const uint32_t gstart = block_excl_scan<kPassBlock>(hcount, s_scan, &total);
  if (tid < kRadix) {
    uint32_t prefix = 0;
    if (tile != 0) {
      prefix = lb_lookback_thread(lb.status, kRadix, tid, tile, lb.epoch);
      lb_publish(lb.status + (uint64_t)tile * kRadix + tid, prefix + tile_count, lb.epoch, kLbInclusive);
    }
    s_loff[tid] = loff;
    s_dbase[tid] = gstart + prefix - loff;
  }
  __syncthreads();

  // ---- reorder the tile by digit in LDS -----------------------------------
#pragma unroll
  for (int i = 0; i < kPassItems; ++i) {
    if (dig[i] != kNoDigit) {
      const uint32_t pos = s_loff[dig[i]] + s_wcnt[w][dig[i]] + rank[i];
      s_keys[pos] = key[i];
      s_rows[pos] = row[i];
    }
  }
  __syncthreads();

  // ---- write each digit's run to its global place --------------------------
#pragma unroll
  for (int i = 0; i < kPassItems; ++i) {
    const uint32_t p = i * kPassBlock + tid;
    if (p < tile_n) {
      const uint32_t k = s_keys[p];
      const uint32_t g = s_dbase[(k >> shift) & (kRadix - 1)] + p;
      dst_keys[g] = k;
      dst_rows[g] = s_rows[p];
    }
  }
}

}  // namespace

int launch_radix_sort_pairs(Env& env, const uint32_t* keys, const uint32_t* rows, uint32_t* skeys,
                            uint32_t* srows, uint64_t n) {
  if (n == 0) return kOk;
  if (!keys || !skeys || !srows) return env.fail(kErrArg, "radix_sort: null buffer");
  if (n >= (1ull << 31)) return env.fail(kErrArg, "radix_sort: n must be below 2^31");
  LookbackArena* ar = env.arena();
  uint32_t* hist = ar->hist[ar->hist_turn];
  uint32_t* hist_next = ar->hist[ar->hist_turn ^ 1u];
  ar->hist_turn ^= 1u;

  uint64_t hgrid = (n + 4095) / 4096;
  if (hgrid > 1024) hgrid = 1024;
  env.prof_begin("radix_hist");
  k_radix_hist<<<dim3((uint32_t)hgrid), dim3(kHistBlock), 0, env.stream()>>>(keys, n, hist, hist_next);
  env.prof_end("radix_hist");
  int rc = check_launch(env, "radix_hist launch");
  if (rc) return rc;

  PassBuffers buf;
  buf.keys_in = keys;
  buf.rows_in = rows;
  buf.keys_a = skeys;
  buf.rows_a = srows;
  buf.keys_b = static_cast<uint32_t*>(env.scratch(n * 4));
  buf.rows_b = static_cast<uint32_t*>(env.scratch(n * 4));
  if (!buf.keys_b || !buf.rows_b) return env.fail(kErrOom, "radix_sort: scratch buffers");
  const uint32_t tiles = (uint32_t)((n + kPassTile - 1) / kPassTile);
  for (uint32_t pass = 0; pass < (uint32_t)kPasses; ++pass) {
    LbArgs lb;
    if (!env.lookback((uint64_t)tiles * kRadix, tiles, &lb)) return env.fail(kErrOom, "radix_sort: look-back");
    env.prof_begin("radix_pass");
    k_radix_pass<<<dim3(tiles), dim3(kPassBlock), 0, env.stream()>>>(buf, hist, pass, (uint32_t)n, lb);
    env.prof_end("radix_pass");
    rc = check_launch(env, "radix_pass launch");
    if (rc) return rc;
  }
  return kOk;
}

}  // namespace ka
