// Exclusive prefix sum and stream compaction of uint32 arrays.
//
// Both are single-pass: every tile (one work-group) is reduced, publishes its
// total, finds its exclusive prefix by decoupled look-back over its
// predecessors and writes its results -- 8 bytes of HBM traffic per element
// for the scan, 4 + 4*kept for the compaction.  Tiles are numbered by
// work-group id and the look-back has a fallback (a predecessor that stays
// silent is reduced from its input by the waiting wave), so no wait depends on
// the order in which work-groups are dispatched.  The fallback reads a
// predecessor's input, which is why the input and output must not overlap.
// (Tiles numbered by a ticket counter instead cost about 8 ns per work-group,
// serialised on the counter.)  The compaction is the primitive of the
// fuseFillsLiterals step (Sec. 4.1): it removes the zero entries and keeps the
// order; its phases "count per group", "scan of the group counts" and "move
// the valid elements" run in one kernel.
//
// Tile layout: round r of thread t holds the 4 consecutive elements starting at
// tile_base + 4 (r * BLOCK + t), so every global access is a coalesced
// 16-byte load or store; element order inside the tile is (round, thread, lane
// of the vector).  The number of rounds R is chosen per launch: 8 (8192
// elements per tile) up to 2^23 elements, where the look-back's latency
// dominates, 16 above, where fewer tiles mean fewer look-backs per byte
// (measured at 2^26: 138 us at 16 rounds, 193 us at 8; at 2^21, 8.7 us at 8
// and 10.5 us at 16).
#include "common.hpp"

namespace ka {
namespace {

constexpr int kScanBlock = 256;
constexpr int kWaves = kScanBlock / 64;
constexpr int kSmallRounds = 8, kLargeRounds = 16;
constexpr uint64_t kLargeScan = 1ull << 23;  // capacities above this use kLargeRounds
constexpr int kCompactRounds = 8;            // the compaction stages a tile in LDS (32 KiB)
template <int R>
constexpr int kTileElems = kScanBlock * R * 4;

template <bool kVec>
__device__ __forceinline__ void load4(const uint32_t* __restrict__ p, uint64_t e, uint64_t n, uint32_t v[4]) {
  if (kVec && e + 4 <= n) {
    const u32x4 q = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p + e));
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
    v[3] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (e + j < n) ? p[e + j] : 0u;
  }
}

template <bool kVec>
__device__ __forceinline__ void store4(uint32_t* __restrict__ p, uint64_t e, uint64_t n, const uint32_t v[4]) {
  if (kVec && e + 4 <= n) {
    u32x4 q;
    q.x = v[0];
    q.y = v[1];
    q.z = v[2];
    q.w = v[3];
    __builtin_nontemporal_store(q, reinterpret_cast<u32x4*>(p + e));
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (e + j < n) p[e + j] = v[j];
  }
}

// Exclusive prefix of each thread's round sums over (round, thread) order,
// plus the tile total.  One barrier.
template <int R>
__device__ __forceinline__ void tile_scan(const uint32_t (&s)[R], uint32_t (&pre)[R], uint32_t* tile_total,
                                          uint32_t (*s_wave)[kWaves]) {
  const uint32_t w = threadIdx.x / 64;
  uint32_t inc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    inc[r] = wave_incl_scan(s[r]);
    if (lane_id() == 63) s_wave[r][w] = inc[r];
  }
  __syncthreads();
  uint32_t round_base = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      const uint32_t t = s_wave[r][i];
      before += (i < (int)w) ? t : 0u;
      tot += t;
    }
    pre[r] = round_base + before + inc[r] - s[r];
    round_base += tot;
  }
  *tile_total = round_base;
}

// Wave 0 publishes the tile total, looks back, publishes the inclusive prefix
// and leaves the tile's exclusive prefix in *s_prefix; reduce(t) gives a
// silent predecessor's total (see lb_lookback_st).  Tile t's status word is
// lb.status[kLbSpread * t].
template <class Reduce>
__device__ __forceinline__ void tile_lookback(const LbArgs& lb, uint32_t tile, uint32_t tile_total,
                                              uint32_t* s_prefix, Reduce&& reduce) {
  if (threadIdx.x < 64) {
    uint32_t prefix = 0;
    uint64_t* slot = lb.status + (uint64_t)kLbSpread * tile;
    if (tile == 0) {
      if (threadIdx.x == 0) lb_publish(slot, tile_total, lb.epoch, kLbInclusive);
    } else {
      if (threadIdx.x == 0) lb_publish(slot, tile_total, lb.epoch, kLbAggregate);
      prefix = lb_lookback_st<kLbSpread>(lb.status, tile, LbEpoch{lb.epoch}, lb.spin_limit, reduce);
      if (threadIdx.x == 0) lb_publish(slot, prefix + tile_total, lb.epoch, kLbInclusive);
    }
    if (threadIdx.x == 0) *s_prefix = prefix;
  }
  __syncthreads();
}

// Total of tile u by one wave (every lane gets it); op maps an element to
// what it adds (itself for the scan, 1 if non-zero for the compaction).
template <int R, bool kVec, class Op>
__device__ __forceinline__ uint32_t wave_tile_total(const uint32_t* in, uint32_t u, uint64_t n, Op op) {
  const uint64_t b = (uint64_t)u * kTileElems<R>;
  uint32_t acc = 0;
#pragma unroll 4
  for (int i = 0; i < kTileElems<R> / 256; ++i) {
    uint32_t q[4];
    load4<kVec>(in, b + 4 * ((uint64_t)i * 64 + lane_id()), n, q);
    acc += op(q[0]) + op(q[1]) + op(q[2]) + op(q[3]);
  }
  return wave_sum(acc);
}

template <int R, bool kVec>
__device__ __forceinline__ void load_tile(const uint32_t* __restrict__ in, uint64_t tile, uint64_t n,
                                          uint32_t (&v)[R][4]) {
  const uint64_t base = tile * kTileElems<R>;
#pragma unroll
  for (int r = 0; r < R; ++r) load4<kVec>(in, base + ((uint64_t)r * kScanBlock + threadIdx.x) * 4, n, v[r]);
}

// One tile per work-group.  The grid is the tile count of n_cap; with a
// smaller device-resident count the surplus work-groups leave at once.
template <int R, bool kVec>
__global__ __launch_bounds__(kScanBlock) void k_exclusive_scan_u32(const uint32_t* __restrict__ in,
                                                                   uint32_t* __restrict__ out, uint64_t n_cap,
                                                                   const uint64_t* __restrict__ d_n, LbArgs lb) {
  constexpr int kTile = kTileElems<R>;
  __shared__ uint32_t s_prefix;
  __shared__ uint32_t s_wave[R][kWaves];
  const uint64_t n = device_count(n_cap, d_n);
  const uint64_t ntiles = (n + kTile - 1) / kTile;
  const uint32_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  const uint64_t base = (uint64_t)tile * kTile;
  uint32_t v[R][4];
  load_tile<R, kVec>(in, tile, n, v);
  uint32_t s[R], pre[R];
#pragma unroll
  for (int r = 0; r < R; ++r) s[r] = v[r][0] + v[r][1] + v[r][2] + v[r][3];
  uint32_t total;
  tile_scan<R>(s, pre, &total, s_wave);
  tile_lookback(lb, tile, total, &s_prefix, [&](uint32_t u) {
    return wave_tile_total<R, kVec>(in, u, n, [](uint32_t x) { return x; });
  });
  const uint32_t tp = s_prefix;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint32_t acc = tp + pre[r], o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      o[j] = acc;
      acc += v[r][j];
    }
    store4<kVec>(out, base + ((uint64_t)r * kScanBlock + threadIdx.x) * 4, n, o);
  }
}

// Kept elements are staged in LDS at their tile-local positions, then copied
// to out[prefix ...] with consecutive work-items writing consecutive words.
template <bool kVec>
__global__ __launch_bounds__(kScanBlock) void k_compact_nonzero_u32(const uint32_t* __restrict__ in,
                                                                    uint32_t* __restrict__ out, uint64_t n_cap,
                                                                    const uint64_t* __restrict__ d_n,
                                                                    uint64_t* __restrict__ d_out_len, LbArgs lb) {
  constexpr int R = kCompactRounds, kTile = kTileElems<R>;
  __shared__ uint32_t s_prefix;
  __shared__ uint32_t s_wave[R][kWaves];
  __shared__ __align__(16) uint32_t s_out[kTile];
  const uint64_t n = device_count(n_cap, d_n);
  const uint64_t ntiles = (n + kTile - 1) / kTile;
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) *d_out_len = 0;  // empty input
  const uint32_t tile = blockIdx.x;
  if (tile >= ntiles) return;
  uint32_t v[R][4];
  load_tile<R, kVec>(in, tile, n, v);
  uint32_t s[R], pre[R];
#pragma unroll
  for (int r = 0; r < R; ++r) s[r] = (v[r][0] != 0) + (v[r][1] != 0) + (v[r][2] != 0) + (v[r][3] != 0);
  uint32_t total;
  tile_scan<R>(s, pre, &total, s_wave);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint32_t pos = pre[r];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (v[r][j] != 0) s_out[pos++] = v[r][j];
  }
  tile_lookback(lb, tile, total, &s_prefix, [&](uint32_t u) {  // ends with a barrier
    return wave_tile_total<R, kVec>(in, u, n, [](uint32_t x) { return x != 0 ? 1u : 0u; });
  });
  const uint64_t dst = s_prefix;
  // four kept words per work-item and step (16-byte stores at word alignment)
  const uint32_t nv = total / 4;
  for (uint32_t v = threadIdx.x; v < nv; v += kScanBlock)
    *reinterpret_cast<u32x4w*>(out + dst + 4 * v) = *reinterpret_cast<const u32x4*>(s_out + 4 * v);
  if (threadIdx.x < total - 4 * nv) out[dst + 4 * nv + threadIdx.x] = s_out[4 * nv + threadIdx.x];
  if (tile == ntiles - 1 && threadIdx.x == 0) *d_out_len = dst + total;
}

inline bool ranges_overlap(const uint32_t* a, const uint32_t* b, uint64_t n) {
  const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
  return x < y + 4 * n && y < x + 4 * n;
}

template <int R>
int scan_launch(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n) {
  const uint32_t grid = (uint32_t)((n_cap + kTileElems<R> - 1) / kTileElems<R>);
  LbArgs lb;
  if (!env.lookback((uint64_t)kLbSpread * grid, &lb))
    return env.fail(kErrOom, "exclusive_scan_u32: look-back state");
  const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15u) == 0;
  const dim3 g(grid), b(kScanBlock);
  env.prof_begin("exclusive_scan_u32");
  if (vec)
    k_exclusive_scan_u32<R, true><<<g, b, 0, env.stream()>>>(in, out, n_cap, d_n, lb);
  else
    k_exclusive_scan_u32<R, false><<<g, b, 0, env.stream()>>>(in, out, n_cap, d_n, lb);
  env.prof_end("exclusive_scan_u32");
  return check_launch(env, "exclusive_scan_u32 launch");
}

}  // namespace

// in and out must not overlap.
int launch_exclusive_scan(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n) {
  if (n_cap == 0) return kOk;
  if (!in || !out) return env.fail(kErrArg, "exclusive_scan_u32: null buffer");
  if (n_cap > 0xFFFFFFFFull) return env.fail(kErrArg, "exclusive_scan_u32: more than 2^32-1 elements");
  if (ranges_overlap(in, out, n_cap)) return env.fail(kErrArg, "exclusive_scan_u32: in and out overlap");
  return n_cap > kLargeScan ? scan_launch<kLargeRounds>(env, in, out, n_cap, d_n)
                            : scan_launch<kSmallRounds>(env, in, out, n_cap, d_n);
}

int launch_compact_nonzero(Env& env, const uint32_t* in, uint32_t* out, uint64_t n_cap, const uint64_t* d_n,
                           uint64_t* d_out_len) {
  if (!d_out_len) return env.fail(kErrArg, "compact_nonzero_u32: no length slot");
  if (n_cap == 0) return launch_set_len(env, d_out_len, 0);
  if (!in || !out) return env.fail(kErrArg, "compact_nonzero_u32: null buffer");
  if (n_cap > 0xFFFFFFFFull) return env.fail(kErrArg, "compact_nonzero_u32: more than 2^32-1 elements");
  if (ranges_overlap(in, out, n_cap)) return env.fail(kErrArg, "compact_nonzero_u32: in and out overlap");
  const uint32_t grid = (uint32_t)((n_cap + kTileElems<kCompactRounds> - 1) / kTileElems<kCompactRounds>);
  LbArgs lb;
  if (!env.lookback((uint64_t)kLbSpread * grid, &lb))
    return env.fail(kErrOom, "compact_nonzero_u32: look-back state");
  const bool vec = (reinterpret_cast<uintptr_t>(in) & 15u) == 0;
  env.prof_begin("compact_nonzero_u32");
  if (vec)
    k_compact_nonzero_u32<true><<<dim3(grid), dim3(kScanBlock), 0, env.stream()>>>(in, out, n_cap, d_n, d_out_len, lb);
  else
    k_compact_nonzero_u32<false><<<dim3(grid), dim3(kScanBlock), 0, env.stream()>>>(in, out, n_cap, d_n, d_out_len,
                                                                                    lb);
  env.prof_end("compact_nonzero_u32");
  return check_launch(env, "compact_nonzero_u32 launch");
}

}  // namespace ka
