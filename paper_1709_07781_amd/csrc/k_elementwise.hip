// Elementwise kernels: the affine stage x <- a*x + b (mod 2^32), the
// per-stage workload of the kernel-stage overhead experiments (Sec. 3.6 empty
// stage probe, Sec. 5.2-5.3), and small fill kernels used instead of
// hipMemsetAsync so that the queued work stays capturable in a hipGraph.

#include <algorithm>

#include "common.hpp"

namespace ka {
namespace {

constexpr int kAffBlock = 256;
constexpr int kAffVecPerThread = 4;                                  // uint4 per thread
constexpr int kAffTile = kAffBlock * kAffVecPerThread * 4;           // elements per work-group
constexpr uint32_t kChainMax = 16;                                   // stages per fused pass

// One affine stage, or up to kChainMax stages applied in turn in one pass
// (x <- a_i x + b_i for i = 0 .. len-1, all mod 2^32).
struct Affine1 {
  uint32_t a, b;
  __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return a * x + b; }
};
struct AffineChain {
  uint32_t a[kChainMax], b[kChainMax];
  uint32_t len;
  __device__ __forceinline__ uint32_t operator()(uint32_t x) const {
    for (uint32_t i = 0; i < len; ++i) x = a[i] * x + b[i];
    return x;
  }
};

// One work-group handles kAffTile consecutive elements; every load and store
// is a coalesced 16-byte access when the buffer is 16-byte aligned.
template <bool kVec, class Op>
__global__ __launch_bounds__(kAffBlock) void k_affine_u32(uint32_t* __restrict__ x, uint64_t n_cap,
                                                          const uint64_t* __restrict__ d_n, Op op) {
  const uint64_t n = device_count(n_cap, d_n);
  const uint64_t base = (uint64_t)blockIdx.x * kAffTile;
  if (base >= n) return;
  if (kVec) {
    u32x4* x4 = reinterpret_cast<u32x4*>(x);
    u32x4 v[kAffVecPerThread];
    bool full[kAffVecPerThread];
#pragma unroll
    for (int k = 0; k < kAffVecPerThread; ++k) {
      const uint64_t e = base + ((uint64_t)k * kAffBlock + threadIdx.x) * 4;
      full[k] = e + 4 <= n;
      if (full[k]) v[k] = __builtin_nontemporal_load(x4 + e / 4);
    }
#pragma unroll
    for (int k = 0; k < kAffVecPerThread; ++k) {
      const uint64_t e = base + ((uint64_t)k * kAffBlock + threadIdx.x) * 4;
      if (full[k]) {
        u32x4 r;
        r.x = op(v[k].x);
        r.y = op(v[k].y);
        r.z = op(v[k].z);
        r.w = op(v[k].w);
        __builtin_nontemporal_store(r, x4 + e / 4);
      } else {
        for (uint64_t j = e; j < n && j < e + 4; ++j) x[j] = op(x[j]);
      }
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < kAffTile / kAffBlock; ++k) {
      const uint64_t e = base + (uint64_t)k * kAffBlock + threadIdx.x;
      if (e < n) x[e] = op(x[e]);
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_u64(uint64_t* __restrict__ p, uint64_t count, uint64_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256)
    p[i] = value;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint64_t count, uint32_t value) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (uint64_t)gridDim.x * 256)
    p[i] = value;
}

__global__ void k_set_len(uint64_t* d_len, uint64_t value) {
  if (threadIdx.x == 0) *d_len = value;
}

__global__ void k_copy_len(uint64_t* dst, const uint64_t* src) {
  if (threadIdx.x == 0) *dst = *src;
}

__global__ void k_len_from_u32(uint64_t* dst, const uint32_t* src) {
  if (threadIdx.x == 0) *dst = *src;
}

inline uint32_t fill_grid(uint64_t count) {
  uint64_t g = (count + 255) / 256;
  if (g > 4096) g = 4096;
  return g ? (uint32_t)g : 1u;
}

}  // namespace

int launch_affine(Env& env, uint32_t* x, uint64_t n_cap, const uint64_t* d_n, uint64_t offset, uint32_t a,
                  uint32_t b) {
  if (n_cap == 0) return kOk;
  if (!x) return env.fail(kErrArg, "affine_u32: null buffer");
  uint32_t* p = x + offset;
  const uint64_t grid = (n_cap + kAffTile - 1) / kAffTile;
  if (grid > 0x7FFFFFFFull) return env.fail(kErrArg, "affine_u32: too many elements");
  env.prof_begin("affine_u32");
  const Affine1 op{a, b};
  if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)
    k_affine_u32<true><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(p, n_cap, d_n, op);
  else
    k_affine_u32<false><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(p, n_cap, d_n, op);
  env.prof_end("affine_u32");
  return check_launch(env, "affine_u32 launch");
}

int launch_affine_chain(Env& env, uint32_t* x, uint64_t n, const uint32_t* a, const uint32_t* b, uint32_t len) {
  if (n == 0 || len == 0) return kOk;
  if (!x || !a || !b) return env.fail(kErrArg, "affine chain: null buffer");
  const uint64_t grid = (n + kAffTile - 1) / kAffTile;
  if (grid > 0x7FFFFFFFull) return env.fail(kErrArg, "affine chain: too many elements");
  const bool vec = (reinterpret_cast<uintptr_t>(x) & 15u) == 0;
  for (uint32_t s0 = 0; s0 < len; s0 += kChainMax) {  // kChainMax stages per pass over x
    AffineChain op{};
    op.len = std::min<uint32_t>(kChainMax, len - s0);
    for (uint32_t i = 0; i < op.len; ++i) {
      op.a[i] = a[s0 + i];
      op.b[i] = b[s0 + i];
    }
    env.prof_begin("affine_chain_u32");
    if (vec)
      k_affine_u32<true><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(x, n, nullptr, op);
    else
      k_affine_u32<false><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(x, n, nullptr, op);
    env.prof_end("affine_chain_u32");
    const int rc = check_launch(env, "affine chain launch");
    if (rc) return rc;
  }
  return kOk;
}

int launch_fill_u64(Env& env, uint64_t* p, uint64_t count, uint64_t value) {
  if (count == 0) return kOk;
  k_fill_u64<<<dim3(fill_grid(count)), dim3(256), 0, env.stream()>>>(p, count, value);
  return check_launch(env, "fill_u64 launch");
}

int launch_fill_u32(Env& env, uint32_t* p, uint64_t count, uint32_t value) {
  if (count == 0) return kOk;
  k_fill_u32<<<dim3(fill_grid(count)), dim3(256), 0, env.stream()>>>(p, count, value);
  return check_launch(env, "fill_u32 launch");
}

int launch_set_len(Env& env, uint64_t* d_len, uint64_t value) {
  k_set_len<<<dim3(1), dim3(64), 0, env.stream()>>>(d_len, value);
  return check_launch(env, "set_len launch");
}

int launch_copy_len(Env& env, uint64_t* dst, const uint64_t* src) {
  k_copy_len<<<dim3(1), dim3(64), 0, env.stream()>>>(dst, src);
  return check_launch(env, "copy_len launch");
}

int launch_len_from_u32(Env& env, uint64_t* dst, const uint32_t* src) {
  k_len_from_u32<<<dim3(1), dim3(64), 0, env.stream()>>>(dst, src);
  return check_launch(env, "len_from_u32 launch");
}

}  // namespace ka
