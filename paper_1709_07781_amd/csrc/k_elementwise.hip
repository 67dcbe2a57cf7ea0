// Elementwise kernels: the affine stage x <- a*x + b (mod 2^32), the
// per-stage workload of the kernel-stage overhead experiments (Sec. 3.6 empty
// stage probe, Sec. 5.2-5.3), and small fill kernels used instead of
// hipMemsetAsync so that the queued work stays capturable in a hipGraph.

#include "common.hpp"

namespace ka {
namespace {

constexpr int kAffBlock = 256;
constexpr int kAffVecPerThread = 4;                                  // uint4 per thread
constexpr int kAffTile = kAffBlock * kAffVecPerThread * 4;           // elements per work-group

// One work-group handles kAffTile consecutive elements; every load and store
// is a coalesced 16-byte access when the buffer is 16-byte aligned.
template <bool kVec>
__global__ __launch_bounds__(kAffBlock) void k_affine_u32(uint32_t* __restrict__ x, uint64_t n_cap,
                                                          const uint64_t* __restrict__ d_n, uint32_t a,
                                                          uint32_t b) {
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
        r.x = a * v[k].x + b;
        r.y = a * v[k].y + b;
        r.z = a * v[k].z + b;
        r.w = a * v[k].w + b;
        __builtin_nontemporal_store(r, x4 + e / 4);
      } else {
        for (uint64_t j = e; j < n && j < e + 4; ++j) x[j] = a * x[j] + b;
      }
    }
  } else {
#pragma unroll 4
    for (int k = 0; k < kAffTile / kAffBlock; ++k) {
      const uint64_t e = base + (uint64_t)k * kAffBlock + threadIdx.x;
      if (e < n) x[e] = a * x[e] + b;
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
  if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0)
    k_affine_u32<true><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(p, n_cap, d_n, a, b);
  else
    k_affine_u32<false><<<dim3((uint32_t)grid), dim3(kAffBlock), 0, env.stream()>>>(p, n_cap, d_n, a, b);
  env.prof_end("affine_u32");
  return check_launch(env, "affine_u32 launch");
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
