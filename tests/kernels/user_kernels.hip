// User kernels for the code-object path of ka_program_load (test fixtures).
// Parameters follow the convention of ka.h: one device pointer per
// in/out/in_out argument, a uint32 LDS byte offset per local argument, the
// priv values, then the ND-range (global sizes and offsets).
#include <hip/hip_runtime.h>
#include <stdint.h>

struct NdRangeDev {
  uint64_t global[3];
  uint64_t offset[3];
};

// The empty stage of the messaging-cost probe (Sec. 3.6): takes a reference, does nothing.
extern "C" __global__ void empty_stage(const uint32_t* in, NdRangeDev r) {
  (void)in;
  (void)r;
}

// c = a + b over the global range (with its offset).
extern "C" __global__ void add_u32(const uint32_t* a, const uint32_t* b, uint32_t* c, NdRangeDev r) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < r.global[0]) {
    const uint64_t j = i + r.offset[0];
    c[j] = a[j] + b[j];
  }
}

// out = reverse of (in * factor) inside each work-group, through a local buffer.
extern "C" __global__ void reverse_scale_local(const uint32_t* in, uint32_t* out, uint32_t lds_off, uint32_t factor,
                                               NdRangeDev r) {
  extern __shared__ uint8_t lds[];
  uint32_t* buf = reinterpret_cast<uint32_t*>(lds + lds_off);
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  buf[threadIdx.x] = i < r.global[0] ? in[i] * factor : 0u;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * blockDim.x;
  const uint64_t src = blockDim.x - 1 - threadIdx.x;
  if (i < r.global[0] && base + src < r.global[0]) out[i] = buf[src];
  else if (i < r.global[0]) out[i] = 0xFFFFFFFFu;
}
