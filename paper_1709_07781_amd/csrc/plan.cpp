// Batch plans: the batched index build of one fixed batch shape recorded once
// into a HIP graph and replayed (Sec. 3.6: once the stages are composed, the
// per-stage messaging is the overhead left; a graph removes the per-launch
// host work as well).
//
// The plan owns every buffer the pipeline touches -- the input, the request
// table, the outputs and one scratch arena handed out by a bump allocator --
// so nothing is allocated while the graph is captured or replayed.  Look-back
// kernels get the plan's own status words, which a fill kernel inside the
// graph clears before each look-back launch: the epoch baked into a replayed
// launch is always the same, so stale words must not survive from the
// previous replay.
#include <cstring>

#include "runtime_internal.hpp"

namespace ka {
namespace {

constexpr uint64_t kPlanAlign = 256;
uint64_t plan_align(uint64_t x) { return (x + kPlanAlign - 1) / kPlanAlign * kPlanAlign; }

class PlanEnv final : public Env {
 public:
  hipStream_t s = nullptr;
  char* mem = nullptr;  // the scratch arena
  uint64_t cap = 0, used = 0;
  LookbackArena lb;

  hipStream_t stream() override { return s; }
  void* scratch(uint64_t bytes) override {
    const uint64_t b = plan_align(bytes ? bytes : 1);
    if (used + b > cap) return nullptr;
    void* p = mem + used;
    used += b;
    return p;
  }
  bool lookback(uint64_t words, LbArgs* out) override {
    if (words > lb.status_words) return false;
    if (launch_fill_u64(*this, lb.status, words, 0) != kOk) return false;
    out->status = lb.status;
    out->epoch = 1;
    out->spin_limit = kLbSpinLimit;
    return true;
  }
  LookbackArena* arena() override { return &lb; }
  void prof_begin(const char*) override {}
  void prof_end(const char*) override {}
  int fail(int code, const char* msg) override { return set_error(code, msg); }
};

}  // namespace

struct Plan {
  System* sys = nullptr;
  uint64_t n = 0;
  uint32_t nreq = 0, value_bits = 0;
  hipStream_t s = nullptr;
  void* mem = nullptr;  // one device allocation for everything
  uint32_t *input = nullptr, *req_off = nullptr, *keys = nullptr, *offsets = nullptr, *words = nullptr;
  uint32_t *key_start = nullptr, *word_start = nullptr;
  uint64_t* lens = nullptr;
  // one recorded graph per sort tile shape (only shape 0 without autotuning)
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t exec[4] = {nullptr, nullptr, nullptr, nullptr};
  int shapes = 1;
  int chosen = 0;        // index of the graph the runs use; -1 until the first run has timed them all
  int forced = -1;       // the one shape recorded by KA_PLAN_SHAPE, else -1
  float shape_ms[4] = {0, 0, 0, 0};
  PlanEnv env;
};

}  // namespace ka

using namespace ka;

struct ka_batch_plan : Plan {};

#define KA_GUARD_BEGIN try {
#define KA_GUARD_END                                              \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    return set_error(KA_E_OOM, "host allocation failed");         \
  }                                                               \
  catch (...) {                                                   \
    return set_error(KA_E_DEVICE, "internal error");              \
  }

static void plan_free(ka_batch_plan* p) {
  for (int i = 0; i < 4; ++i) {
    if (p->exec[i]) (void)hipGraphExecDestroy(p->exec[i]);
    if (p->graph[i]) (void)hipGraphDestroy(p->graph[i]);
  }
  if (p->s) {
    (void)hipStreamSynchronize(p->s);
    (void)hipStreamDestroy(p->s);
  }
  if (p->mem) (void)hipFree(p->mem);
  (void)hipGetLastError();
  if (p->sys) p->sys->release();
  delete p;
}

KA_API int ka_batch_plan_create(ka_system* sys, const uint32_t* req_off, uint32_t nreq, uint32_t value_bits,
                                uint32_t flags, ka_batch_plan** out) {
  KA_GUARD_BEGIN
  if (!sys || !req_off || !out) return set_error(KA_E_ARG, "null argument");
  if (nreq == 0) return set_error(KA_E_ARG, "no requests");
  const uint64_t n = req_off[nreq];
  if (req_off[0] != 0) return set_error(KA_E_ARG, "req_off must start at 0");
  uint32_t biggest = 0;  // the largest request (selects the small-request path)
  for (uint32_t j = 0; j < nreq; ++j) {
    if (req_off[j + 1] < req_off[j]) return set_error(KA_E_ARG, "req_off must be non-decreasing");
    biggest = std::max(biggest, req_off[j + 1] - req_off[j]);
  }
  if (n >= (1ull << 30)) return set_error(KA_E_ARG, "n must be below 2^30");
  if (value_bits == 0 || value_bits > 32) return set_error(KA_E_ARG, "value_bits must be 1..32");
  const uint32_t req_bits = nreq > 1 ? 32u - (uint32_t)__builtin_clz(nreq - 1) : 0u;
  if (value_bits + req_bits > 32) return set_error(KA_E_ARG, "value_bits + bits of nreq - 1 exceed 32");
  int rc = sys->ensure_init();
  if (rc) return rc;
  if ((rc = sys->use_device())) return rc;

  ka_batch_plan* p = new ka_batch_plan();
  p->sys = sys;
  sys->retain();
  p->n = n;
  p->nreq = nreq;
  p->value_bits = value_bits;
  // ---- one allocation: input, table, outputs, look-back state, scratch arena -----------
  const uint64_t n1 = n ? n : 1;
  // the segmented sort cuts tiles at request boundaries: at most one more per request
  const uint64_t sort_tiles = (n + 8191) / 8192 + nreq, enc_tiles = (n + 4095) / 4096;
  const uint64_t scan_tiles = 2 * ((256 * sort_tiles + 4095) / 4096) + 2;  // scan tiles hold >= 4096 entries
  const uint64_t arena_bytes = 24 * n1 + 16ull * nreq + 2 * sort_tiles * 2064 + 8 * enc_tiles + (64ull << 10);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += plan_align(bytes);
    return o;
  };
  const uint64_t o_in = take(4 * n1), o_req = take(4 * (nreq + 1ull)), o_keys = take(4 * n1);
  const uint64_t o_offs = take(4 * (n + nreq)), o_words = take(8 * n1), o_ks = take(4 * (nreq + 1ull));
  const uint64_t o_ws = take(4 * (nreq + 1ull)), o_lens = take(5 * 8);
  const uint64_t o_plan = take(kSortPlanBytes), o_status = take(8 * scan_tiles), o_arena = take(arena_bytes);
  if (hipMalloc(&p->mem, off) != hipSuccess) {
    (void)hipGetLastError();
    plan_free(p);
    return set_error(KA_E_OOM, "plan: device allocation");
  }
  char* m = static_cast<char*>(p->mem);
  p->input = reinterpret_cast<uint32_t*>(m + o_in);
  p->req_off = reinterpret_cast<uint32_t*>(m + o_req);
  p->keys = reinterpret_cast<uint32_t*>(m + o_keys);
  p->offsets = reinterpret_cast<uint32_t*>(m + o_offs);
  p->words = reinterpret_cast<uint32_t*>(m + o_words);
  p->key_start = reinterpret_cast<uint32_t*>(m + o_ks);
  p->word_start = reinterpret_cast<uint32_t*>(m + o_ws);
  p->lens = reinterpret_cast<uint64_t*>(m + o_lens);
  PlanEnv& e = p->env;
  e.lb.plan = m + o_plan;
  e.lb.status = reinterpret_cast<uint64_t*>(m + o_status);
  e.lb.status_words = scan_tiles;
  e.mem = m + o_arena;
  e.cap = arena_bytes;
  if (hipStreamCreateWithFlags(&p->s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    plan_free(p);
    return set_error(KA_E_DEVICE, "plan: stream creation");
  }
  e.s = p->s;
  // the request table is uploaded once
  if (hipMemcpyAsync(p->req_off, req_off, 4 * (nreq + 1ull), hipMemcpyHostToDevice, p->s) != hipSuccess ||
      hipStreamSynchronize(p->s) != hipSuccess) {
    (void)hipGetLastError();
    plan_free(p);
    return set_error(KA_E_DEVICE, "plan: initialisation");
  }
  // ---- record the pipeline, once per tile shape tried ---------------------------------
  const int forced = (int)((flags >> 8) & 0xFFu) - 1;  // KA_PLAN_SHAPE(s): record shape s only
  if (forced >= sort_shape_count()) {
    plan_free(p);
    return set_error(KA_E_ARG, "unknown tile shape");
  }
  p->forced = forced;
  p->shapes = (flags & KA_PLAN_AUTOTUNE) && forced < 0 ? std::min(sort_shape_count(), 4) : 1;
  p->chosen = p->shapes > 1 ? -1 : 0;
  for (int v = 0; v < p->shapes; ++v) {
    const int shape = forced >= 0 ? forced : v;
    e.used = 0;  // the shapes' graphs run one at a time on the plan's stream: they share the arena
    if (hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      plan_free(p);
      return set_error(KA_E_DEVICE, "plan: begin capture");
    }
    rc = launch_wah_batch(e, p->input, n, p->req_off, nreq, value_bits, p->keys, p->offsets, p->words,
                          p->key_start, p->word_start, p->lens, p->lens + 1, p->lens + 2, p->lens + 3, p->lens + 4,
                          shape, biggest);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->s, &g);
    p->graph[v] = g;
    if (rc || ec != hipSuccess || !g) {
      (void)hipGetLastError();
      plan_free(p);
      return rc ? rc : set_error(KA_E_DEVICE, "plan: end capture");
    }
    if (hipGraphInstantiate(&p->exec[v], p->graph[v], nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGetLastError();
      plan_free(p);
      return set_error(KA_E_DEVICE, "plan: graph instantiation");
    }
  }
  *out = p;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_batch_plan_input(ka_batch_plan* plan, uint32_t** values_dev) {
  if (!plan || !values_dev) return set_error(KA_E_ARG, "null argument");
  *values_dev = plan->input;
  return KA_OK;
}

KA_API int ka_batch_plan_stream(ka_batch_plan* plan, void** stream) {
  if (!plan || !stream) return set_error(KA_E_ARG, "null argument");
  *stream = plan->s;
  return KA_OK;
}

KA_API int ka_batch_plan_run(ka_batch_plan* plan, const uint32_t* values, uint32_t flags) {
  if (!plan) return set_error(KA_E_ARG, "null plan");
  int rc = plan->sys->use_device();
  if (rc) return rc;
  if (values && plan->n &&
      hipMemcpyAsync(plan->input, values, 4 * plan->n,
                     (flags & KA_WAH_INPUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                     plan->s) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "plan: input copy");
  }
  if (plan->chosen < 0) {
    // Autotuning: the first run times every recorded shape on these values
    // (each leaves the same outputs) and keeps the fastest for later runs.
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      (void)hipGetLastError();
      if (a) (void)hipEventDestroy(a);
      return set_error(KA_E_DEVICE, "plan: events");
    }
    int best = 0;
    for (int v = 0; v < plan->shapes; ++v) {
      if (hipEventRecord(a, plan->s) != hipSuccess || hipGraphLaunch(plan->exec[v], plan->s) != hipSuccess ||
          hipEventRecord(b, plan->s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&plan->shape_ms[v], a, b) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return set_error(KA_E_LAUNCH, "plan: autotuning run");
      }
      if (plan->shape_ms[v] < plan->shape_ms[best]) best = v;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    plan->chosen = best;
    return KA_OK;
  }
  if (hipGraphLaunch(plan->exec[plan->chosen], plan->s) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_LAUNCH, "plan: graph launch");
  }
  return KA_OK;
}

KA_API int ka_batch_plan_shape(ka_batch_plan* plan, int* shape, float* ms, uint32_t nms) {
  if (!plan || !shape) return set_error(KA_E_ARG, "null argument");
  *shape = plan->chosen < 0 ? -1 : (plan->forced >= 0 ? plan->forced : plan->chosen);
  for (uint32_t i = 0; ms && i < nms; ++i) ms[i] = i < (uint32_t)plan->shapes ? plan->shape_ms[i] : 0.0f;
  return KA_OK;
}

KA_API int ka_batch_plan_result(ka_batch_plan* plan, ka_wah_batch_result* out) {
  KA_GUARD_BEGIN
  if (!plan || !out) return set_error(KA_E_ARG, "null argument");
  int rc = plan->sys->use_device();
  if (rc) return rc;
  uint64_t len[5];
  if (hipStreamSynchronize(plan->s) != hipSuccess ||
      hipMemcpy(len, plan->lens, sizeof(len), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "plan: synchronisation");
  }
  if (len[3] == 0) return set_error(KA_E_ARG, "a value is at or above 2^value_bits");
  ka_wah_batch_result r{};
  r.nreq = plan->nreq;
  r.n = plan->n;
  r.D = len[0];
  r.W = len[2];
  const uint32_t* src[5] = {plan->keys, plan->offsets, plan->words, plan->key_start, plan->word_start};
  uint32_t** dst[5] = {&r.keys, &r.offsets, &r.words, &r.key_start, &r.word_start};
  for (int i = 0; i < 5 && !rc; ++i) {
    *dst[i] = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(len[i], 1) * 4));
    if (!*dst[i]) {
      rc = set_error(KA_E_OOM, "host allocation failed");
    } else if (len[i] && hipMemcpy(*dst[i], src[i], 4 * len[i], hipMemcpyDeviceToHost) != hipSuccess) {
      (void)hipGetLastError();
      rc = set_error(KA_E_DEVICE, "plan: result copy");
    }
  }
  if (rc) {
    for (auto d : dst) std::free(*d);
    return rc;
  }
  *out = r;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_batch_plan_destroy(ka_batch_plan* plan) {
  if (!plan) return set_error(KA_E_ARG, "null plan");
  (void)plan->sys->use_device();
  plan_free(plan);
  return KA_OK;
}
