// Batch plans: the batched index build of one fixed batch shape recorded once
// into a HIP graph and replayed (Sec. 3.6: once the stages are composed, the
// per-stage messaging is the overhead left; a graph removes the per-launch
// host work as well).
//
// The plan owns every buffer the pipeline touches -- the input, the request
// table, the outputs and one scratch arena handed out by a bump allocator --
// so nothing is allocated while the graph is captured or replayed.
//
// A plan for any batch is recorded for capacities (values, requests) instead
// of one shape: the request table lives on the device with max_requests + 1
// entries, a batch of fewer requests is padded with empty ones, and the
// graph's first kernel reads the value count from the table's last entry, so
// every kernel sizes its grid by the capacity and works on the count it finds
// there.  Each run uploads a table and values and replays the same graph.  Look-back
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
  // any-batch plans: capacities, the largest request allowed, the count slot
  // the graph fills from the table, and two pinned tables used in turn (each
  // rewritten once its previous upload has finished)
  bool any = false;
  uint64_t n_cap = 0;
  uint32_t nreq_cap = 0, max_req = kMaxReqUnknown;
  uint64_t* d_n = nullptr;
  uint32_t* h_tab[2] = {nullptr, nullptr};
  hipEvent_t tab_done[2] = {nullptr, nullptr};
  int tab_next = 0;
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
  for (int i = 0; i < 2; ++i) {
    if (p->tab_done[i]) (void)hipEventDestroy(p->tab_done[i]);
    if (p->h_tab[i]) (void)hipHostFree(p->h_tab[i]);
  }
  if (p->mem) (void)hipFree(p->mem);
  (void)hipGetLastError();
  if (p->sys) p->sys->release();
  delete p;
}

// Allocates a plan for n values in nreq requests and records its graphs; the
// request table is uploaded from req_off (nreq + 1 host entries), and with
// any_batch the graph reads the value count from the table on the device.
static int plan_build(ka_system* sys, const uint32_t* req_off, uint64_t n, uint32_t nreq, uint32_t value_bits,
                      uint32_t biggest, bool any_batch, uint32_t flags, ka_batch_plan** out) {
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
  p->any = any_batch;
  p->n_cap = n;
  p->nreq_cap = nreq;
  p->max_req = biggest;
  // ---- one allocation: input, table, outputs, look-back state, scratch arena -----------
  const uint64_t n1 = n ? n : 1;
  // the segmented sort cuts tiles at request boundaries: at most one more per request
  const uint64_t sort_tiles = (n + 8191) / 8192 + nreq, enc_tiles = (n + 4095) / 4096;
  const uint64_t scan_tiles = 2 * ((256 * sort_tiles + 4095) / 4096) + 2;  // scan tiles hold >= 4096 entries
  // look-back status slots (kLbSpread words each): the encoder's tiles, or the
  // requests of the fused small-request launch
  const uint64_t arena_bytes = 24 * n1 + (16ull + 8 * kLbSpread) * nreq + 2 * sort_tiles * 2064 +
                               8ull * kLbSpread * enc_tiles + (64ull << 10);
  uint64_t off = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t o = off;
    off += plan_align(bytes);
    return o;
  };
  const uint64_t o_in = take(4 * n1), o_req = take(4 * (nreq + 1ull)), o_keys = take(4 * n1);
  const uint64_t o_offs = take(4 * (n + nreq)), o_words = take(8 * n1), o_ks = take(4 * (nreq + 1ull));
  const uint64_t o_ws = take(4 * (nreq + 1ull)), o_lens = take(6 * 8);
  const uint64_t o_plan = take(kSortPlanBytes), o_status = take(8ull * kLbSpread * scan_tiles);
  const uint64_t o_arena = take(arena_bytes);
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
  p->d_n = p->lens + 5;
  PlanEnv& e = p->env;
  e.lb.plan = m + o_plan;
  e.lb.status = reinterpret_cast<uint64_t*>(m + o_status);
  e.lb.status_words = (uint64_t)kLbSpread * scan_tiles;
  e.mem = m + o_arena;
  e.cap = arena_bytes;
  if (hipStreamCreateWithFlags(&p->s, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    plan_free(p);
    return set_error(KA_E_DEVICE, "plan: stream creation");
  }
  e.s = p->s;
  if (any_batch) {
    for (int i = 0; i < 2; ++i)
      if (hipHostMalloc(reinterpret_cast<void**>(&p->h_tab[i]), 4 * (nreq + 1ull), hipHostMallocDefault) !=
              hipSuccess ||
          hipEventCreateWithFlags(&p->tab_done[i], hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        plan_free(p);
        return set_error(KA_E_OOM, "plan: pinned request tables");
      }
  }
  // the request table is uploaded (a fixed plan's once and for all)
  if (hipMemcpyAsync(p->req_off, req_off, 4 * (nreq + 1ull), hipMemcpyHostToDevice, p->s) != hipSuccess ||
      hipStreamSynchronize(p->s) != hipSuccess) {
    (void)hipGetLastError();
    plan_free(p);
    return set_error(KA_E_DEVICE, "plan: initialisation");
  }
  // ---- record the pipeline, once per tile shape tried ---------------------------------
  const int forced = (int)((flags >> 8) & 0xFFu) - 1;  // KA_PLAN_SHAPE(s): record shape s only
  if (forced >= batch_variant_count()) {
    plan_free(p);
    return set_error(KA_E_ARG, "unknown tile shape");
  }
  p->forced = forced;
  p->shapes = (flags & KA_PLAN_AUTOTUNE) && forced < 0 ? std::min(batch_variant_count(), 4) : 1;
  p->chosen = p->shapes > 1 ? -1 : 0;
  for (int v = 0; v < p->shapes; ++v) {
    const int shape = forced >= 0 ? forced : v;
    e.used = 0;  // the shapes' graphs run one at a time on the plan's stream: they share the arena
    if (hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();
      plan_free(p);
      return set_error(KA_E_DEVICE, "plan: begin capture");
    }
    rc = any_batch ? launch_len_from_u32(e, p->d_n, p->req_off + nreq) : kOk;
    if (!rc)
      rc = launch_wah_batch(e, p->input, n, p->req_off, nreq, value_bits, p->keys, p->offsets, p->words,
                            p->key_start, p->word_start, p->lens, p->lens + 1, p->lens + 2, p->lens + 3, p->lens + 4,
                            shape, biggest, nullptr, any_batch ? p->d_n : nullptr);
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
  if (any_batch) {  // the plan starts out holding an empty batch
    p->n = 0;
    p->nreq = 0;
  }
  *out = p;
  return KA_OK;
}

KA_API int ka_batch_plan_create(ka_system* sys, const uint32_t* req_off, uint32_t nreq, uint32_t value_bits,
                                uint32_t flags, ka_batch_plan** out) {
  KA_GUARD_BEGIN
  if (!sys || !req_off || !out) return set_error(KA_E_ARG, "null argument");
  if (nreq == 0) return set_error(KA_E_ARG, "no requests");
  if (req_off[0] != 0) return set_error(KA_E_ARG, "req_off must start at 0");
  uint32_t biggest = 0;  // the largest request (selects the small-request path)
  for (uint32_t j = 0; j < nreq; ++j) {
    if (req_off[j + 1] < req_off[j]) return set_error(KA_E_ARG, "req_off must be non-decreasing");
    biggest = std::max(biggest, req_off[j + 1] - req_off[j]);
  }
  return plan_build(sys, req_off, req_off[nreq], nreq, value_bits, biggest, false, flags, out);
  KA_GUARD_END
}

KA_API int ka_batch_plan_create_any(ka_system* sys, uint64_t max_values, uint32_t max_requests,
                                    uint32_t max_request_values, uint32_t value_bits, uint32_t flags,
                                    ka_batch_plan** out) {
  KA_GUARD_BEGIN
  if (!sys || !out) return set_error(KA_E_ARG, "null argument");
  if (max_requests == 0) return set_error(KA_E_ARG, "max_requests must be at least 1");
  if (max_values >= (1ull << 30)) return set_error(KA_E_ARG, "max_values must be below 2^30");
  const uint32_t biggest = max_request_values ? max_request_values : kMaxReqUnknown;
  std::vector<uint32_t> empty(max_requests + 1ull, 0u);  // the empty batch the plan starts with
  return plan_build(sys, empty.data(), max_values, max_requests, value_bits, biggest, true, flags, out);
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
    // Each graph is launched once untimed first: a graph's first launch pays
    // one-time costs that would count against whichever variant is timed
    // first.
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      (void)hipGetLastError();
      if (a) (void)hipEventDestroy(a);
      return set_error(KA_E_DEVICE, "plan: events");
    }
    int best = 0;
    for (int v = 0; v < plan->shapes; ++v)
      if (hipGraphLaunch(plan->exec[v], plan->s) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return set_error(KA_E_LAUNCH, "plan: autotuning warm-up");
      }
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

KA_API int ka_batch_plan_run_batch(ka_batch_plan* plan, const uint32_t* values, const uint32_t* req_off,
                                   uint32_t nreq, uint32_t flags) {
  KA_GUARD_BEGIN
  if (!plan || !req_off) return set_error(KA_E_ARG, "null argument");
  if (!plan->any) return set_error(KA_E_STATE, "the plan was recorded for one batch shape");
  if (nreq > plan->nreq_cap) return set_error(KA_E_ARG, "more requests than the plan holds");
  if (req_off[0] != 0) return set_error(KA_E_ARG, "req_off must start at 0");
  for (uint32_t j = 0; j < nreq; ++j) {
    if (req_off[j + 1] < req_off[j]) return set_error(KA_E_ARG, "req_off must be non-decreasing");
    if (plan->max_req != kMaxReqUnknown && req_off[j + 1] - req_off[j] > plan->max_req)
      return set_error(KA_E_ARG, "a request is larger than the plan's largest request");
  }
  const uint64_t n = req_off[nreq];
  if (n > plan->n_cap) return set_error(KA_E_ARG, "more values than the plan holds");
  int rc = plan->sys->use_device();
  if (rc) return rc;
  // the table, padded with empty requests, through a pinned buffer whose
  // previous upload has finished
  const int k = plan->tab_next;
  if (hipEventSynchronize(plan->tab_done[k]) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "plan: table upload");
  }
  uint32_t* t = plan->h_tab[k];
  std::memcpy(t, req_off, 4 * (nreq + 1ull));
  for (uint32_t j = nreq + 1; j <= plan->nreq_cap; ++j) t[j] = (uint32_t)n;
  if (hipMemcpyAsync(plan->req_off, t, 4 * (plan->nreq_cap + 1ull), hipMemcpyHostToDevice, plan->s) != hipSuccess ||
      hipEventRecord(plan->tab_done[k], plan->s) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "plan: table upload");
  }
  plan->tab_next = k ^ 1;
  plan->n = n;
  plan->nreq = nreq;
  return ka_batch_plan_run(plan, values, flags);
  KA_GUARD_END
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
  // an any-batch plan's padding (empty requests after the real ones) adds one
  // offsets entry and one table entry each, at the ends
  const uint64_t pad = plan->nreq_cap - plan->nreq;
  len[1] -= pad;
  len[3] -= pad;
  len[4] -= pad;
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
