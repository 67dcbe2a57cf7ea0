// The served form: an actor's mailbox (Sec. 2.1: messages wait at the receiver
// in order of arrival until they are processed; Sec. 3.6: an OpenCL actor's
// mailbox maps to a command queue of the device) turned into continuous
// batching.
//
//  * ka_server_submit copies the request's data into pinned host memory
//    (recycled by size class) and appends it to the mailbox with its arrival
//    time.  A large payload is cut into chunks that the submitting thread and
//    the server's copy threads copy together; an index payload's values are
//    checked against 2^value_bits in the same pass.
//  * The mailbox thread forms a batch from the oldest waiting requests as soon
//    as a stream slot is free and the HBM budget admits them (at most
//    max_batch requests and max_batch_bytes of input; a request that arrives
//    while batches run waits for the next slot).  Each request's data is
//    copied straight from its pinned buffer to its place in the batch's
//    device layout, then the kernels run per kind, all on the batch's stream:
//    the index requests as one batched index build, the scans as one scan of
//    their concatenation rebased per request, the affine chains as the chain
//    over their concatenation in one pass (an elementwise map needs no
//    per-request work, and one kernel applies every stage);
//    the outputs go back to one pinned buffer, then an event.
//  * The completion thread waits for batches in launch order, points each
//    request at its slices of the batch's pinned outputs (no copy; the buffer
//    is recycled once every request of the batch is released), releases
//    device memory and budget, and records each request's latency from its
//    arrival time.
// Batches on different streams overlap on the device; max_batch = 1 with one
// stream is the plain per-request form of the same kernels.
#include <time.h>

#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>

#include "runtime_internal.hpp"

namespace ka {

double clock_us() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return ts.tv_sec * 1e6 + ts.tv_nsec * 1e-3;
}

namespace {

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Device bytes a request holds while its batch runs (inputs, outputs and the
// pipeline's scratch), an upper bound used for admission.
uint64_t request_bytes(uint32_t kind, uint64_t n) {
  switch (kind) {
    case KA_REQ_WAH:
      // values, tagged keys, sorted pairs, ping-pong pairs, tile offsets,
      // keys, offsets, 2n words, tables
      return 4 * n + 4 * n + 8 * n + 8 * n + 4 * n + 4 * n + 4 * n + 8 * n + 64 + n / 8;
    case KA_REQ_SCAN:
      return 8 * n + 64;
    default:
      return 4 * n + 64;
  }
}

// dst[i] = src[i] for i < n; returns the OR of the values shifted right by
// shift (0 for shift >= 32): nonzero iff some value is at or above 2^shift.
uint32_t copy_checked(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, uint64_t n, uint32_t shift) {
  if (shift >= 32) {
    std::memcpy(dst, src, 4 * n);
    return 0;
  }
  uint32_t o = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t x = src[i];
    dst[i] = x;
    o |= x;
  }
  return o >> shift;
}

// Copies host payloads into pinned memory.  A payload of kSplitBytes or more
// is cut into kChunk-element chunks; the submitting thread and the pool's
// threads take chunks until none is left.  A job stays reachable only while it
// is queued; the submitter unqueues it and waits until no thread is inside it.
class CopyPool {
 public:
  static constexpr uint64_t kSplitBytes = 1ull << 20;
  static constexpr uint64_t kChunk = 1ull << 16;  // elements (256 KiB)

  void start(uint32_t threads) {
    for (uint32_t i = 0; i < threads; ++i) th_.emplace_back([this] { work(); });
  }
  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      stopping_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
    th_.clear();
  }
  uint32_t copy(uint32_t* dst, const uint32_t* src, uint64_t n, uint32_t shift) {
    if (th_.empty() || 4 * n < kSplitBytes) return copy_checked(dst, src, n, shift);
    Job j{dst, src, n, shift, (n + kChunk - 1) / kChunk};
    {
      std::lock_guard<std::mutex> g(mu_);
      jobs_.push_back(&j);
    }
    cv_.notify_all();
    run(j);
    std::unique_lock<std::mutex> lk(mu_);
    for (auto it = jobs_.begin(); it != jobs_.end(); ++it)
      if (*it == &j) {
        jobs_.erase(it);
        break;
      }
    cv_idle_.wait(lk, [&] { return j.active == 0; });
    return j.over.load();
  }

 private:
  struct Job {
    uint32_t* dst;
    const uint32_t* src;
    uint64_t n;
    uint32_t shift;
    uint64_t chunks;
    std::atomic<uint64_t> next{0};
    std::atomic<uint32_t> over{0};
    uint32_t active = 0;  // pool threads inside the job (under mu_)
  };
  static void run(Job& j) {
    uint32_t o = 0;
    for (uint64_t c; (c = j.next.fetch_add(1)) < j.chunks;) {
      const uint64_t b = c * kChunk, e = std::min(j.n, b + kChunk);
      o |= copy_checked(j.dst + b, j.src + b, e - b, j.shift);
    }
    if (o) j.over.fetch_or(o);
  }
  void work() {
    for (;;) {
      Job* j = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stopping_ || !jobs_.empty(); });
        if (stopping_) return;
        j = jobs_.front();
        if (j->next.load() >= j->chunks) {  // every chunk is taken: nothing left here
          jobs_.pop_front();
          continue;
        }
        ++j->active;
      }
      run(*j);
      {
        std::lock_guard<std::mutex> g(mu_);
        --j->active;
      }
      cv_idle_.notify_all();
    }
  }
  std::mutex mu_;
  std::condition_variable cv_, cv_idle_;
  std::deque<Job*> jobs_;
  std::vector<std::thread> th_;
  bool stopping_ = false;
};

}  // namespace

// Pinned output buffer of one batch, shared by its requests.
struct OutBuf {
  System* sys = nullptr;
  void* p = nullptr;
  std::atomic<int> refs{0};
  void release() {
    if (refs.fetch_sub(1) == 1) {
      if (p) sys->stage.give_back(p);
      delete this;
    }
  }
};

struct SrvReq {
  virtual ~SrvReq() {
    if (pin) sys->stage.give_back(pin);
    if (dref) ref_release(dref);
    for (auto* o : out_ref)
      if (o) ref_release(o);
    if (outbuf) outbuf->release();
  }
  std::atomic<int> refs{2};  // the caller's handle and the server's
  System* sys = nullptr;
  uint32_t kind = 0;
  uint64_t n = 0;
  void* pin = nullptr;   // the input, pinned (host input)
  Ref* dref = nullptr;   // the input on the device (+1 held until the batch has copied it)
  bool out_refs = false; // outputs as device references
  Ref* out_ref[3] = {nullptr, nullptr, nullptr};
  double arrival_us = 0;
  OutBuf* outbuf = nullptr;  // outputs: slices of the batch's pinned buffer
  const uint32_t* out[3] = {nullptr, nullptr, nullptr};
  uint64_t out_n[3] = {0, 0, 0};
  std::mutex mu;
  std::condition_variable cv;
  bool done = false;
  int rc = KA_OK;
  void finish(int code) {
    {
      std::lock_guard<std::mutex> g(mu);
      rc = code;
      done = true;
    }
    cv.notify_all();
  }
  void release() {
    if (refs.fetch_sub(1) == 1) delete this;
  }
};

struct Batch {
  uint32_t si = 0;
  hipEvent_t done = nullptr;
  uint64_t budget = 0;
  std::vector<SrvReq*> reqs[3];  // by kind
  uint64_t n[3] = {0, 0, 0};
  void* d_buf = nullptr;
  uint64_t d_bytes = 0;
  uint64_t d_out = 0, d_chain = 0;  // device offsets of the output region and of the chain values
  void* h_tab = nullptr;  // pinned request tables
  OutBuf* out = nullptr;
  // host output layout
  uint64_t o_keys = 0, o_offs = 0, o_words = 0, o_ks = 0, o_ws = 0, o_lens = 0, o_bad = 0, o_scan = 0, o_chain = 0;
  int rc = KA_OK;
};

struct Server {
  System* sys = nullptr;
  uint32_t streams = 2, max_batch = 1024, value_bits = 12;
  uint64_t budget = 64ull << 30;
  uint64_t max_batch_bytes = 16ull << 20;
  std::vector<uint32_t> chain_a, chain_b;

  std::mutex mu;
  std::condition_variable cv_loop, cv_done;
  std::deque<SrvReq*> mailbox;
  std::deque<Batch*> inflight;
  uint64_t budget_in_use = 0, budget_peak = 0;
  uint32_t next_stream = 0;
  bool stop = false;
  bool loop_done = false;  // the mailbox thread has exited: no batch will be added
  std::thread loop, completion;

  CopyPool copier;

  std::mutex st_mu;
  std::vector<double> lat_us;
  uint64_t completed = 0, failed = 0, elements = 0, batches = 0, batched_requests = 0;

  void run_loop();
  void run_completion();
  Batch* launch(std::vector<SrvReq*>& take, uint64_t bytes);
  void complete(Batch* b);
};

// Packs, copies and launches one batch on its stream; returns it with an
// event recorded after its output copies (b->rc holds a launch failure).
Batch* Server::launch(std::vector<SrvReq*>& take, uint64_t bytes) {
  Batch* b = new Batch();
  b->budget = bytes;
  b->si = next_stream;
  next_stream = (next_stream + 1) % streams;
  for (auto* r : take) {
    b->reqs[r->kind].push_back(r);
    b->n[r->kind] += r->n;
  }
  const uint64_t nw = b->n[KA_REQ_WAH], ns = b->n[KA_REQ_SCAN], nc = b->n[KA_REQ_CHAIN];
  const uint32_t rw = (uint32_t)b->reqs[KA_REQ_WAH].size(), rs = (uint32_t)b->reqs[KA_REQ_SCAN].size();

  // ---- device layout: inputs (values by kind, request tables), outputs, lengths ----
  uint64_t off = 0;
  auto place = [&](uint64_t bytes_) {
    const uint64_t o = off;
    off += align_up(bytes_ ? bytes_ : 4);
    return o;
  };
  const uint64_t d_vw = place(4 * nw), d_vs = place(4 * ns), d_vc = place(4 * nc);
  const uint64_t d_rw = place(4 * (rw + 1ull)), d_rs = place(4 * (rs + 1ull));
  // a request has at most 2^value_bits distinct values: that bounds the lookup tables
  const uint64_t dcap = value_bits >= 32 ? nw : std::min<uint64_t>(nw, (uint64_t)rw << value_bits);
  const uint64_t d_keys = place(4 * dcap), d_offs = place(4 * (dcap + rw)), d_words = place(8 * nw);
  const uint64_t d_ks = place(4 * (rw + 1ull)), d_ws = place(4 * (rw + 1ull)), d_lens = place(5 * 8);
  const uint64_t d_bad = place(4 * (rw + 1ull));  // per-request rejection flags
  const uint64_t d_scan = place(4 * ns);
  const uint64_t total = off;
  // host output layout: the WAH outputs and lengths in device order, then scan, then chain
  b->o_keys = 0;
  b->o_offs = d_offs - d_keys;
  b->o_words = d_words - d_keys;
  b->o_ks = d_ks - d_keys;
  b->o_ws = d_ws - d_keys;
  b->o_lens = d_lens - d_keys;
  b->o_bad = d_bad - d_keys;
  b->o_scan = d_scan - d_keys;
  b->d_out = d_keys;
  b->d_chain = d_vc;
  b->o_chain = total - d_keys;
  const uint64_t out_bytes = b->o_chain + 4 * nc;

  int rc = sys->pool.alloc(total, b->si, &b->d_buf, &b->d_bytes);
  if (rc) {
    b->rc = rc;
    return b;
  }
  b->h_tab = sys->stage.get(sys, 4 * (rw + 1ull) + 4 * (rs + 1ull));
  b->out = new OutBuf();
  b->out->sys = sys;
  b->out->p = sys->stage.get(sys, std::max<uint64_t>(out_bytes, 4));
  if (!b->h_tab || !b->out->p) {
    b->rc = set_error(KA_E_OOM, "server: pinned staging");
    return b;
  }
  // ---- request tables -----------------------------------------------------------------
  uint32_t* tab = static_cast<uint32_t*>(b->h_tab);
  auto table = [&](int k, uint32_t* t) {
    uint64_t pos = 0;
    uint32_t j = 0;
    for (auto* r : b->reqs[k]) {
      t[j++] = (uint32_t)pos;
      pos += r->n;
    }
    t[j] = (uint32_t)pos;
  };
  table(KA_REQ_WAH, tab);
  table(KA_REQ_SCAN, tab + rw + 1);

  char* dev = static_cast<char*>(b->d_buf);
  auto u32 = [&](uint64_t o) { return reinterpret_cast<uint32_t*>(dev + o); };
  {
    CmdEnv env(sys, b->si);
    hipStream_t s = env.stream();
    // each request's data from its pinned buffer to its place; then the tables
    hipError_t e = hipSuccess;
    const uint64_t kind_off[3] = {d_vw, d_vs, d_vc};
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      uint64_t pos = 0;
      for (auto* r : b->reqs[k]) {
        if (r->n && e == hipSuccess) {
          if (r->dref) {  // device input: ordered after its writer, copied on the device
            if ((rc = ref_use_on(r->dref, b->si, false))) {
              b->rc = rc;
              return b;
            }
            e = hipMemcpyAsync(dev + kind_off[k] + 4 * pos, r->dref->ptr, 4 * r->n, hipMemcpyDeviceToDevice, s);
          } else {
            e = hipMemcpyAsync(dev + kind_off[k] + 4 * pos, r->pin, 4 * r->n, hipMemcpyHostToDevice, s);
          }
        }
        pos += r->n;
      }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(dev + d_rw, tab, 4 * (rw + 1ull), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dev + d_rs, tab + rw + 1, 4 * (rs + 1ull), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b->rc = set_error(KA_E_DEVICE, "server: input copy");
      return b;
    }
    uint64_t* lens = reinterpret_cast<uint64_t*>(dev + d_lens);
    uint32_t biggest = 0;
    for (auto* r : b->reqs[KA_REQ_WAH]) biggest = std::max<uint32_t>(biggest, (uint32_t)r->n);
    if (rw)
      rc = launch_wah_batch(env, u32(d_vw), nw, u32(d_rw), rw, value_bits, u32(d_keys), u32(d_offs), u32(d_words),
                            u32(d_ks), u32(d_ws), lens, lens + 1, lens + 2, lens + 3, lens + 4, 0, biggest,
                            u32(d_bad));
    if (!rc && rs) rc = launch_segmented_scan(env, u32(d_vs), u32(d_scan), ns, u32(d_rs), rs);
    if (!rc && nc)
      rc = launch_affine_chain(env, u32(d_vc), nc, chain_a.data(), chain_b.data(), (uint32_t)chain_a.size());
    if (rc) {
      b->rc = rc;
      return b;
    }
    // outputs back: the WAH and scan region in one copy, the chain region in another
    e = hipMemcpyAsync(b->out->p, dev + d_keys, b->o_chain, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && nc)
      e = hipMemcpyAsync(static_cast<char*>(b->out->p) + b->o_chain, dev + d_vc, 4 * nc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) {
      b->done = sys->get_event(false);
      e = b->done ? hipEventRecord(b->done, s) : hipErrorOutOfMemory;
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      b->rc = set_error(KA_E_DEVICE, "server: output copy");
    }
  }
  return b;
}

// Splits a finished batch's outputs per request and frees its resources.
void Server::complete(Batch* b) {
  if (b->done && hipEventSynchronize(b->done) != hipSuccess) {
    (void)hipGetLastError();
    if (!b->rc) b->rc = KA_E_DEVICE;
  }
  if (b->rc && hipStreamSynchronize(sys->streams[b->si]->s) != hipSuccess)  // nothing may still read the staging
    (void)hipGetLastError();
  const double now = clock_us();
  if (b->out) b->out->refs.fetch_add(1);  // the batch's own hold while requests are finished
  const char* ho = b->out && b->out->p ? static_cast<const char*>(b->out->p) : nullptr;
  auto u32 = [&](uint64_t o) { return reinterpret_cast<const uint32_t*>(ho + o); };
  uint64_t lens[5] = {0, 0, 0, 0, 0};
  if (!b->rc && !b->reqs[KA_REQ_WAH].empty()) {
    std::memcpy(lens, ho + b->o_lens, sizeof(lens));
    if (lens[3] == 0) b->rc = KA_E_DEVICE;  // the batch's tables are missing
  }
  // Outputs wanted as device references: copied from the batch's device
  // buffer into refs of their own on the batch's stream, before the buffer
  // goes back to the pool (in stream order).
  const char* dev = static_cast<const char*>(b->d_buf);
  auto to_ref = [&](uint64_t dev_off, uint64_t count, Ref** out) -> int {
    Ref* nr = nullptr;
    int rc = ref_create(sys, KA_U32, count, b->si, false, &nr);
    if (rc) return rc;
    if (count && hipMemcpyAsync(nr->ptr, dev + dev_off, 4 * count, hipMemcpyDeviceToDevice,
                                sys->streams[b->si]->s) != hipSuccess) {
      (void)hipGetLastError();
      ref_release(nr);
      return set_error(KA_E_DEVICE, "server: result copy");
    }
    *out = nr;
    return KA_OK;
  };
  uint64_t done_ok = 0, done_bad = 0, elems = 0;
  std::vector<double> lat;
  for (int k = 0; k < 3; ++k) {
    uint64_t pos = 0;
    for (size_t j = 0; j < b->reqs[k].size(); ++j) {
      SrvReq* r = b->reqs[k][j];
      const uint64_t n = r->n;
      int rrc = b->rc;
      if (!rrc && k == KA_REQ_WAH && u32(b->o_bad)[j]) rrc = KA_E_ARG;  // a value at or above 2^value_bits
      if (!rrc) {
        if (k == KA_REQ_WAH) {
          const uint32_t* ks = u32(b->o_ks);
          const uint32_t* ws = u32(b->o_ws);
          const uint32_t k0 = ks[j], k1 = ks[j + 1], w0 = ws[j], w1 = ws[j + 1];
          r->out[0] = u32(b->o_keys) + k0;
          r->out_n[0] = k1 - k0;
          r->out[1] = u32(b->o_offs) + k0 + j;
          r->out_n[1] = k1 - k0 + 1;
          r->out[2] = u32(b->o_words) + w0;
          r->out_n[2] = w1 - w0;
        } else {
          r->out[0] = u32(k == KA_REQ_SCAN ? b->o_scan : b->o_chain) + pos;
          r->out_n[0] = n;
        }
        if (r->out_refs) {
          const int outs = k == KA_REQ_WAH ? 3 : 1;
          for (int i = 0; i < outs && !rrc; ++i) {
            const uint64_t at = k == KA_REQ_CHAIN ? b->d_chain + 4 * pos
                                                  : b->d_out + (uint64_t)((const char*)r->out[i] - ho);
            rrc = to_ref(at, r->out_n[i], &r->out_ref[i]);
          }
        }
      }
      if (!rrc) {
        b->out->refs.fetch_add(1);
        r->outbuf = b->out;
        ++done_ok;
        elems += n;
        lat.push_back(now - r->arrival_us);
      } else {
        ++done_bad;
      }
      pos += n;
      if (r->pin) {
        sys->stage.give_back(r->pin);
        r->pin = nullptr;
      }
      if (r->dref) {  // its copy into the batch is queued before any later use of the memory
        ref_release(r->dref);
        r->dref = nullptr;
      }
      r->finish(rrc);
      r->release();
    }
  }
  if (b->d_buf) sys->pool.release(b->d_buf, b->d_bytes, b->si, 1ull << b->si);
  if (b->h_tab) sys->stage.give_back(b->h_tab);
  if (b->out) b->out->release();  // the requests hold the pinned outputs from here on
  if (b->done) sys->put_event(b->done);
  {
    std::lock_guard<std::mutex> g(st_mu);
    completed += done_ok;
    failed += done_bad;
    elements += elems;
    batches += 1;
    batched_requests += done_ok + done_bad;
    lat_us.insert(lat_us.end(), lat.begin(), lat.end());
  }
  delete b;
}

void Server::run_loop() {
  (void)sys->use_device();
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_loop.wait(lk, [&] { return stop || (!mailbox.empty() && inflight.size() < streams); });
    if (stop) break;
    // admission: the oldest requests, while the budget holds them (one request
    // is admitted whenever nothing else holds memory)
    std::vector<SrvReq*> take;
    uint64_t bytes = 0, in_bytes = 0;
    while (!mailbox.empty() && take.size() < max_batch) {
      SrvReq* r = mailbox.front();
      const uint64_t need = request_bytes(r->kind, r->n);
      if (budget_in_use + bytes + need > budget && !(take.empty() && budget_in_use == 0)) break;
      if (!take.empty() && in_bytes + 4 * r->n > max_batch_bytes) break;
      take.push_back(r);
      bytes += need;
      in_bytes += 4 * r->n;
      mailbox.pop_front();
    }
    if (take.empty()) {  // wait for memory to be freed
      cv_loop.wait(lk, [&] { return stop || inflight.empty() || budget_in_use == 0; });
      continue;
    }
    budget_in_use += bytes;
    budget_peak = std::max(budget_peak, budget_in_use);
    lk.unlock();
    Batch* b = launch(take, bytes);
    lk.lock();
    inflight.push_back(b);
    cv_done.notify_all();
  }
  loop_done = true;
  cv_done.notify_all();
}

void Server::run_completion() {
  (void)sys->use_device();
  for (;;) {
    Batch* b = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_done.wait(lk, [&] { return !inflight.empty() || loop_done; });
      if (inflight.empty()) break;
      b = inflight.front();
    }
    const uint64_t bytes = b->budget;
    complete(b);
    {
      std::lock_guard<std::mutex> lk(mu);
      inflight.pop_front();
      budget_in_use -= bytes;
    }
    cv_loop.notify_all();
  }
}

}  // namespace ka

using namespace ka;

struct ka_server : Server {};
struct ka_srv_req : SrvReq {};

#define KA_GUARD_BEGIN try {
#define KA_GUARD_END                                              \
  }                                                               \
  catch (const std::bad_alloc&) {                                 \
    return set_error(KA_E_OOM, "host allocation failed");         \
  }                                                               \
  catch (...) {                                                   \
    return set_error(KA_E_DEVICE, "internal error");              \
  }

KA_API int ka_server_clock_us(double* now) {
  if (!now) return set_error(KA_E_ARG, "null argument");
  *now = clock_us();
  return KA_OK;
}

KA_API int ka_server_create(ka_system* sys, const ka_server_config* cfg, ka_server** out) {
  KA_GUARD_BEGIN
  if (!sys || !out) return set_error(KA_E_ARG, "null argument");
  int rc = sys->ensure_init();
  if (rc) return rc;
  ka_server* s = new ka_server();
  s->sys = sys;
  const uint32_t want = cfg && cfg->streams ? cfg->streams : 2;
  s->streams = std::max<uint32_t>(1, std::min<uint32_t>(want, (uint32_t)sys->streams.size()));
  s->max_batch = cfg && cfg->max_batch ? cfg->max_batch : 1024;
  s->max_batch_bytes = cfg && cfg->max_batch_bytes ? cfg->max_batch_bytes : (16ull << 20);
  s->budget = cfg && cfg->hbm_budget_bytes ? cfg->hbm_budget_bytes : (64ull << 30);
  s->value_bits = cfg && cfg->value_bits ? cfg->value_bits : 12;
  const uint32_t req_bits = s->max_batch > 1 ? 32u - (uint32_t)__builtin_clz(s->max_batch - 1) : 0u;
  if (s->value_bits > 32 || s->value_bits + req_bits > 32) {
    delete s;
    return set_error(KA_E_ARG, "value_bits + bits of max_batch - 1 exceed 32");
  }
  const uint32_t len = cfg && cfg->chain_len ? cfg->chain_len : 0;
  if (len && (!cfg->chain_a || !cfg->chain_b)) {
    delete s;
    return set_error(KA_E_ARG, "chain parameters missing");
  }
  for (uint32_t i = 0; i < len; ++i) {
    s->chain_a.push_back(cfg->chain_a[i]);
    s->chain_b.push_back(cfg->chain_b[i]);
  }
  // Warm the caches the batches draw from: per stream slot two device blocks,
  // and two pinned buffers, of every power of two from 1 MiB up to what a
  // full batch needs, taken and given back at once.  A cached block of up to
  // twice a size class is reused, so the first batches of every size find
  // memory cached instead of calling hipMalloc / hipHostMalloc, which take
  // milliseconds and stall the mailbox or submitting thread meanwhile.  (A
  // block the pool's budget refuses is skipped.)
  {
    const uint64_t dev_top = request_bytes(KA_REQ_WAH, s->max_batch_bytes / 4);
    const uint64_t pin_top = 4 * s->max_batch_bytes;  // a full batch's outputs
    for (uint32_t si = 0; si < s->streams; ++si)
      for (uint64_t b = 1ull << 20; b < 2 * dev_top; b <<= 1) {
        void* p[2] = {nullptr, nullptr};
        uint64_t got[2] = {0, 0};
        for (int k = 0; k < 2; ++k)
          if (sys->pool.alloc(b, si, &p[k], &got[k]) != KA_OK) p[k] = nullptr;
        for (int k = 0; k < 2; ++k)
          if (p[k]) sys->pool.release(p[k], got[k], si, 1ull << si);
      }
    for (uint64_t b = 1ull << 20; b < 2 * pin_top; b <<= 1) {
      void* p[2] = {sys->stage.get(sys, b), sys->stage.get(sys, b)};
      for (int k = 0; k < 2; ++k)
        if (p[k]) sys->stage.give_back(p[k]);
    }
  }
  s->copier.start(cfg && cfg->copy_threads ? std::min<uint32_t>(cfg->copy_threads - 1, 64) : 3);
  sys->retain();
  s->loop = std::thread([s] { s->run_loop(); });
  s->completion = std::thread([s] { s->run_completion(); });
  *out = s;
  return KA_OK;
  KA_GUARD_END
}

namespace {

// Queues one request: host data (copied into pinned memory here) or a device
// reference (retained until its batch has copied it).
int server_enqueue(ka_server* srv, uint32_t kind, const uint32_t* data, Ref* dref, uint64_t n, double arrival_us,
                   bool out_refs, SrvReq** out) {
  if (kind > KA_REQ_CHAIN) return set_error(KA_E_ARG, "unknown request kind");
  if (n >= (1ull << 30)) return set_error(KA_E_ARG, "n must be below 2^30");
  if (request_bytes(kind, n) > srv->budget) return set_error(KA_E_BUDGET, "request larger than the server budget");
  ka_srv_req* r = new ka_srv_req();
  r->sys = srv->sys;
  r->kind = kind;
  r->n = n;
  r->out_refs = out_refs;
  if (n && data) {
    r->pin = srv->sys->stage.get(srv->sys, 4 * n);
    if (!r->pin) {
      delete r;
      return set_error(KA_E_OOM, "server: pinned staging");
    }
    const uint32_t shift = kind == KA_REQ_WAH ? srv->value_bits : 32u;
    if (srv->copier.copy(static_cast<uint32_t*>(r->pin), data, n, shift)) {
      delete r;
      return set_error(KA_E_ARG, "an index value is at or above 2^value_bits");
    }
  }
  if (dref) {
    ref_retain(dref);
    r->dref = dref;
  }
  r->arrival_us = arrival_us > 0 ? arrival_us : clock_us();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) {
      delete r;
      return set_error(KA_E_STATE, "server is shutting down");
    }
    srv->mailbox.push_back(r);
  }
  srv->cv_loop.notify_all();
  *out = r;
  return KA_OK;
}

// A ticket answered by a served request: waits on the request, then hands its
// outputs on as host values (slices of the batch's pinned outputs, kept alive
// by the ticket) or as the device references made for it.
struct ServedTicket final : HostCompletion {
  explicit ServedTicket(SrvReq* req) : r(req) {}
  ~ServedTicket() override { r->release(); }
  int wait(Ticket* t, int64_t timeout_us) override {
    {
      std::unique_lock<std::mutex> lk(r->mu);
      if (timeout_us < 0) {
        r->cv.wait(lk, [&] { return r->done; });
      } else if (!r->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return r->done; })) {
        return set_error(KA_E_TIMEOUT, "response not ready");
      }
    }
    if (r->rc) {
      t->status = r->rc;
      return set_error(r->rc, "request failed");
    }
    std::lock_guard<std::mutex> g(mu);
    if (!filled) {
      for (size_t i = 0; i < t->outs.size(); ++i) {
        MsgVal& v = t->outs[i];
        v.dtype = KA_U32;
        if (r->out_refs) {
          v.mode = KA_REF;
          v.ref = r->out_ref[i];  // the ticket takes the request's reference
          r->out_ref[i] = nullptr;
        } else {
          v.mode = KA_VAL;
          v.host = r->out[i];
          v.count = r->out_n[i];
        }
      }
      filled = true;
    }
    return KA_OK;
  }
  SrvReq* r;
  std::mutex mu;
  bool filled = false;
};

}  // namespace

KA_API int ka_server_submit(ka_server* srv, uint32_t kind, const uint32_t* data, uint64_t n, double arrival_us,
                            ka_srv_req** out) {
  KA_GUARD_BEGIN
  if (!srv || !out || (n && !data)) return set_error(KA_E_ARG, "null argument");
  SrvReq* r = nullptr;
  int rc = server_enqueue(srv, kind, n ? data : nullptr, nullptr, n, arrival_us, false, &r);
  if (rc) return rc;
  *out = static_cast<ka_srv_req*>(r);
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_server_send(ka_server* srv, uint32_t kind, const ka_value* in, uint32_t nin, uint32_t flags,
                          double arrival_us, ka_ticket** out) {
  KA_GUARD_BEGIN
  if (!srv || !out || !in) return set_error(KA_E_ARG, "null argument");
  if (nin != 1) return set_error(KA_E_ARITY, "a served request is one message element");
  if (flags & ~KA_SRV_OUTPUT_REFS) return set_error(KA_E_ARG, "unknown flags");
  const ka_value& v = in[0];
  const uint32_t* data = nullptr;
  Ref* dref = nullptr;
  uint64_t n = 0;
  if (v.mode == KA_VAL) {
    if (v.dtype != KA_U32) return set_error(KA_E_TYPE, "served requests take uint32 data");
    if (v.count && !v.ptr) return set_error(KA_E_ARG, "null value data");
    data = static_cast<const uint32_t*>(v.ptr);
    n = v.count;
  } else if (v.mode == KA_REF) {
    if (!v.ref) return set_error(KA_E_ARG, "null reference");
    if (v.ref->sys != srv->sys) return set_error(KA_E_ARG, "reference of another system");
    if (v.ref->dtype != KA_U32) return set_error(KA_E_TYPE, "served requests take uint32 data");
    dref = v.ref;
    int rc = ref_length(dref, &n);
    if (rc) return rc;
  } else {
    return set_error(KA_E_ARG, "unknown value mode");
  }
  SrvReq* r = nullptr;
  int rc = server_enqueue(srv, kind, n ? data : nullptr, n ? dref : nullptr, n, arrival_us,
                          (flags & KA_SRV_OUTPUT_REFS) != 0, &r);
  if (rc) return rc;
  ka_ticket* t = new ka_ticket();
  t->sys = srv->sys;
  srv->sys->retain();
  t->outs.resize(kind == KA_REQ_WAH ? 3 : 1);
  t->hc = new ServedTicket(r);  // holds the caller's reference of the request
  *out = t;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_server_wait(ka_srv_req* req, int64_t timeout_us) {
  if (!req) return set_error(KA_E_ARG, "null request");
  std::unique_lock<std::mutex> lk(req->mu);
  if (timeout_us < 0) {
    req->cv.wait(lk, [&] { return req->done; });
  } else if (!req->cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return req->done; })) {
    return set_error(KA_E_TIMEOUT, "request not finished");
  }
  if (req->rc) return set_error(req->rc, "request failed");
  return KA_OK;
}

KA_API int ka_server_result(ka_srv_req* req, uint32_t i, uint32_t* host, uint64_t cap, uint64_t* count) {
  if (!req || !count) return set_error(KA_E_ARG, "null argument");
  {
    std::lock_guard<std::mutex> g(req->mu);
    if (!req->done) return set_error(KA_E_STATE, "request not finished");
    if (req->rc) return set_error(req->rc, "request failed");
  }
  const uint32_t outs = req->kind == KA_REQ_WAH ? 3 : 1;
  if (i >= outs) return set_error(KA_E_ARG, "no such output");
  *count = req->out_n[i];
  if (!host) return KA_OK;
  if (cap < req->out_n[i]) return set_error(KA_E_ARG, "buffer too small");
  if (req->out_n[i]) std::memcpy(host, req->out[i], 4 * req->out_n[i]);
  return KA_OK;
}

KA_API int ka_server_request_release(ka_srv_req* req) {
  if (!req) return set_error(KA_E_ARG, "null request");
  req->release();
  return KA_OK;
}

KA_API int ka_server_get_stats(ka_server* srv, ka_server_stats* out) {
  if (!srv || !out) return set_error(KA_E_ARG, "null argument");
  std::vector<double> lat;
  ka_server_stats st{};
  {
    std::lock_guard<std::mutex> g(srv->st_mu);
    lat = srv->lat_us;
    st.completed = srv->completed;
    st.failed = srv->failed;
    st.elements = srv->elements;
    st.batches = srv->batches;
    st.mean_batch = srv->batches ? (double)srv->batched_requests / srv->batches : 0.0;
  }
  {
    std::lock_guard<std::mutex> g(srv->mu);
    st.queued = srv->mailbox.size();
    st.budget_in_use = srv->budget_in_use;
    st.budget_peak = srv->budget_peak;
  }
  if (!lat.empty()) {
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) { return lat[std::min<size_t>(lat.size() - 1, (size_t)(p * (lat.size() - 1) + 0.5))]; };
    st.p50_us = pct(0.50);
    st.p99_us = pct(0.99);
    st.max_us = lat.back();
    double s = 0;
    for (double x : lat) s += x;
    st.mean_us = s / lat.size();
  }
  *out = st;
  return KA_OK;
}

KA_API int ka_server_reset_stats(ka_server* srv) {
  if (!srv) return set_error(KA_E_ARG, "null argument");
  std::lock_guard<std::mutex> g(srv->st_mu);
  srv->lat_us.clear();
  srv->completed = srv->failed = srv->elements = srv->batches = srv->batched_requests = 0;
  {
    std::lock_guard<std::mutex> g2(srv->mu);
    srv->budget_peak = srv->budget_in_use;
  }
  return KA_OK;
}

KA_API int ka_server_destroy(ka_server* srv) {
  if (!srv) return set_error(KA_E_ARG, "null server");
  std::deque<SrvReq*> cancelled;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    cancelled.swap(srv->mailbox);
  }
  srv->cv_loop.notify_all();
  srv->cv_done.notify_all();
  if (srv->loop.joinable()) srv->loop.join();  // no batch is launched after this
  srv->cv_done.notify_all();
  if (srv->completion.joinable()) srv->completion.join();  // in-flight batches finish first
  srv->copier.stop();  // no submission may still run (the caller's contract)
  for (auto* r : cancelled) {
    r->finish(KA_E_CANCELLED);
    r->release();
  }
  System* sys = srv->sys;
  delete srv;
  sys->release();
  return KA_OK;
}
