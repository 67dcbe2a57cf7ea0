// Host runtime of the kernel actors: system and lazy device initialisation,
// stream-ordered device memory pool, references, programs, kernel actors,
// composition, messaging and the C ABI of ka.h.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "runtime_internal.hpp"

namespace ka {

int launch_copy_len(Env& env, uint64_t* dst, const uint64_t* src);

// ---------------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------------
static thread_local std::string t_last_error;

int set_error(int code, const std::string& msg) {
  t_last_error = msg;
  return code;
}

static int hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // a handled failure must not stay pending for later HIP users (torch)
  return set_error(KA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define KA_HIP(expr, what)                           \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

uint32_t dtype_size(uint32_t dtype) {
  switch (dtype) {
    case KA_U32:
    case KA_I32:
    case KA_F32:
      return 4;
    case KA_U64:
      return 8;
    case KA_U8:
      return 1;
    default:
      return 0;
  }
}

// ---------------------------------------------------------------------------------
// system
// ---------------------------------------------------------------------------------
int System::use_device() {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != cfg.device) KA_HIP(hipSetDevice(cfg.device), "hipSetDevice");
  return KA_OK;
}

int System::ensure_init() {
  if (destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  std::lock_guard<std::mutex> g(init_mu);
  if (inited) {
    if (init_rc) set_error(init_rc, init_err);
    return init_rc ? init_rc : use_device();
  }
  inited = true;
  auto fail = [&](int code, const std::string& msg) {
    init_rc = code;
    init_err = msg;
    return set_error(code, msg);
  };
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    (void)hipGetLastError();
    return fail(KA_E_DEVICE, "no HIP device available");
  }
  if (cfg.device < 0 || cfg.device >= count) return fail(KA_E_DEVICE, "device ordinal out of range");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg.device) != hipSuccess) return fail(KA_E_DEVICE, "device query failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(KA_E_DEVICE, std::string("device is ") + prop.gcnArchName + ", kernels are built for gfx950");
  if (hipSetDevice(cfg.device) != hipSuccess) return fail(KA_E_DEVICE, "hipSetDevice failed");
  const uint32_t ns = cfg.n_streams ? cfg.n_streams : 1;
  for (uint32_t i = 0; i < ns; ++i) {
    auto sc = std::make_unique<StreamCtx>();
    if (i == 0 && cfg.stream) {
      sc->s = static_cast<hipStream_t>(cfg.stream);
      sc->owned = false;
    } else {
      if (hipStreamCreateWithFlags(&sc->s, hipStreamNonBlocking) != hipSuccess)
        return fail(KA_E_DEVICE, "stream creation failed");
      sc->owned = true;
    }
    streams.push_back(std::move(sc));
  }
  pool.init(this, cfg.hbm_budget_bytes);
  // Look-back spin limit: polls of a silent predecessor tile before its total
  // is computed from its input instead (1 = at once; for tests of that path).
  if (const char* e = std::getenv("KA_LOOKBACK_SPIN")) {
    const long v = std::strtol(e, nullptr, 10);
    lb_spin = v < 1 ? 1u : v > 1000000 ? 1000000u : (uint32_t)v;
  }
  // Per-stream sort plan storage (the status words come from the pool on first use).
  for (auto& sc : streams) {
    void* p = nullptr;
    if (hipMalloc(&p, kSortPlanBytes) != hipSuccess) return fail(KA_E_OOM, "arena allocation failed");
    if (hipMemset(p, 0, kSortPlanBytes) != hipSuccess) return fail(KA_E_DEVICE, "arena clear failed");
    sc->arena.plan = p;
  }
  init_rc = KA_OK;
  return KA_OK;
}

hipEvent_t System::get_event(bool timing) {
  {
    std::lock_guard<std::mutex> g(ev_mu);
    auto& pool = timing ? timing_events : events;
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void System::put_event(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> g(ev_mu);
  events.push_back(e);
}

void System::put_timing_event(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> g(ev_mu);
  timing_events.push_back(e);
}

// Profile records are folded in launch order; the events go back to the
// timing pool, so a long profiled run holds a bounded number of them.
void System::prof_fold_locked(bool all) {
  size_t k = 0;
  for (; k < prof_pending.size(); ++k) {
    ProfRec& p = prof_pending[k];
    if (all) {
      hipEventSynchronize(p.b);
    } else if (hipEventQuery(p.b) != hipSuccess) {
      (void)hipGetLastError();  // "not ready" must not stay pending
      break;
    }
    float ms = 0.f;
    hipEventElapsedTime(&ms, p.a, p.b);
    auto& acc = prof_acc[p.name];
    acc.first += 1;
    acc.second += ms;
    put_timing_event(p.a);
    put_timing_event(p.b);
  }
  prof_pending.erase(prof_pending.begin(), prof_pending.begin() + k);
}

void System::release() {
  if (rc.fetch_sub(1) == 1) delete static_cast<ka_system*>(this);
}

// ---------------------------------------------------------------------------------
// pool
// ---------------------------------------------------------------------------------
uint64_t Pool::size_class(uint64_t bytes) {
  if (bytes <= 256) return 256;
  if (bytes <= (1ull << 20)) {
    uint64_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  const uint64_t g = 2ull << 20;
  return (bytes + g - 1) / g * g;
}

void Pool::init(System* sys, uint64_t budget) {
  sys_ = sys;
  budget_ = budget;
  free_.assign(sys->streams.size(), {});
}

void Pool::poll_deferred_locked() {
  for (size_t i = 0; i < deferred_.size();) {
    Deferred& d = deferred_[i];
    bool done = true;
    for (hipEvent_t e : d.events)
      if (hipEventQuery(e) != hipSuccess) {
        (void)hipGetLastError();  // "not ready" must not stay pending
        done = false;
      }
    if (done) {
      for (hipEvent_t e : d.events) sys_->put_event(e);
      free_[d.home].emplace(d.bytes, d.p);
      deferred_[i] = deferred_.back();
      deferred_.pop_back();
    } else {
      ++i;
    }
  }
}

int Pool::trim_locked() {
  // Give cached blocks back to the device (all work must be done first).
  for (auto& sc : sys_->streams) hipStreamSynchronize(sc->s);
  poll_deferred_locked();
  for (auto& fl : free_) {
    for (auto& kv : fl) {
      hipFree(kv.second);
      all_.erase(kv.second);
      reserved_ -= kv.first;
    }
    fl.clear();
  }
  return KA_OK;
}

int Pool::alloc(uint64_t bytes, uint32_t stream, void** out, uint64_t* got) {
  const uint64_t c = size_class(bytes);
  std::lock_guard<std::mutex> g(mu_);
  if (!deferred_.empty()) poll_deferred_locked();
  // a free block of the size class or up to twice it (batches of varying
  // size then reuse blocks instead of calling hipMalloc each time)
  auto& fl = free_[stream];
  auto it = fl.lower_bound(c);
  if (it != fl.end() && it->first <= 2 * c) {
    *out = it->second;
    *got = it->first;
    in_use_ += it->first;
    fl.erase(it);
    return KA_OK;
  }
  if (budget_ && in_use_ + c > budget_)
    return set_error(KA_E_BUDGET, "HBM budget exceeded (" + std::to_string(in_use_ + c) + " > " +
                                      std::to_string(budget_) + " bytes)");
  if (budget_ && reserved_ + c > budget_) trim_locked();
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    trim_locked();
    e = hipMalloc(&p, c);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(KA_E_OOM, "device allocation of " + std::to_string(c) + " bytes failed");
    }
  }
  reserved_ += c;
  in_use_ += c;
  all_[p] = c;
  *out = p;
  *got = c;
  return KA_OK;
}

void Pool::release(void* p, uint64_t bytes, uint32_t home, uint64_t used_mask) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  in_use_ -= bytes;
  used_mask &= ~(1ull << home);
  if (!used_mask) {
    free_[home].emplace(bytes, p);
    return;
  }
  Deferred d{p, bytes, home, {}};
  for (uint32_t s = 0; s < sys_->streams.size(); ++s) {
    if (!((used_mask >> s) & 1ull)) continue;
    hipEvent_t e = sys_->get_event();
    if (e && hipEventRecord(e, sys_->streams[s]->s) == hipSuccess) d.events.push_back(e);
  }
  deferred_.push_back(std::move(d));
}

void Pool::destroy() {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& d : deferred_)
    for (hipEvent_t e : d.events) hipEventDestroy(e);
  deferred_.clear();
  for (auto& fl : free_) fl.clear();
  for (auto& kv : all_) hipFree(kv.first);  // also blocks still held by live refs
  all_.clear();
  reserved_ = in_use_ = 0;
}

// ---------------------------------------------------------------------------------
// pinned host staging
// ---------------------------------------------------------------------------------
// A free buffer of the size class, or of up to twice it, is reused; otherwise
// a new one is allocated -- outside the lock, since pinning takes
// milliseconds for large buffers and other threads (request submission, the
// mailbox thread) take buffers meanwhile.
void* HostStage::get(System* sys, uint64_t bytes) {
  const uint64_t c = Pool::size_class(bytes);
  {
    std::lock_guard<std::mutex> g(mu_);
    for (size_t i = 0; i < busy_.size();) {
      const hipError_t q = hipEventQuery(busy_[i].done);
      if (q != hipSuccess) (void)hipGetLastError();  // "not ready" must not stay pending
      if (q == hipSuccess) {
        sys->put_event(busy_[i].done);
        free_.emplace(busy_[i].bytes, busy_[i].p);
        busy_[i] = busy_.back();
        busy_.pop_back();
      } else {
        ++i;
      }
    }
    auto it = free_.lower_bound(c);
    if (it != free_.end() && it->first <= 2 * c) {
      void* p = it->second;
      free_.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> g(mu_);
  sizes_[p] = c;
  return p;
}

void HostStage::retire(System* sys, void* p, hipEvent_t done) {
  (void)sys;
  std::lock_guard<std::mutex> g(mu_);
  busy_.push_back({p, sizes_[p], done});
}

void HostStage::give_back(void* p) {
  std::lock_guard<std::mutex> g(mu_);
  free_.emplace(sizes_[p], p);
}

void HostStage::destroy(System* sys) {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& b : busy_) {
    hipEventSynchronize(b.done);
    sys->put_event(b.done);
    free_.emplace(b.bytes, b.p);
  }
  busy_.clear();
  for (auto& kv : free_) hipHostFree(kv.second);
  free_.clear();
  sizes_.clear();
}

// ---------------------------------------------------------------------------------
// references
// ---------------------------------------------------------------------------------
int ref_create(System* sys, uint32_t dtype, uint64_t count, uint32_t si, bool device_len, Ref** out) {
  const uint32_t es = dtype_size(dtype);
  if (!es) return set_error(KA_E_TYPE, "unknown dtype");
  const uint64_t data = (count * es + 255) / 256 * 256;
  void* p = nullptr;
  uint64_t got = 0;
  int rc = sys->pool.alloc(data + 256, si, &p, &got);
  if (rc) return rc;
  ka_ref* r = new ka_ref();
  r->sys = sys;
  sys->retain();
  r->dtype = dtype;
  r->ptr = p;
  r->cap = count;
  r->alloc_bytes = got;
  r->borrowed = false;
  r->d_len = reinterpret_cast<uint64_t*>(static_cast<char*>(p) + data);
  r->len_known.store(!device_len);
  r->len = count;
  r->home = si;
  r->used_mask.store(1ull << si);
  *out = r;
  return KA_OK;
}

void ref_retain(Ref* r) { r->rc.fetch_add(1); }

void ref_release(Ref* r) {
  if (!r || r->rc.fetch_sub(1) != 1) return;
  System* sys = r->sys;
  if (!r->borrowed && !sys->destroyed.load()) sys->pool.release(r->ptr, r->alloc_bytes, r->home, r->used_mask.load());
  Ref* parent = r->parent;
  delete static_cast<ka_ref*>(r);
  sys->release();
  if (parent) ref_release(parent);
}

int ref_view(Ref* parent, uint64_t offset, uint64_t count, Ref** out) {
  const uint32_t es = dtype_size(parent->dtype);
  if (offset > parent->cap || count > parent->cap - offset) return set_error(KA_E_ARG, "view beyond its buffer");
  ka_ref* r = new ka_ref();
  r->sys = parent->sys;
  parent->sys->retain();
  r->dtype = parent->dtype;
  r->access = KA_ACCESS_READ;
  r->ptr = static_cast<char*>(parent->ptr) + offset * es;
  r->cap = count;
  r->borrowed = true;
  r->len_known.store(true);
  r->len = count;
  r->home = parent->home;
  r->used_mask.store(parent->used_mask.load());
  ref_retain(parent);
  r->parent = parent;
  *out = r;
  return KA_OK;
}

int ref_sync(Ref* r) {
  System* sys = r->sys;
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  int rc = sys->ensure_init();
  if (rc) return rc;
  const uint64_t m = r->used_mask.load() | (1ull << r->home);
  for (uint32_t s = 0; s < sys->streams.size(); ++s)
    if ((m >> s) & 1ull) KA_HIP(hipStreamSynchronize(sys->streams[s]->s), "stream synchronize");
  return KA_OK;
}

int ref_length(Ref* r, uint64_t* len) {
  if (r->len_known.load()) {
    *len = r->len;
    return KA_OK;
  }
  int rc = ref_sync(r);
  if (rc) return rc;
  r->sys->length_reads.fetch_add(1);
  uint64_t v = 0;
  KA_HIP(hipMemcpy(&v, r->d_len, sizeof(v), hipMemcpyDeviceToHost), "length read-back");
  if (v > r->cap) v = r->cap;
  r->len = v;
  r->len_known.store(true);
  *len = v;
  return KA_OK;
}

int ref_use_on(Ref* r, uint32_t si, bool write) {
  System* sys = r->sys;
  // A read waits for the last writer; a write also waits for every stream that
  // may still be reading the buffer (no write-after-read across streams).
  uint64_t wait = write ? (r->used_mask.load() | (1ull << r->home)) : (1ull << r->home);
  wait &= ~(1ull << si);
  for (uint32_t s = 0; wait && s < sys->streams.size(); ++s) {
    if (!((wait >> s) & 1ull)) continue;
    hipEvent_t e = sys->get_event();
    if (!e) return set_error(KA_E_DEVICE, "event creation failed");
    KA_HIP(hipEventRecord(e, sys->streams[s]->s), "hipEventRecord");
    KA_HIP(hipStreamWaitEvent(sys->streams[si]->s, e, 0), "hipStreamWaitEvent");
    sys->put_event(e);  // reusable: the wait is already queued
  }
  // After a write on si every earlier use is ordered before si's later work.
  if (write)
    r->used_mask.store(1ull << si);
  else
    r->used_mask.fetch_or(1ull << si);
  for (Ref* p = r->parent; p; p = p->parent) p->used_mask.fetch_or(1ull << si);  // the memory is the parent's
  return KA_OK;
}

// ---------------------------------------------------------------------------------
// the launch environment
// ---------------------------------------------------------------------------------

// ---------------------------------------------------------------------------------
// messages
// ---------------------------------------------------------------------------------
void msg_clear(Msg& m) {
  for (auto& v : m)
    if (v.ref) ref_release(v.ref);
  m.clear();
}

static bool is_input(uint32_t dir) { return dir == KA_IN || dir == KA_IN_OUT; }
static bool is_output(uint32_t dir) { return dir == KA_OUT || dir == KA_IN_OUT; }

// Host copy of a value result that is still on the device (value semantics
// between stages: the data make a round trip through the host, Sec. 3.5).
static int materialize(MsgVal& v) {
  if (v.mode != KA_VAL || !v.ref) return KA_OK;
  uint64_t len = 0;
  int rc = ref_length(v.ref, &len);
  if (!rc) rc = ref_sync(v.ref);  // the producer runs on a non-blocking stream
  if (rc) return rc;
  const uint32_t es = dtype_size(v.ref->dtype);
  auto buf = std::make_shared<std::vector<uint8_t>>(len * es);
  if (len) KA_HIP(hipMemcpy(buf->data(), v.ref->ptr, len * es, hipMemcpyDeviceToHost), "value read-back");
  v.dtype = v.ref->dtype;
  v.owned = buf;
  v.host = buf->data();
  v.count = len;
  ref_release(v.ref);
  v.ref = nullptr;
  return KA_OK;
}

static void to_c_values(const Msg& m, std::vector<ka_value>& out) {
  out.clear();
  for (const auto& v : m) {
    ka_value c{};
    c.mode = v.mode;
    if (v.ref && v.mode == KA_REF) {
      c.ref = static_cast<ka_ref*>(v.ref);
      c.dtype = v.ref->dtype;
      c.count = v.ref->len_known.load() ? v.ref->len : v.ref->cap;
    } else {
      c.dtype = v.dtype;
      c.ptr = const_cast<void*>(v.host);
      c.count = v.count;
    }
    out.push_back(c);
  }
}

int msg_from_values(const ka_value* vals, uint32_t n, Msg& out) {
  out.clear();
  for (uint32_t i = 0; i < n; ++i) {
    const ka_value& c = vals[i];
    MsgVal v;
    v.mode = c.mode;
    if (c.mode == KA_REF) {
      if (!c.ref) return set_error(KA_E_ARG, "REF value without a reference");
      v.ref = c.ref;
      v.dtype = c.ref->dtype;
      ref_retain(v.ref);
    } else if (c.mode == KA_VAL) {
      const uint32_t es = dtype_size(c.dtype);
      if (!es) return set_error(KA_E_TYPE, "VAL value with an unknown dtype");
      if (c.count && !c.ptr) return set_error(KA_E_ARG, "VAL value without data");
      v.dtype = c.dtype;
      v.count = c.count;
      v.host = c.ptr;
    } else {
      return set_error(KA_E_ARG, "unknown value mode");
    }
    out.push_back(std::move(v));
  }
  return KA_OK;
}

// Applies a mapping function: `m` is replaced by its result.  Value results
// still on the device are read back first: a mapping function sees values as
// host data (Sec. 3.4).
static int apply_map(ka_map_fn fn, void* ud, Msg& m) {
  for (auto& v : m) {
    const int rc = materialize(v);
    if (rc) {
      msg_clear(m);
      return rc;
    }
  }
  std::vector<ka_value> in;
  to_c_values(m, in);
  const uint32_t cap = 64;
  std::vector<ka_value> out(cap);
  uint32_t n_out = 0;
  int rc = fn(in.data(), (uint32_t)in.size(), out.data(), &n_out, cap, ud);
  if (rc) {
    msg_clear(m);
    return set_error(rc < 0 ? rc : KA_E_ARG, "mapping function failed");
  }
  if (n_out > cap) n_out = cap;
  Msg res;
  rc = msg_from_values(out.data(), n_out, res);
  // VAL data returned by the function are only valid during the call: copy.
  for (auto& v : res) {
    if (v.mode == KA_VAL && !v.ref && v.count) {
      auto buf = std::make_shared<std::vector<uint8_t>>((const uint8_t*)v.host,
                                                        (const uint8_t*)v.host + v.count * dtype_size(v.dtype));
      v.owned = buf;
      v.host = buf->data();
    }
  }
  msg_clear(m);
  if (rc) {
    msg_clear(res);
    return rc;
  }
  m = std::move(res);
  return KA_OK;
}

// Uploads a host value into a fresh device buffer on stream si.
int msg_upload(System* sys, const MsgVal& v, uint32_t si, Ref** out) {
  Ref* r = nullptr;
  int rc = ref_create(sys, v.dtype, v.count, si, false, &r);
  if (rc) return rc;
  const uint64_t bytes = v.count * dtype_size(v.dtype);
  if (bytes) {
    void* st = sys->stage.get(sys, bytes);
    if (!st) {
      ref_release(r);
      return set_error(KA_E_OOM, "pinned staging allocation failed");
    }
    std::memcpy(st, v.host, bytes);
    hipStream_t s = sys->streams[si]->s;
    hipError_t e = hipMemcpyAsync(r->ptr, st, bytes, hipMemcpyHostToDevice, s);
    hipEvent_t done = sys->get_event();
    if (e == hipSuccess && done) e = hipEventRecord(done, s);
    if (e != hipSuccess || !done) {
      hipStreamSynchronize(s);
      if (done) sys->put_event(done);
      sys->stage.give_back(st);
      ref_release(r);
      return e != hipSuccess ? hip_fail(e, "value upload") : set_error(KA_E_DEVICE, "event creation failed");
    }
    sys->stage.retire(sys, st, done);
  }
  *out = r;
  return KA_OK;
}

// ---------------------------------------------------------------------------------
// kernel actor: one message -> one command
// ---------------------------------------------------------------------------------
static int launch_module(Actor* a, CmdEnv& env, std::vector<Bound>& args, uint64_t n) {
  // Packed kernel arguments, each aligned to its size.
  std::vector<uint8_t> buf;
  auto put = [&](const void* p, size_t sz) {
    size_t off = (buf.size() + sz - 1) / sz * sz;
    buf.resize(off + sz);
    std::memcpy(buf.data() + off, p, sz);
  };
  uint32_t lds = 0;
  for (size_t i = 0; i < a->sig.size(); ++i) {
    const ka_arg& s = a->sig[i].a;
    if (s.dir == KA_LOCAL) {
      put(&args[i].lds_offset, 4);
      lds = std::max<uint32_t>(lds, args[i].lds_offset + (uint32_t)(s.count * dtype_size(s.dtype)));
    } else if (s.dir == KA_PRIV) {
      const auto& v = a->sig[i].init;
      const uint32_t es = dtype_size(s.dtype);
      for (size_t off = 0; off + es <= v.size(); off += es) put(v.data() + off, es);
    } else {
      put(&args[i].ptr, 8);
    }
  }
  ka_nd_range_dev nd{};
  uint32_t grid[3] = {1, 1, 1}, block[3] = {1, 1, 1};
  const uint32_t dims = a->range.dims ? a->range.dims : 1;
  const uint32_t defl[3][3] = {{256, 1, 1}, {16, 16, 1}, {8, 8, 4}};
  for (uint32_t d = 0; d < 3; ++d) {
    uint64_t g = d < dims ? a->range.global[d] : 1;
    if (d == 0 && g == 0) g = n;
    nd.global[d] = g;
    nd.offset[d] = d < dims ? a->range.offset[d] : 0;
    block[d] = d < dims ? (a->range.local[d] ? a->range.local[d] : defl[dims - 1][d]) : 1;
    const uint64_t gb = (g + block[d] - 1) / block[d];
    if (gb > 0x7FFFFFFFull) return set_error(KA_E_ARG, "ND-range too large");
    grid[d] = gb ? (uint32_t)gb : 1u;
  }
  if (nd.global[0] == 0 || nd.global[1] == 0 || nd.global[2] == 0) return KA_OK;  // empty index space
  {
    const size_t off = (buf.size() + 7) / 8 * 8;  // the struct is 8-byte aligned
    buf.resize(off + sizeof(nd));
    std::memcpy(buf.data() + off, &nd, sizeof(nd));
  }
  size_t sz = buf.size();
  void* cfg[] = {HIP_LAUNCH_PARAM_BUFFER_POINTER, buf.data(), HIP_LAUNCH_PARAM_BUFFER_SIZE, &sz,
                 HIP_LAUNCH_PARAM_END};
  env.prof_begin(a->kernel.c_str());
  hipError_t e = hipModuleLaunchKernel(a->fn, grid[0], grid[1], grid[2], block[0], block[1], block[2], lds,
                                       env.stream(), nullptr, cfg);
  env.prof_end(a->kernel.c_str());
  if (e != hipSuccess) return set_error(KA_E_LAUNCH, std::string("module kernel launch: ") + hipGetErrorString(e));
  return KA_OK;
}

static int run_kernel_actor(Actor* a, Msg& msg, Msg& out, uint32_t si) {
  System* sys = a->sys;
  std::lock_guard<std::mutex> lock(a->mu);
  int rc = KA_OK;
  if (a->pre && (rc = apply_map(a->pre, a->map_ud, msg))) return rc;

  // ---- match the message against the in / in_out arguments (Sec. 3.4) ----
  std::vector<size_t> in_idx;
  for (size_t i = 0; i < a->sig.size(); ++i)
    if (is_input(a->sig[i].a.dir)) in_idx.push_back(i);
  if (msg.size() != in_idx.size()) {
    msg_clear(msg);
    return set_error(KA_E_ARITY, "actor " + a->kernel + " expects " + std::to_string(in_idx.size()) +
                                     " message elements, got " + std::to_string(msg.size()));
  }
  for (size_t j = 0; j < in_idx.size(); ++j) {
    const ka_arg& s = a->sig[in_idx[j]].a;
    const MsgVal& v = msg[j];
    const uint32_t dt = v.ref ? v.ref->dtype : v.dtype;
    if (v.mode != s.in_mode || dt != s.dtype) {
      msg_clear(msg);
      return set_error(KA_E_TYPE, "actor " + a->kernel + ": message element " + std::to_string(j) +
                                      " does not match the signature (mode/dtype)");
    }
    if (v.mode == KA_VAL && v.ref) {
      // a value result still on the device: value semantics go through the host
      if ((rc = materialize(msg[j]))) {
        msg_clear(msg);
        return rc;
      }
    }
  }
  rc = sys->ensure_init();
  if (rc) {
    msg_clear(msg);
    return rc;
  }

  // ---- work-items ---------------------------------------------------------
  std::vector<Bound> args(a->sig.size());
  std::vector<Ref*> temps;  // uploaded values not handed on
  auto cleanup = [&]() {
    for (auto& b : args)
      if (b.ref) ref_release(b.ref);
    for (Ref* t : temps) ref_release(t);
    msg_clear(msg);
  };
  // Bind inputs.
  for (size_t j = 0; j < in_idx.size(); ++j) {
    const size_t i = in_idx[j];
    MsgVal& v = msg[j];
    Bound& b = args[i];
    Ref* r = nullptr;
    if (v.mode == KA_VAL) {
      if ((rc = msg_upload(sys, v, si, &r))) {
        cleanup();
        return rc;
      }
    } else {
      r = v.ref;
      ref_retain(r);
      if ((rc = ref_use_on(r, si, a->sig[i].a.dir == KA_IN_OUT))) {
        ref_release(r);
        cleanup();
        return rc;
      }
    }
    b.ref = r;
    b.ptr = r->ptr;
    b.cap = r->cap;
    if (r->len_known.load()) {
      b.len = r->len;
      b.d_len = nullptr;
    } else {
      b.len = r->cap;
      b.d_len = r->d_len;
    }
  }
  uint64_t n = a->range.global[0];
  const uint64_t* d_n = nullptr;
  if (n == 0 && !in_idx.empty()) {
    const Bound& b0 = args[in_idx[0]];
    n = b0.len;
    d_n = b0.d_len;
    if (d_n && a->bk && a->bk->needs_host_n) {
      // The kernel plans its launch on the host: read the length (a sync).
      uint64_t len = 0;
      if ((rc = ref_length(b0.ref, &len))) {
        cleanup();
        return rc;
      }
      n = len;
      d_n = nullptr;
    }
  }
  // Bind outputs, local and private arguments.
  std::vector<ka_value> cin;
  bool have_cin = false;
  uint32_t lds_off = 0;
  for (size_t i = 0; i < a->sig.size(); ++i) {
    const SigArg& s = a->sig[i];
    Bound& b = args[i];
    if (s.a.dir == KA_OUT) {
      uint64_t cap = s.a.count;
      if (s.a.size_fn) {
        if (!have_cin) {
          to_c_values(msg, cin);
          have_cin = true;
        }
        cap = s.a.size_fn(cin.data(), (uint32_t)cin.size(), s.a.size_ud);
      }
      const bool dlen = (a->bk && a->bk->device_len((uint32_t)i)) || (d_n != nullptr);
      if (a->bk) {
        const uint64_t need = a->bk->default_cap((uint32_t)i, n, args);
        if (cap == 0) cap = need;
        if (cap < need) {
          cleanup();
          return set_error(KA_E_ARG, "actor " + a->kernel + ": output " + std::to_string(i) + " needs capacity " +
                                         std::to_string(need));
        }
      } else if (cap == 0) {
        cap = n;  // default: one element per work-item (Sec. 3.4)
      }
      Ref* r = nullptr;
      if ((rc = ref_create(sys, s.a.dtype, cap, si, dlen, &r))) {
        cleanup();
        return rc;
      }
      if (!dlen) r->len = (a->bk ? std::min<uint64_t>(n, cap) : cap);
      b.ref = r;
      b.ptr = r->ptr;
      b.cap = cap;
      b.d_len = dlen ? r->d_len : nullptr;
    } else if (s.a.dir == KA_LOCAL) {
      b.lds_offset = lds_off;
      lds_off += (uint32_t)((s.a.count * dtype_size(s.a.dtype) + 15) / 16 * 16);
    } else if (s.a.dir == KA_PRIV) {
      const uint32_t es = dtype_size(s.a.dtype);
      for (size_t k = 0; k < 4 && (k + 1) * es <= s.init.size(); ++k) {
        uint64_t v = 0;
        std::memcpy(&v, s.init.data() + k * es, es);
        b.priv[k] = v;
      }
    }
  }

  // ---- launch ----------------------------------------------------------------
  {
    CmdEnv env(sys, si);
    if (a->bk) {
      LaunchCtx c{&env, n, d_n, &a->range, &args};
      rc = a->bk->launch(c);
      // Default-sized outputs of a device-counted range get the same count.
      if (!rc && d_n) {
        for (size_t i = 0; i < a->sig.size() && !rc; ++i)
          if (a->sig[i].a.dir == KA_OUT && !a->bk->device_len((uint32_t)i))
            rc = launch_copy_len(env, const_cast<uint64_t*>(args[i].d_len), d_n);
      }
    } else {
      rc = launch_module(a, env, args, n);
    }
  }
  if (rc) {
    cleanup();
    return rc;
  }
  // Writers become the home stream of their buffers.
  for (size_t i = 0; i < a->sig.size(); ++i)
    if (is_output(a->sig[i].a.dir) && args[i].ref) args[i].ref->home = si;

  // ---- response: in_out and out arguments in order (Sec. 3.4) -------------
  out.clear();
  for (size_t i = 0; i < a->sig.size(); ++i) {
    const ka_arg& s = a->sig[i].a;
    if (!is_output(s.dir)) continue;
    MsgVal v;
    v.mode = s.out_mode;
    v.dtype = s.dtype;
    v.ref = args[i].ref;
    ref_retain(v.ref);
    out.push_back(std::move(v));
  }
  cleanup();
  if (a->post && (rc = apply_map(a->post, a->map_ud, out))) return rc;
  return KA_OK;
}

int actor_run(Actor* a, Msg& in, Msg& out, uint32_t si) {
  if (!a->composed) return run_kernel_actor(a, in, out, si);
  int rc = KA_OK;
  if (a->pre && (rc = apply_map(a->pre, a->map_ud, in))) return rc;
  Msg cur = std::move(in);
  in.clear();
  for (Actor* st : a->stages) {
    Msg next;
    rc = actor_run(st, cur, next, si);
    msg_clear(cur);
    if (rc) {
      msg_clear(next);
      return rc;
    }
    cur = std::move(next);
  }
  out = std::move(cur);
  if (a->post && (rc = apply_map(a->post, a->map_ud, out))) return rc;
  return KA_OK;
}

}  // namespace ka

// =================================================================================
// C ABI
// =================================================================================
using namespace ka;

#define KA_GUARD_BEGIN try {
#define KA_GUARD_END                                                      \
  }                                                                       \
  catch (const std::bad_alloc&) {                                         \
    return set_error(KA_E_OOM, "host allocation failed");                 \
  }                                                                       \
  catch (...) {                                                           \
    return set_error(KA_E_DEVICE, "unexpected internal error");           \
  }

extern "C" {

KA_API const char* ka_error_string(int code) {
  switch (code) {
    case KA_OK:
      return "ok";
    case KA_E_ARG:
      return "invalid argument";
    case KA_E_TYPE:
      return "type mismatch";
    case KA_E_ARITY:
      return "arity mismatch";
    case KA_E_NOKERNEL:
      return "no such kernel";
    case KA_E_DEVICE:
      return "device error";
    case KA_E_OOM:
      return "out of memory";
    case KA_E_BUDGET:
      return "HBM budget exceeded";
    case KA_E_TIMEOUT:
      return "timeout";
    case KA_E_NOT_SERIALIZABLE:
      return "device references are not serializable";
    case KA_E_LAUNCH:
      return "kernel launch failed";
    case KA_E_CANCELLED:
      return "cancelled";
    case KA_E_STATE:
      return "invalid state";
    default:
      return "unknown error";
  }
}

KA_API const char* ka_last_error(void) { return t_last_error.c_str(); }

// ---- system ----------------------------------------------------------------------
KA_API int ka_system_create(const ka_system_config* cfg, ka_system** out) {
  KA_GUARD_BEGIN
  if (!out) return set_error(KA_E_ARG, "null out");
  if (cfg && (cfg->device < 0 || cfg->n_streams > 64)) return set_error(KA_E_ARG, "bad system configuration");
  ka_system* s = new ka_system();
  if (cfg) s->cfg = *cfg;
  if (s->cfg.n_streams == 0) s->cfg.n_streams = 1;
  s->profile = (s->cfg.flags & KA_SYS_PROFILE) != 0;
  *out = s;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_system_destroy(ka_system* sys) {
  KA_GUARD_BEGIN
  if (!sys) return set_error(KA_E_ARG, "null system");
  if (sys->destroyed.exchange(true)) return set_error(KA_E_STATE, "system already destroyed");
  {
    std::lock_guard<std::mutex> g(sys->wah_mu);
    for (auto& row : sys->wah_actor)
      for (auto& a : row)
        if (a) {
          ka_actor_release(static_cast<ka_actor*>(a));
          a = nullptr;
        }
    if (sys->builtin) {
      ka_program_release(static_cast<ka_program*>(sys->builtin));
      sys->builtin = nullptr;
    }
  }
  if (sys->inited && sys->init_rc == KA_OK) {
    sys->use_device();
    for (auto& sc : sys->streams) hipStreamSynchronize(sc->s);
    {
      std::lock_guard<std::mutex> g(sys->prof_mu);
      for (auto& p : sys->prof_pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
      }
      sys->prof_pending.clear();
    }
    sys->stage.destroy(sys);
    for (auto& sc : sys->streams) {
      sc->arena.status = nullptr;  // a pool block, freed with the pool below
      hipFree(sc->arena.plan);
    }
    sys->pool.destroy();
    {
      std::lock_guard<std::mutex> g(sys->ev_mu);
      for (hipEvent_t e : sys->events) hipEventDestroy(e);
      for (hipEvent_t e : sys->timing_events) hipEventDestroy(e);
      sys->timing_events.clear();
      sys->events.clear();
    }
    for (auto& sc : sys->streams)
      if (sc->owned) hipStreamDestroy(sc->s);
  }
  sys->release();
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_system_synchronize(ka_system* sys) {
  KA_GUARD_BEGIN
  if (!sys) return set_error(KA_E_ARG, "null system");
  int rc = sys->ensure_init();
  if (rc) return rc;
  for (auto& sc : sys->streams) KA_HIP(hipStreamSynchronize(sc->s), "stream synchronize");
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_system_stream(ka_system* sys, uint32_t i, void** stream) {
  KA_GUARD_BEGIN
  if (!sys || !stream) return set_error(KA_E_ARG, "null argument");
  int rc = sys->ensure_init();
  if (rc) return rc;
  if (i >= sys->streams.size()) return set_error(KA_E_ARG, "stream index out of range");
  *stream = sys->streams[i]->s;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_system_memory(ka_system* sys, uint64_t* in_use, uint64_t* reserved) {
  if (!sys) return set_error(KA_E_ARG, "null system");
  if (in_use) *in_use = sys->pool.in_use();
  if (reserved) *reserved = sys->pool.reserved();
  return KA_OK;
}

KA_API int ka_system_length_reads(ka_system* sys, uint64_t* count) {
  if (!sys || !count) return set_error(KA_E_ARG, "null argument");
  *count = sys->length_reads.load();
  return KA_OK;
}

// ---- programs --------------------------------------------------------------------
KA_API int ka_program_builtin(ka_system* sys, ka_program** out) {
  KA_GUARD_BEGIN
  if (!sys || !out) return set_error(KA_E_ARG, "null argument");
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  ka_program* p = new ka_program();
  p->sys = sys;
  sys->retain();
  p->builtin = true;
  *out = p;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_program_load(ka_system* sys, const char* path, ka_program** out) {
  KA_GUARD_BEGIN
  if (!sys || !path || !out) return set_error(KA_E_ARG, "null argument");
  int rc = sys->ensure_init();
  if (rc) return rc;
  hipModule_t m = nullptr;
  hipError_t e = hipModuleLoad(&m, path);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_ARG, std::string("cannot load code object ") + path);
  }
  ka_program* p = new ka_program();
  p->sys = sys;
  sys->retain();
  p->builtin = false;
  p->module = m;
  p->path = path;
  *out = p;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_program_release(ka_program* prog) {
  if (!prog) return set_error(KA_E_ARG, "null program");
  if (prog->rc.fetch_sub(1) == 1) {
    System* sys = prog->sys;
    if (prog->module && !sys->destroyed.load()) {
      sys->use_device();
      hipModuleUnload(prog->module);
    }
    delete prog;
    sys->release();
  }
  return KA_OK;
}

// ---- actors ----------------------------------------------------------------------
KA_API int ka_spawn(ka_system* sys, ka_program* prog, const char* kernel, const ka_nd_range* range,
                    const ka_arg* sig, uint32_t nargs, ka_actor** out) {
  KA_GUARD_BEGIN
  if (!sys || !prog || !kernel || !out || (nargs && !sig)) return set_error(KA_E_ARG, "null argument");
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  if (prog->sys != sys) return set_error(KA_E_ARG, "program belongs to another system");
  ka_nd_range rg{};
  rg.dims = 1;
  if (range) rg = *range;
  if (rg.dims < 1 || rg.dims > 3) return set_error(KA_E_ARG, "ND-range needs 1..3 dimensions");
  const BuiltinKernel* bk = nullptr;
  hipFunction_t fn = nullptr;
  if (prog->builtin) {
    bk = find_builtin(kernel);
    if (!bk) return set_error(KA_E_NOKERNEL, std::string("no built-in kernel named ") + kernel);
    if (nargs != bk->sig.size())
      return set_error(KA_E_ARITY, std::string(kernel) + " takes " + std::to_string(bk->sig.size()) + " arguments");
    for (uint32_t i = 0; i < nargs; ++i)
      if (sig[i].dir != bk->sig[i].first || sig[i].dtype != bk->sig[i].second)
        return set_error(KA_E_TYPE, std::string(kernel) + ": argument " + std::to_string(i) +
                                        " has the wrong direction or dtype");
    if (rg.dims != 1) return set_error(KA_E_ARG, "built-in kernels use a 1-D range");
    if (rg.local[0] != 0) return set_error(KA_E_ARG, "built-in kernels choose their own work-group size");
    if (rg.offset[0] != 0 && std::string(kernel) != "affine_u32")
      return set_error(KA_E_ARG, "only affine_u32 accepts a global offset");
  } else {
    int rc = sys->ensure_init();
    if (rc) return rc;
    hipError_t e = hipModuleGetFunction(&fn, prog->module, kernel);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_error(KA_E_NOKERNEL, std::string("no kernel named ") + kernel + " in module");
    }
  }
  std::vector<SigArg> s(nargs);
  for (uint32_t i = 0; i < nargs; ++i) {
    const ka_arg& a = sig[i];
    if (a.dir < KA_IN || a.dir > KA_PRIV) return set_error(KA_E_ARG, "bad argument direction");
    if (!dtype_size(a.dtype)) return set_error(KA_E_TYPE, "bad argument dtype");
    if ((a.in_mode > KA_REF) || (a.out_mode > KA_REF)) return set_error(KA_E_ARG, "bad argument mode");
    s[i].a = a;
    if (a.dir == KA_PRIV) {
      if (!a.init || a.count == 0) return set_error(KA_E_ARG, "priv argument needs an initial value");
      const uint8_t* b = static_cast<const uint8_t*>(a.init);
      s[i].init.assign(b, b + a.count * dtype_size(a.dtype));
      s[i].a.init = nullptr;
    }
    if (a.dir == KA_LOCAL && a.count == 0) return set_error(KA_E_ARG, "local argument needs a size");
  }
  ka_actor* act = new ka_actor();
  act->sys = sys;
  sys->retain();
  act->prog = prog;
  prog->rc.fetch_add(1);
  act->bk = bk;
  act->fn = fn;
  act->kernel = kernel;
  act->range = rg;
  act->sig = std::move(s);
  *out = act;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_actor_set_mapping(ka_actor* actor, ka_map_fn pre, ka_map_fn post, void* ud) {
  if (!actor) return set_error(KA_E_ARG, "null actor");
  std::lock_guard<std::mutex> g(actor->mu);
  actor->pre = pre;
  actor->post = post;
  actor->map_ud = ud;
  return KA_OK;
}

// (mode, dtype) of the response of an actor / the message it accepts.
static void response_shape(Actor* a, std::vector<std::pair<uint32_t, uint32_t>>& r) {
  if (a->composed) return response_shape(a->stages.back(), r);
  r.clear();
  for (auto& s : a->sig)
    if (is_output(s.a.dir)) r.emplace_back(s.a.out_mode, s.a.dtype);
}
static void message_shape(Actor* a, std::vector<std::pair<uint32_t, uint32_t>>& r) {
  if (a->composed) return message_shape(a->stages.front(), r);
  r.clear();
  for (auto& s : a->sig)
    if (is_input(s.a.dir)) r.emplace_back(s.a.in_mode, s.a.dtype);
}
static bool has_mapping(Actor* a) {
  if (a->pre || a->post) return true;
  for (Actor* s : a->stages)
    if (has_mapping(s)) return true;
  return false;
}

KA_API int ka_compose(ka_actor* outer, ka_actor* inner, ka_actor** out) {
  KA_GUARD_BEGIN
  if (!outer || !inner || !out) return set_error(KA_E_ARG, "null argument");
  if (outer->sys != inner->sys) return set_error(KA_E_ARG, "actors belong to different systems");
  if (!has_mapping(outer) && !has_mapping(inner)) {
    std::vector<std::pair<uint32_t, uint32_t>> resp, msg;
    response_shape(inner, resp);
    message_shape(outer, msg);
    if (resp.size() != msg.size())
      return set_error(KA_E_TYPE, "the inner actor's response does not match the outer actor's message (arity)");
    for (size_t i = 0; i < resp.size(); ++i)
      if (resp[i] != msg[i])
        return set_error(KA_E_TYPE, "the inner actor's response element " + std::to_string(i) +
                                        " does not match the outer actor's message (mode/dtype)");
  }
  ka_actor* c = new ka_actor();
  c->sys = outer->sys;
  c->sys->retain();
  c->composed = true;
  c->kernel = "(" + outer->kernel + " . " + inner->kernel + ")";
  c->stream = inner->stream;
  inner->rc.fetch_add(1);
  outer->rc.fetch_add(1);
  c->stages = {inner, outer};
  *out = c;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_actor_retain(ka_actor* actor) {
  if (!actor) return set_error(KA_E_ARG, "null actor");
  actor->rc.fetch_add(1);
  return KA_OK;
}

KA_API int ka_actor_release(ka_actor* actor) {
  if (!actor) return set_error(KA_E_ARG, "null actor");
  if (actor->rc.fetch_sub(1) == 1) {
    for (Actor* s : actor->stages) ka_actor_release(static_cast<ka_actor*>(s));
    if (actor->prog) ka_program_release(static_cast<ka_program*>(actor->prog));
    System* sys = actor->sys;
    delete actor;
    sys->release();
  }
  return KA_OK;
}

KA_API int ka_actor_set_stream(ka_actor* actor, uint32_t stream) {
  if (!actor) return set_error(KA_E_ARG, "null actor");
  if (stream >= actor->sys->cfg.n_streams) return set_error(KA_E_ARG, "stream index out of range");
  actor->stream = stream;
  return KA_OK;
}

// ---- messaging -------------------------------------------------------------------
KA_API int ka_send(ka_actor* actor, const ka_value* args, uint32_t nargs, ka_ticket** out) {
  KA_GUARD_BEGIN
  if (!actor || !out || (nargs && !args)) return set_error(KA_E_ARG, "null argument");
  System* sys = actor->sys;
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  Msg in, res;
  int rc = msg_from_values(args, nargs, in);
  if (rc) {
    msg_clear(in);
    return rc;
  }
  const uint32_t si = actor->stream;
  rc = actor_run(actor, in, res, si);
  msg_clear(in);
  if (rc) {
    msg_clear(res);
    return rc;
  }
  ka_ticket* t = new ka_ticket();
  t->sys = sys;
  sys->retain();
  t->outs = std::move(res);
  t->stream = si;
  if (sys->inited && sys->init_rc == KA_OK) {
    t->done = sys->get_event();
    if (t->done) hipEventRecord(t->done, sys->streams[si]->s);
  }
  *out = t;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_send_as(ka_actor* target, ka_actor* reply_to, const ka_value* args, uint32_t nargs, ka_ticket** out) {
  KA_GUARD_BEGIN
  if (!target || !reply_to || !out || (nargs && !args)) return set_error(KA_E_ARG, "null argument");
  System* sys = target->sys;
  if (reply_to->sys != sys) return set_error(KA_E_ARG, "actors of different systems");
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  Msg in, mid, res;
  int rc = msg_from_values(args, nargs, in);
  if (rc) {
    msg_clear(in);
    return rc;
  }
  // target's response becomes reply_to's message, on each actor's own stream
  rc = actor_run(target, in, mid, target->stream);
  msg_clear(in);
  if (!rc) rc = actor_run(reply_to, mid, res, reply_to->stream);
  msg_clear(mid);
  if (rc) {
    msg_clear(res);
    return rc;
  }
  const uint32_t si = reply_to->stream;
  ka_ticket* t = new ka_ticket();
  t->sys = sys;
  sys->retain();
  t->outs = std::move(res);
  t->stream = si;
  if (sys->inited && sys->init_rc == KA_OK) {
    t->done = sys->get_event();
    if (t->done) hipEventRecord(t->done, sys->streams[si]->s);
  }
  *out = t;
  return KA_OK;
  KA_GUARD_END
}

static int ticket_wait(ka_ticket* t, int64_t timeout_us) {
  if (t->hc) return t->hc->wait(t, timeout_us);
  if (t->complete.load() || !t->done) return KA_OK;
  if (timeout_us < 0) {
    KA_HIP(hipEventSynchronize(t->done), "waiting for the response");
    t->complete.store(true);
    return KA_OK;
  }
  const auto until = std::chrono::steady_clock::now() + std::chrono::microseconds(timeout_us);
  for (;;) {
    hipError_t e = hipEventQuery(t->done);
    if (e == hipSuccess) {
      t->complete.store(true);
      return KA_OK;
    }
    if (e != hipErrorNotReady) return hip_fail(e, "waiting for the response");
    (void)hipGetLastError();
    if (std::chrono::steady_clock::now() >= until) return set_error(KA_E_TIMEOUT, "response not ready");
    std::this_thread::yield();
  }
}

KA_API int ka_receive(ka_ticket* t, ka_value* outs, uint32_t nouts, int64_t timeout_us) {
  KA_GUARD_BEGIN
  if (!t || (nouts && !outs)) return set_error(KA_E_ARG, "null argument");
  System* sys = t->sys;
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  if (t->status) return set_error(t->status, "request failed");
  if (nouts != t->outs.size())
    return set_error(KA_E_ARITY, "the response has " + std::to_string(t->outs.size()) + " elements");
  if (sys->inited && sys->init_rc == KA_OK) {
    int rc = sys->use_device();
    if (rc) return rc;
  }
  int rc = ticket_wait(t, timeout_us);
  if (rc) return rc;
  if (t->status) return set_error(t->status, "request failed");
  int result = KA_OK;
  for (uint32_t i = 0; i < nouts; ++i) {
    MsgVal& v = t->outs[i];
    ka_value& o = outs[i];
    if (v.mode == KA_REF) {
      o.mode = KA_REF;
      o.dtype = v.ref->dtype;
      ref_retain(v.ref);
      o.ref = static_cast<ka_ref*>(v.ref);
      o.count = v.ref->len_known.load() ? v.ref->len : v.ref->cap;
      continue;
    }
    // VAL: produced count, copied if a large enough buffer is given
    uint64_t len = 0;
    const void* src_host = nullptr;
    uint32_t dt = v.dtype;
    if (v.ref) {
      if ((rc = ref_length(v.ref, &len))) return rc;
      dt = v.ref->dtype;
    } else {
      len = v.count;
      src_host = v.host;
    }
    const uint32_t es = dtype_size(dt);
    o.mode = KA_VAL;
    o.dtype = dt;
    if (o.ptr) {
      if (o.count < len) {
        o.count = len;
        result = set_error(KA_E_ARG, "receive buffer too small");
        continue;
      }
      if (len) {
        if (v.ref)
          KA_HIP(hipMemcpy(o.ptr, v.ref->ptr, len * es, hipMemcpyDeviceToHost), "result read-back");
        else
          std::memcpy(o.ptr, src_host, len * es);
      }
    }
    o.count = len;
  }
  return result;
  KA_GUARD_END
}

KA_API int ka_ticket_arity(ka_ticket* t, uint32_t* n) {
  if (!t || !n) return set_error(KA_E_ARG, "null argument");
  *n = (uint32_t)t->outs.size();
  return KA_OK;
}

KA_API int ka_ticket_release(ka_ticket* t) {
  if (!t) return set_error(KA_E_ARG, "null ticket");
  if (t->rc.fetch_sub(1) == 1) {
    System* sys = t->sys;
    msg_clear(t->outs);
    delete t->hc;
    if (t->done) {
      if (!sys->destroyed.load())
        sys->put_event(t->done);
    }
    delete t;
    sys->release();
  }
  return KA_OK;
}

// ---- references --------------------------------------------------------------------
KA_API int ka_ref_info(ka_ref* ref, uint32_t* dtype, uint64_t* count, uint32_t* access) {
  KA_GUARD_BEGIN
  if (!ref) return set_error(KA_E_ARG, "null ref");
  if (count) {
    if (ref->sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
    uint64_t len = 0;
    int rc = ref_length(ref, &len);
    if (rc) return rc;
    *count = len;
  }
  if (dtype) *dtype = ref->dtype;
  if (access) *access = ref->access;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_ref_capacity(ka_ref* ref, uint64_t* capacity) {
  if (!ref || !capacity) return set_error(KA_E_ARG, "null argument");
  *capacity = ref->cap;
  return KA_OK;
}

KA_API int ka_ref_read(ka_ref* ref, void* host, uint64_t bytes) {
  KA_GUARD_BEGIN
  if (!ref || (bytes && !host)) return set_error(KA_E_ARG, "null argument");
  if (ref->sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  int rc = ref->sys->ensure_init();
  if (rc) return rc;
  uint64_t len = 0;
  if ((rc = ref_length(ref, &len))) return rc;
  if ((rc = ref_sync(ref))) return rc;
  const uint64_t n = std::min<uint64_t>(bytes, len * dtype_size(ref->dtype));
  if (n) KA_HIP(hipMemcpy(host, ref->ptr, n, hipMemcpyDeviceToHost), "ref read");
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_ref_device_ptr(ka_ref* ref, void** dptr) {
  if (!ref || !dptr) return set_error(KA_E_ARG, "null argument");
  *dptr = ref->ptr;
  return KA_OK;
}

KA_API int ka_ref_wrap(ka_system* sys, void* dptr, uint32_t dtype, uint64_t count, uint32_t access, ka_ref** out) {
  KA_GUARD_BEGIN
  if (!sys || !out || (count && !dptr)) return set_error(KA_E_ARG, "null argument");
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  if (!dtype_size(dtype)) return set_error(KA_E_TYPE, "bad dtype");
  ka_ref* r = new ka_ref();
  r->sys = sys;
  sys->retain();
  r->dtype = dtype;
  r->access = access ? access : KA_ACCESS_RW;
  r->ptr = dptr;
  r->cap = count;
  r->len = count;
  r->borrowed = true;
  r->home = 0;
  r->used_mask.store(1ull);
  *out = r;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_ref_alloc(ka_system* sys, uint32_t dtype, uint64_t count, ka_ref** out) {
  KA_GUARD_BEGIN
  if (!sys || !out) return set_error(KA_E_ARG, "null argument");
  int rc = sys->ensure_init();
  if (rc) return rc;
  Ref* r = nullptr;
  if ((rc = ref_create(sys, dtype, count, 0, false, &r))) return rc;
  *out = static_cast<ka_ref*>(r);
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_ref_retain(ka_ref* ref) {
  if (!ref) return set_error(KA_E_ARG, "null ref");
  ref_retain(ref);
  return KA_OK;
}

KA_API int ka_ref_release(ka_ref* ref) {
  if (!ref) return set_error(KA_E_ARG, "null ref");
  ref_release(ref);
  return KA_OK;
}

KA_API int ka_ref_serialize(const ka_ref* ref, void* buf, uint64_t cap, uint64_t* len) {
  (void)ref;
  (void)buf;
  (void)cap;
  (void)len;
  return set_error(KA_E_NOT_SERIALIZABLE, "device references are bound to this process");
}

// ---- the composed WAH index ---------------------------------------------------------
// The built-in wah_index actor (sort of (value, row) pairs, then the encoder)
// with a value-bits hint and a word format; one actor per pair, kept by the
// system.
static int wah_actor(ka_system* sys, uint32_t value_bits, uint32_t format, ka_actor** out) {
  std::lock_guard<std::mutex> g(sys->wah_mu);
  if (!sys->wah_actor[value_bits][format]) {
    if (!sys->builtin) {
      ka_program* p = nullptr;
      int rc = ka_program_builtin(sys, &p);
      if (rc) return rc;
      sys->builtin = p;  // released by ka_system_destroy
    }
    ka_program* prog = static_cast<ka_program*>(sys->builtin);
    ka_arg sig[5] = {};
    sig[0] = {KA_IN, KA_U32, KA_REF, KA_REF, 0, nullptr, nullptr, nullptr};
    const uint32_t priv[2] = {value_bits, format};
    sig[1] = {KA_PRIV, KA_U32, KA_VAL, KA_VAL, 2, nullptr, nullptr, priv};
    for (int i = 2; i < 5; ++i) sig[i] = {KA_OUT, KA_U32, KA_REF, KA_REF, 0, nullptr, nullptr, nullptr};
    ka_nd_range r{};
    r.dims = 1;
    ka_actor* act = nullptr;
    int rc = ka_spawn(sys, prog, "wah_index", &r, sig, 5, &act);
    if (rc) return rc;
    sys->wah_actor[value_bits][format] = act;  // released by ka_system_destroy
  }
  *out = static_cast<ka_actor*>(sys->wah_actor[value_bits][format]);
  return KA_OK;
}

// The lengths of an index's three outputs (written on the device by one launch,
// so on one stream) in one round trip: three 8-byte copies into pinned memory,
// one synchronisation.  Each becomes the ref's host-known length.
static int read_lengths3(System* sys, Ref* const r[3], uint64_t len[3]) {
  const uint32_t home = r[0]->home;
  if (r[1]->home != home || r[2]->home != home) {
    for (int i = 0; i < 3; ++i) {
      int rc = ref_length(r[i], &len[i]);
      if (rc) return rc;
    }
    return KA_OK;
  }
  uint64_t* hl = static_cast<uint64_t*>(sys->stage.get(sys, 3 * sizeof(uint64_t)));
  if (!hl) return set_error(KA_E_OOM, "pinned staging");
  hipStream_t s = sys->streams[home]->s;
  hipError_t e = hipSuccess;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    if (r[i]->len_known.load())
      hl[i] = r[i]->len;
    else
      e = hipMemcpyAsync(&hl[i], r[i]->d_len, sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sys->stage.give_back(hl);
    return set_error(KA_E_DEVICE, "length read-back");
  }
  for (int i = 0; i < 3; ++i) {
    if (!r[i]->len_known.load()) {
      sys->length_reads.fetch_add(1);
      r[i]->len = std::min<uint64_t>(hl[i], r[i]->cap);
      r[i]->len_known.store(true);
    }
    len[i] = r[i]->len;
  }
  sys->stage.give_back(hl);
  return KA_OK;
}

// Host copies of three outputs of one stream after their lengths are known:
// through one pinned staging buffer and one synchronisation when they are
// small, else one blocking copy each.
static int read_outputs3(System* sys, Ref* const r[3], void* const dst[3], const uint64_t bytes[3]) {
  constexpr uint64_t kStagedMax = 8ull << 20;
  const uint64_t total = bytes[0] + bytes[1] + bytes[2];
  const uint32_t home = r[0]->home;
  if (total == 0) return KA_OK;
  if (total > kStagedMax || r[1]->home != home || r[2]->home != home) {
    for (int i = 0; i < 3; ++i) {
      int rc = bytes[i] ? ka_ref_read(static_cast<ka_ref*>(r[i]), dst[i], bytes[i]) : KA_OK;
      if (rc) return rc;
    }
    return KA_OK;
  }
  char* st = static_cast<char*>(sys->stage.get(sys, total));
  if (!st) return set_error(KA_E_OOM, "pinned staging");
  hipStream_t s = sys->streams[home]->s;
  hipError_t e = hipSuccess;
  uint64_t off = 0;
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    if (bytes[i]) e = hipMemcpyAsync(st + off, r[i]->ptr, bytes[i], hipMemcpyDeviceToHost, s);
    off += bytes[i];
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    sys->stage.give_back(st);
    return set_error(KA_E_DEVICE, "result read-back");
  }
  off = 0;
  for (int i = 0; i < 3; ++i) {
    if (bytes[i]) std::memcpy(dst[i], st + off, bytes[i]);
    off += bytes[i];
  }
  sys->stage.give_back(st);
  return KA_OK;
}

KA_API int ka_wah_index(ka_system* sys, const uint32_t* values, uint64_t n, uint32_t flags, ka_wah_result* out) {
  KA_GUARD_BEGIN
  if (!sys || !out || (n && !values)) return set_error(KA_E_ARG, "null argument");
  if (n >= (1ull << 30)) return set_error(KA_E_ARG, "n must be below 2^30");
  const uint32_t value_bits = (flags >> 8) & 0xFFu;
  const uint32_t format = (flags >> 16) & 0xFFu;
  if (value_bits > 32) return set_error(KA_E_ARG, "KA_WAH_VALUE_BITS must be 0..32");
  if (format > 2) return set_error(KA_E_ARG, "KA_WAH_FORMAT must be 0..2");
  int rc = sys->ensure_init();
  if (rc) return rc;
  ka_actor* act = nullptr;
  if ((rc = wah_actor(sys, value_bits, format, &act))) return rc;
  ka_ref* in = nullptr;
  if (flags & KA_WAH_INPUT_DEVICE) {
    rc = ka_ref_wrap(sys, const_cast<uint32_t*>(values), KA_U32, n, KA_ACCESS_READ, &in);
  } else {
    MsgVal v;
    v.mode = KA_VAL;
    v.dtype = KA_U32;
    v.host = values;
    v.count = n;
    Ref* r = nullptr;
    rc = msg_upload(sys, v, act->stream, &r);
    in = static_cast<ka_ref*>(r);
  }
  if (rc) return rc;
  ka_value msg{};
  msg.mode = KA_REF;
  msg.ref = in;
  ka_ticket* t = nullptr;
  rc = ka_send(act, &msg, 1, &t);
  ka_ref_release(in);
  if (rc) return rc;
  ka_value res[3] = {};
  rc = ka_receive(t, res, 3, -1);
  ka_ticket_release(t);
  if (rc) return rc;
  ka_wah_result r{};
  r.n = n;
  Ref* const outs[3] = {static_cast<Ref*>(res[0].ref), static_cast<Ref*>(res[1].ref), static_cast<Ref*>(res[2].ref)};
  uint64_t lens[3] = {0, 0, 0};
  rc = read_lengths3(sys, outs, lens);
  const uint64_t D = lens[0], O = lens[1], W = lens[2];
  if (!rc && O == 0 && n > 0) rc = set_error(KA_E_ARG, "a value is at or above 2^value_bits");
  if (!rc && O != D + 1) rc = set_error(KA_E_DEVICE, "inconsistent index lengths");
  if (!rc) {
    r.D = D;
    r.W = W;
    if (flags & KA_WAH_OUTPUT_REFS) {
      r.keys_ref = res[0].ref;
      r.offsets_ref = res[1].ref;
      r.words_ref = res[2].ref;
      *out = r;
      return KA_OK;
    }
    r.keys = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(D, 1) * 4));
    r.offsets = static_cast<uint32_t*>(std::malloc((D + 1) * 4));
    r.words = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(W, 1) * 4));
    if (!r.keys || !r.offsets || !r.words) rc = set_error(KA_E_OOM, "host allocation failed");
    if (!rc) {
      void* const dst[3] = {r.keys, r.offsets, r.words};
      const uint64_t bytes[3] = {D * 4, (D + 1) * 4, W * 4};
      rc = read_outputs3(sys, outs, dst, bytes);
    }
  }
  for (auto& v : res)
    if (v.ref) ka_ref_release(v.ref);
  if (rc) {
    std::free(r.keys);
    std::free(r.offsets);
    std::free(r.words);
    return rc;
  }
  *out = r;
  return KA_OK;
  KA_GUARD_END
}

// ---- batched index builds --------------------------------------------------------
KA_API int ka_wah_batch(ka_system* sys, const uint32_t* values, uint64_t n, const uint32_t* req_off, uint32_t nreq,
                        uint32_t value_bits, uint32_t flags, ka_wah_batch_result* out) {
  KA_GUARD_BEGIN
  if (!sys || !out || !req_off || (n && !values)) return set_error(KA_E_ARG, "null argument");
  if (nreq == 0) return set_error(KA_E_ARG, "no requests");
  if (n >= (1ull << 30)) return set_error(KA_E_ARG, "n must be below 2^30");
  if (value_bits == 0 || value_bits > 32) return set_error(KA_E_ARG, "value_bits must be 1..32");
  const uint32_t req_bits = nreq > 1 ? 32u - (uint32_t)__builtin_clz(nreq - 1) : 0u;
  if (value_bits + req_bits > 32) return set_error(KA_E_ARG, "value_bits + bits of nreq - 1 exceed 32");
  if (req_off[0] != 0 || req_off[nreq] != n) return set_error(KA_E_ARG, "req_off must run from 0 to n");
  for (uint32_t j = 0; j < nreq; ++j)
    if (req_off[j + 1] < req_off[j]) return set_error(KA_E_ARG, "req_off must be non-decreasing");
  int rc = sys->ensure_init();
  if (rc) return rc;
  {
    std::lock_guard<std::mutex> g(sys->wah_mu);
    if (!sys->builtin) {
      ka_program* p = nullptr;
      if ((rc = ka_program_builtin(sys, &p))) return rc;
      sys->builtin = p;  // released by ka_system_destroy
    }
  }
  ka_arg sig[8] = {};
  sig[0] = {KA_IN, KA_U32, KA_REF, KA_REF, 0, nullptr, nullptr, nullptr};
  sig[1] = {KA_IN, KA_U32, KA_VAL, KA_REF, 0, nullptr, nullptr, nullptr};
  // private values: value_bits, and the largest request plus one (a hint for
  // the small-request path; 0 = unknown)
  uint64_t biggest = 0;
  for (uint32_t j = 0; j < nreq; ++j) biggest = std::max<uint64_t>(biggest, (uint64_t)req_off[j + 1] - req_off[j]);
  const uint32_t priv_vals[2] = {value_bits, biggest < 0xFFFFFFFEull ? (uint32_t)biggest + 1u : 0u};
  sig[2] = {KA_PRIV, KA_U32, KA_VAL, KA_VAL, 2, nullptr, nullptr, priv_vals};
  for (int i = 3; i < 8; ++i) sig[i] = {KA_OUT, KA_U32, KA_REF, KA_REF, 0, nullptr, nullptr, nullptr};
  ka_nd_range r{};
  r.dims = 1;
  ka_actor* act = nullptr;
  if ((rc = ka_spawn(sys, static_cast<ka_program*>(sys->builtin), "wah_index_batch", &r, sig, 8, &act))) return rc;
  ka_ref* in = nullptr;
  if (flags & KA_WAH_INPUT_DEVICE) {
    rc = ka_ref_wrap(sys, const_cast<uint32_t*>(values), KA_U32, n, KA_ACCESS_READ, &in);
  } else {
    MsgVal v;
    v.mode = KA_VAL;
    v.dtype = KA_U32;
    v.host = values;
    v.count = n;
    Ref* rr = nullptr;
    rc = msg_upload(sys, v, act->stream, &rr);
    in = static_cast<ka_ref*>(rr);
  }
  if (rc) {
    ka_actor_release(act);
    return rc;
  }
  ka_value msg[2] = {};
  msg[0].mode = KA_REF;
  msg[0].ref = in;
  msg[1].mode = KA_VAL;
  msg[1].dtype = KA_U32;
  msg[1].ptr = const_cast<uint32_t*>(req_off);
  msg[1].count = (uint64_t)nreq + 1;
  ka_ticket* t = nullptr;
  rc = ka_send(act, msg, 2, &t);
  ka_ref_release(in);
  ka_actor_release(act);
  if (rc) return rc;
  ka_value res[5] = {};
  rc = ka_receive(t, res, 5, -1);
  ka_ticket_release(t);
  if (rc) return rc;
  uint64_t len[5] = {};
  for (int i = 0; i < 5 && !rc; ++i) rc = ref_length(res[i].ref, &len[i]);
  if (!rc && len[3] == 0) rc = set_error(KA_E_ARG, "a value is at or above 2^value_bits");
  if (!rc && (len[1] != len[0] + nreq || len[3] != nreq + 1ull || len[4] != nreq + 1ull))
    rc = set_error(KA_E_DEVICE, "inconsistent batch index lengths");
  ka_wah_batch_result br{};
  br.nreq = nreq;
  br.n = n;
  if (!rc) {
    br.D = len[0];
    br.W = len[2];
    if (flags & KA_WAH_OUTPUT_REFS) {
      br.keys_ref = res[0].ref;
      br.offsets_ref = res[1].ref;
      br.words_ref = res[2].ref;
      br.key_start_ref = res[3].ref;
      br.word_start_ref = res[4].ref;
      *out = br;
      return KA_OK;
    }
    uint32_t** dst[5] = {&br.keys, &br.offsets, &br.words, &br.key_start, &br.word_start};
    for (int i = 0; i < 5 && !rc; ++i) {
      *dst[i] = static_cast<uint32_t*>(std::malloc(std::max<uint64_t>(len[i], 1) * 4));
      if (!*dst[i])
        rc = set_error(KA_E_OOM, "host allocation failed");
      else
        rc = ka_ref_read(res[i].ref, *dst[i], len[i] * 4);
    }
  }
  for (auto& v : res)
    if (v.ref) ka_ref_release(v.ref);
  if (rc) {
    std::free(br.keys);
    std::free(br.offsets);
    std::free(br.words);
    std::free(br.key_start);
    std::free(br.word_start);
    return rc;
  }
  *out = br;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_wah_batch_result_free(ka_wah_batch_result* res) {
  if (!res) return set_error(KA_E_ARG, "null result");
  std::free(res->keys);
  std::free(res->offsets);
  std::free(res->words);
  std::free(res->key_start);
  std::free(res->word_start);
  ka_ref* refs[5] = {res->keys_ref, res->offsets_ref, res->words_ref, res->key_start_ref, res->word_start_ref};
  for (auto* r : refs)
    if (r) ka_ref_release(r);
  std::memset(res, 0, sizeof(*res));
  return KA_OK;
}

KA_API int ka_wah_result_free(ka_wah_result* res) {
  if (!res) return set_error(KA_E_ARG, "null result");
  std::free(res->keys);
  std::free(res->offsets);
  std::free(res->words);
  if (res->keys_ref) ka_ref_release(res->keys_ref);
  if (res->offsets_ref) ka_ref_release(res->offsets_ref);
  if (res->words_ref) ka_ref_release(res->words_ref);
  std::memset(res, 0, sizeof(*res));
  return KA_OK;
}

// ---- profiling ------------------------------------------------------------------------
static void prof_drain(ka_system* sys) {
  std::lock_guard<std::mutex> g(sys->prof_mu);
  sys->prof_fold_locked(true);
}

KA_API int ka_profile_get(ka_system* sys, const char* kernel, uint64_t* launches, double* total_ms) {
  KA_GUARD_BEGIN
  if (!sys || !kernel) return set_error(KA_E_ARG, "null argument");
  if (sys->inited && sys->init_rc == KA_OK) prof_drain(sys);
  std::lock_guard<std::mutex> g(sys->prof_mu);
  auto it = sys->prof_acc.find(kernel);
  if (launches) *launches = it == sys->prof_acc.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == sys->prof_acc.end() ? 0.0 : it->second.second;
  return KA_OK;
  KA_GUARD_END
}

KA_API int ka_affine_chain_raw(ka_system* sys, uint32_t* x, uint64_t n, const uint32_t* a, const uint32_t* b,
                               uint32_t stages) {
  KA_GUARD_BEGIN
  if (!sys || (n && !x) || (stages && (!a || !b))) return set_error(KA_E_ARG, "null argument");
  int rc = sys->ensure_init();
  if (rc) return rc;
  if ((rc = sys->use_device())) return rc;
  CmdEnv env(sys, 0);
  for (uint32_t i = 0; i < stages && !rc; ++i) rc = launch_affine(env, x, n, nullptr, 0, a[i], b[i]);
  return rc;
  KA_GUARD_END
}

KA_API int ka_profile_enable(ka_system* sys, int on) {
  if (!sys) return set_error(KA_E_ARG, "null system");
  sys->profile = on != 0;
  return KA_OK;
}

KA_API int ka_profile_reset(ka_system* sys) {
  KA_GUARD_BEGIN
  if (!sys) return set_error(KA_E_ARG, "null system");
  if (sys->inited && sys->init_rc == KA_OK) prof_drain(sys);
  std::lock_guard<std::mutex> g(sys->prof_mu);
  sys->prof_acc.clear();
  return KA_OK;
  KA_GUARD_END
}

}  // extern "C"
