// Host runtime internals: system, device memory pool, references, programs,
// actors and tickets.  Everything here sits behind the C ABI of ka.h.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ka.h"
#include "common.hpp"

namespace ka {

int set_error(int code, const std::string& msg);
uint32_t dtype_size(uint32_t dtype);

struct System;

// ---- device memory pool --------------------------------------------------------
// Caching allocator with stream-ordered reuse: a block freed after use on one
// stream only goes back to that stream's free list, so work queued later on
// that stream runs after every kernel that used the block.  Blocks also used
// on other streams wait for events recorded on those streams.
class Pool {
 public:
  void init(System* sys, uint64_t budget);
  // bytes are rounded up to a size class; *got receives the size of the block
  // handed out (the class, or a cached block of up to twice it).
  int alloc(uint64_t bytes, uint32_t stream, void** out, uint64_t* got);
  void release(void* p, uint64_t bytes, uint32_t home, uint64_t used_mask);
  void destroy();
  uint64_t in_use() const { return in_use_; }
  uint64_t reserved() const { return reserved_; }
  uint64_t budget() const { return budget_; }
  static uint64_t size_class(uint64_t bytes);

 private:
  struct Deferred {
    void* p;
    uint64_t bytes;
    uint32_t home;
    std::vector<hipEvent_t> events;
  };
  void poll_deferred_locked();
  int trim_locked();
  System* sys_ = nullptr;
  std::mutex mu_;
  std::vector<std::multimap<uint64_t, void*>> free_;
  std::vector<Deferred> deferred_;
  std::unordered_map<void*, uint64_t> all_;  // every block obtained from hipMalloc
  uint64_t in_use_ = 0, reserved_ = 0, budget_ = 0;
};

// ---- pinned host staging for value inputs -------------------------------------
class HostStage {
 public:
  void* get(System* sys, uint64_t bytes);                  // pinned buffer of >= bytes
  void retire(System* sys, void* p, hipEvent_t done);      // reusable once `done` completed
  void give_back(void* p);                                 // reusable at once
  void destroy(System* sys);

 private:
  struct Entry {
    void* p;
    uint64_t bytes;
    hipEvent_t done;
  };
  std::mutex mu_;
  std::vector<Entry> busy_;
  std::multimap<uint64_t, void*> free_;
  std::unordered_map<void*, uint64_t> sizes_;
};

struct StreamCtx {
  hipStream_t s = nullptr;
  bool owned = false;
  LookbackArena arena;
  std::mutex mu;  // serialises look-back bookkeeping of this stream
};

struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};

struct Actor;
struct Program;

struct System {
  ka_system_config cfg{};
  std::atomic<int> rc{1};
  std::atomic<bool> destroyed{false};
  std::mutex init_mu;
  bool inited = false;
  int init_rc = 0;
  std::string init_err;
  std::vector<std::unique_ptr<StreamCtx>> streams;
  Pool pool;
  HostStage stage;
  std::atomic<bool> profile{false};
  std::atomic<uint64_t> length_reads{0};  // device-resident lengths read back on the host (each waits)
  uint32_t lb_spin = kLbSpinLimit;  // look-back spin limit (KA_LOOKBACK_SPIN)
  std::mutex ev_mu;
  std::vector<hipEvent_t> events;         // pool of timing-disabled events
  std::vector<hipEvent_t> timing_events;  // pool of timing events (profiling)
  std::mutex prof_mu;
  std::vector<ProfRec> prof_pending;
  std::map<std::string, std::pair<uint64_t, double>> prof_acc;
  // built-in program and the index actors used by ka_wah_index (one per
  // value-bits hint, 0 = none)
  std::mutex wah_mu;
  Program* builtin = nullptr;
  Actor* wah_actor[33][3] = {};  // [value bits][format]

  int ensure_init();   // lazily initialises HIP on first use
  int use_device();    // makes the system's device current for this thread
  hipEvent_t get_event(bool timing = false);
  void put_event(hipEvent_t e);
  void put_timing_event(hipEvent_t e);
  // Folds finished profile records into the totals: all of them, waiting for
  // each (all = true), or the finished ones at the front (caller holds prof_mu).
  void prof_fold_locked(bool all);
  void retain() { rc.fetch_add(1); }
  void release();
};

// ---- launch environment of one command ------------------------------------------
// Holds the stream's lock for the whole command, so the stream's look-back
// arena serves one launch at a time, in stream order; scratch memory returns
// to the pool in stream order when the command ends.
class CmdEnv final : public Env {
 public:
  // The stream's lock is held for the whole command, so the stream's
  // look-back arena (status words, epochs, sort plan) serves one launch
  // at a time, in stream order.
  CmdEnv(System* sys, uint32_t si) : sys_(sys), si_(si), lock_(sys->streams[si]->mu) {}
  ~CmdEnv() override {
    for (auto& s : scratch_) sys_->pool.release(s.first, s.second, si_, 1ull << si_);
  }
  hipStream_t stream() override { return sys_->streams[si_]->s; }
  void* scratch(uint64_t bytes) override {
    void* p = nullptr;
    uint64_t got = 0;
    if (sys_->pool.alloc(bytes, si_, &p, &got) != KA_OK) return nullptr;
    scratch_.emplace_back(p, got);
    return p;
  }
  bool lookback(uint64_t words, LbArgs* out) override {
    LookbackArena& ar = sys_->streams[si_]->arena;
    if (words > ar.status_words) {
      uint64_t nw = std::max<uint64_t>(words, 2 * ar.status_words);
      nw = std::max<uint64_t>(nw, 1 << 16);
      void* p = nullptr;
      uint64_t got = 0;
      if (sys_->pool.alloc(nw * 8, si_, &p, &got) != KA_OK) return false;
      if (ar.status) sys_->pool.release(ar.status, ar.status_bytes, si_, 1ull << si_);
      ar.status = static_cast<uint64_t*>(p);
      ar.status_words = got / 8;
      ar.status_bytes = got;
      if (launch_fill_u64(*this, ar.status, ar.status_words, 0) != KA_OK) return false;
    }
    if (ar.epoch + 1 >= (1u << 30)) {
      if (launch_fill_u64(*this, ar.status, ar.status_words, 0) != KA_OK) return false;
      ar.epoch = 0;
    }
    ar.epoch += 1;
    out->status = ar.status;
    out->epoch = ar.epoch;
    out->spin_limit = sys_->lb_spin;
    return true;
  }
  LookbackArena* arena() override { return &sys_->streams[si_]->arena; }
  uint32_t spin_limit() override { return sys_->lb_spin; }
  void prof_begin(const char* kernel) override {
    if (!sys_->profile) return;
    (void)kernel;
    ev0_ = sys_->get_event(true);
    if (ev0_) hipEventRecord(ev0_, stream());
  }
  void prof_end(const char* kernel) override {
    if (!sys_->profile || !ev0_) return;
    hipEvent_t ev1 = sys_->get_event(true);
    if (!ev1) return;
    hipEventRecord(ev1, stream());
    std::lock_guard<std::mutex> g(sys_->prof_mu);
    sys_->prof_pending.push_back({kernel, ev0_, ev1});
    ev0_ = nullptr;
    // keep the live timing events bounded: fold the finished front records
    if (sys_->prof_pending.size() >= 4096) sys_->prof_fold_locked(false);
  }
  int fail(int code, const char* msg) override { return set_error(code, msg); }
  uint32_t si() const { return si_; }

 private:
  System* sys_;
  uint32_t si_;
  std::lock_guard<std::mutex> lock_;
  std::vector<std::pair<void*, uint64_t>> scratch_;
  hipEvent_t ev0_ = nullptr;
};

// ---- references (mem_ref) ----------------------------------------------------
struct Ref {
  std::atomic<int> rc{1};
  System* sys = nullptr;
  uint32_t dtype = KA_U32;
  uint32_t access = KA_ACCESS_RW;
  void* ptr = nullptr;
  uint64_t cap = 0;          // elements
  uint64_t alloc_bytes = 0;  // pool block size (0: borrowed)
  bool borrowed = false;
  uint64_t* d_len = nullptr;  // device-resident length (data-dependent outputs)
  std::atomic<bool> len_known{true};
  uint64_t len = 0;
  uint32_t home = 0;  // stream of the last writer
  std::atomic<uint64_t> used_mask{0};
  Ref* parent = nullptr;  // a view: elements of the parent's buffer (+1 held on the parent)
};

// Allocates a pool-backed ref of `count` elements on stream `si`.  With
// `device_len` the length lives in a device slot behind the data.
int ref_create(System* sys, uint32_t dtype, uint64_t count, uint32_t si, bool device_len, Ref** out);
void ref_retain(Ref* r);
void ref_release(Ref* r);
// Waits until the streams that touched the ref are idle.
int ref_sync(Ref* r);
// The true length (reads the device slot if needed; waits).
int ref_length(Ref* r, uint64_t* len);
// Orders stream si after the last writer of r (and, for a write, after every
// stream that used r) and records the use.
int ref_use_on(Ref* r, uint32_t si, bool write);
// A read-only view of count elements of parent from element `offset` on; it
// keeps the parent alive, and its uses are recorded on the parent too.
int ref_view(Ref* parent, uint64_t offset, uint64_t count, Ref** out);

// ---- programs and built-in kernels -------------------------------------------
struct Bound {  // one signature argument bound for a launch
  void* ptr = nullptr;
  uint64_t cap = 0;
  uint64_t len = 0;               // host-known length (inputs), valid when d_len == nullptr
  const uint64_t* d_len = nullptr;  // device length of an input, or slot of an output
  Ref* ref = nullptr;
  uint64_t priv[4] = {0, 0, 0, 0};
  uint32_t lds_offset = 0;
};

struct LaunchCtx {
  Env* env;
  uint64_t n;               // work-items (host-known upper bound)
  const uint64_t* d_n;      // device-resident work-item count, or null
  const ka_nd_range* range;
  std::vector<Bound>* args;
};

struct BuiltinKernel {
  const char* name;
  std::vector<std::pair<uint32_t, uint32_t>> sig;  // (dir, dtype)
  // default capacity of the out/in_out argument at signature index i, given
  // the work-item count and the bound arguments (inputs are bound by then)
  uint64_t (*default_cap)(uint32_t i, uint64_t n, const std::vector<Bound>& args);
  bool (*device_len)(uint32_t i);  // output length written by the kernel
  bool needs_host_n;               // work-item count must be known on the host
  int (*launch)(LaunchCtx& c);
};

const BuiltinKernel* find_builtin(const char* name);
const std::vector<BuiltinKernel>& builtin_kernels();

struct Program {
  std::atomic<int> rc{1};
  System* sys = nullptr;
  bool builtin = true;
  hipModule_t module = nullptr;
  std::string path;
};

// ---- actors --------------------------------------------------------------------
struct SigArg {
  ka_arg a;
  std::vector<uint8_t> init;  // PRIV values
};

struct Actor {
  std::atomic<int> rc{1};
  System* sys = nullptr;
  bool composed = false;
  // kernel actor
  Program* prog = nullptr;
  const BuiltinKernel* bk = nullptr;
  hipFunction_t fn = nullptr;
  std::string kernel;
  ka_nd_range range{};
  std::vector<SigArg> sig;
  // composed actor: stages, innermost first
  std::vector<Actor*> stages;
  ka_map_fn pre = nullptr, post = nullptr;
  void* map_ud = nullptr;
  uint32_t stream = 0;
  std::mutex mu;  // one message at a time, in order of arrival
};

// One element of a message in flight.
struct MsgVal {
  uint32_t mode = KA_VAL;
  uint32_t dtype = KA_U32;
  const void* host = nullptr;  // VAL on the host
  uint64_t count = 0;
  std::shared_ptr<std::vector<uint8_t>> owned;
  Ref* ref = nullptr;  // REF, or a VAL result still on the device (+1 held)
};
using Msg = std::vector<MsgVal>;
void msg_clear(Msg& m);

struct Ticket;

// Completion of a ticket that the host finishes (a served request): wait()
// blocks until the request is done (or timeout_us passes; < 0: no limit),
// then fills the ticket's outputs; a failed request sets t->status.
struct HostCompletion {
  virtual ~HostCompletion() = default;
  virtual int wait(Ticket* t, int64_t timeout_us) = 0;
};

struct Ticket {
  std::atomic<int> rc{1};
  System* sys = nullptr;
  int status = KA_OK;
  Msg outs;
  hipEvent_t done = nullptr;
  uint32_t stream = 0;
  std::atomic<bool> complete{false};
  HostCompletion* hc = nullptr;  // owned; null for device-ordered tickets
};

// Runs a message through an actor (all stages), queueing the device work.
int actor_run(Actor* a, Msg& in, Msg& out, uint32_t si);
// Copies a C message into a Msg (REF values retained).
int msg_from_values(const ka_value* vals, uint32_t n, Msg& out);
// Uploads a host value into a new ref on stream si (pinned staging).
int msg_upload(System* sys, const MsgVal& v, uint32_t si, Ref** out);

}  // namespace ka

// The opaque C handles are the runtime structs.
struct ka_system : ka::System {};
struct ka_program : ka::Program {};
struct ka_actor : ka::Actor {};
struct ka_ref : ka::Ref {};
struct ka_ticket : ka::Ticket {};
