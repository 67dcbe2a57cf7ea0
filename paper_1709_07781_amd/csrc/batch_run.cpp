// ka_batch_run: many independent requests to one actor as one batch (Sec. 3.6:
// data parallelism nested inside one kernel is an alternative level of
// composition to one actor invocation per request).
//
// The built-in actors with a batched form run every request of the call in one
// pass of their kernels, on the actor's stream:
//   wah_index (with a value-bits hint)  one batched index build (request-tagged
//                                        sort keys, request-relative rows);
//   exclusive_scan_u32                   one scan of the concatenation, rebased
//                                        at each request's first position;
//   affine_u32                           one launch over the concatenation.
// The requests' data are gathered into one device buffer (host values through
// pinned staging, device references copied on the device after their last
// writer), and request i's response is built from its slices of the batch's
// outputs: read-only views for REF outputs, host values read back once for VAL
// outputs.  Any other actor (and wah_index without a usable hint) gets the
// requests one after another through ka_send.  Either way tickets[i] answers
// request i exactly as ka_send would.
#include <cstring>

#include "runtime_internal.hpp"

namespace ka {
namespace {

struct Input {
  const uint32_t* host = nullptr;  // VAL
  Ref* ref = nullptr;              // REF (borrowed from the caller)
  uint64_t n = 0;
};

// A finished response: outputs are host values or views, ordered after the
// batch's work on stream si.
ka_ticket* make_ticket(System* sys, uint32_t si, Msg&& outs, int status) {
  ka_ticket* t = new ka_ticket();
  t->sys = sys;
  sys->retain();
  t->outs = std::move(outs);
  t->stream = si;
  t->status = status;
  t->done = sys->get_event();
  if (t->done) hipEventRecord(t->done, sys->streams[si]->s);
  return t;
}

// Copies every request's data to dst (device), request j at offset off[j].
int gather(System* sys, uint32_t si, const std::vector<Input>& in, const std::vector<uint64_t>& off,
           uint32_t* dst) {
  hipStream_t s = sys->streams[si]->s;
  uint64_t host_bytes = 0;
  for (const auto& x : in)
    if (!x.ref) host_bytes += 4 * x.n;
  char* st = nullptr;
  if (host_bytes) {
    st = static_cast<char*>(sys->stage.get(sys, host_bytes));
    if (!st) return set_error(KA_E_OOM, "pinned staging allocation failed");
  }
  uint64_t at = 0;
  hipError_t e = hipSuccess;
  for (size_t j = 0; j < in.size() && e == hipSuccess; ++j) {
    const Input& x = in[j];
    if (!x.n) continue;
    if (x.ref) {
      int rc = ref_use_on(x.ref, si, false);
      if (rc) return rc;
      e = hipMemcpyAsync(dst + off[j], x.ref->ptr, 4 * x.n, hipMemcpyDeviceToDevice, s);
    } else {
      std::memcpy(st + at, x.host, 4 * x.n);
      e = hipMemcpyAsync(dst + off[j], st + at, 4 * x.n, hipMemcpyHostToDevice, s);
      at += 4 * x.n;
    }
  }
  if (st) {
    hipEvent_t done = sys->get_event();
    if (e == hipSuccess && done && hipEventRecord(done, s) == hipSuccess) {
      sys->stage.retire(sys, st, done);
    } else {
      hipStreamSynchronize(s);
      if (done) sys->put_event(done);
      sys->stage.give_back(st);
    }
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "batch input copy");
  }
  return KA_OK;
}

// Host copy of count uint32 of a ref from element `from` (waits for the stream).
int read_u32(Ref* r, uint64_t from, uint64_t count, uint32_t* host) {
  if (!count) return KA_OK;
  int rc = ref_sync(r);
  if (rc) return rc;
  if (hipMemcpy(host, static_cast<uint32_t*>(r->ptr) + from, 4 * count, hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(KA_E_DEVICE, "batch result read-back");
  }
  return KA_OK;
}

// One output of request j: a view of parent[off, off + count) or, for a VAL
// output, the same elements of `host` (a read-back of parent, kept alive by
// the message).
int output(Ref* parent, uint32_t mode, uint64_t off, uint64_t count,
           const std::shared_ptr<std::vector<uint8_t>>& host, MsgVal* out) {
  MsgVal v;
  v.dtype = KA_U32;
  if (mode == KA_REF) {
    Ref* view = nullptr;
    int rc = ref_view(parent, off, count, &view);
    if (rc) return rc;
    v.mode = KA_REF;
    v.ref = view;
  } else {
    v.mode = KA_VAL;
    v.owned = host;
    v.host = host->data() + 4 * off;
    v.count = count;
  }
  *out = std::move(v);
  return KA_OK;
}

std::shared_ptr<std::vector<uint8_t>> read_all(Ref* r, uint64_t count, int* rc) {
  auto h = std::make_shared<std::vector<uint8_t>>(4 * std::max<uint64_t>(count, 1));
  *rc = read_u32(r, 0, count, reinterpret_cast<uint32_t*>(h->data()));
  return h;
}

struct Refs {  // refs made by the batch; released when the call returns (views keep theirs)
  std::vector<Ref*> v;
  ~Refs() {
    for (auto* r : v) ref_release(r);
  }
  int make(System* sys, uint64_t count, uint32_t si, Ref** out) {
    int rc = ref_create(sys, KA_U32, std::max<uint64_t>(count, 1), si, false, out);
    if (!rc) v.push_back(*out);
    return rc;
  }
};

// ---- wah_index -------------------------------------------------------------------
int run_wah(Actor* a, uint32_t value_bits, const std::vector<Input>& in, ka_ticket** tickets) {
  System* sys = a->sys;
  const uint32_t si = a->stream;
  const uint32_t nreq = (uint32_t)in.size();
  std::vector<uint64_t> off(nreq + 1, 0);
  uint32_t biggest = 0;
  for (uint32_t j = 0; j < nreq; ++j) {
    off[j + 1] = off[j] + in[j].n;
    biggest = std::max<uint32_t>(biggest, (uint32_t)in[j].n);
  }
  const uint64_t n = off[nreq];
  if (n >= (1ull << 30)) return set_error(KA_E_ARG, "a batch holds fewer than 2^30 values");
  Refs made;
  Ref *vals, *roff, *keys, *offs, *words, *ks, *ws, *lens, *bad;
  int rc;
  if ((rc = made.make(sys, n, si, &vals)) || (rc = made.make(sys, nreq + 1ull, si, &roff)) ||
      (rc = made.make(sys, n, si, &keys)) || (rc = made.make(sys, n + nreq, si, &offs)) ||
      (rc = made.make(sys, 2 * n, si, &words)) || (rc = made.make(sys, nreq + 1ull, si, &ks)) ||
      (rc = made.make(sys, nreq + 1ull, si, &ws)) || (rc = made.make(sys, 10, si, &lens)) ||
      (rc = made.make(sys, nreq, si, &bad)))
    return rc;
  {
    CmdEnv env(sys, si);
    if ((rc = gather(sys, si, in, off, static_cast<uint32_t*>(vals->ptr)))) return rc;
    std::vector<uint32_t> hoff(off.begin(), off.end());
    Input tab;
    tab.host = hoff.data();
    tab.n = nreq + 1ull;
    if ((rc = gather(sys, si, {tab}, {0}, static_cast<uint32_t*>(roff->ptr)))) return rc;
    uint64_t* l = static_cast<uint64_t*>(lens->ptr);
    rc = launch_wah_batch(env, static_cast<uint32_t*>(vals->ptr), n, static_cast<uint32_t*>(roff->ptr), nreq,
                          value_bits, static_cast<uint32_t*>(keys->ptr), static_cast<uint32_t*>(offs->ptr),
                          static_cast<uint32_t*>(words->ptr), static_cast<uint32_t*>(ks->ptr),
                          static_cast<uint32_t*>(ws->ptr), l, l + 1, l + 2, l + 3, l + 4, 0, biggest,
                          static_cast<uint32_t*>(bad->ptr));
    if (rc) return rc;
  }
  // The per-request tables decide every response's slices.
  std::vector<uint32_t> hks(nreq + 1), hws(nreq + 1), hbad(nreq);
  if ((rc = read_u32(ks, 0, nreq + 1ull, hks.data())) || (rc = read_u32(ws, 0, nreq + 1ull, hws.data())) ||
      (rc = read_u32(bad, 0, nreq, hbad.data())))
    return rc;
  const uint32_t D = hks[nreq], W = hws[nreq];
  uint32_t modes[3];
  bool any_val = false;
  for (int i = 0; i < 3; ++i) {
    modes[i] = a->sig[2 + i].a.out_mode;
    any_val |= modes[i] == KA_VAL;
  }
  std::shared_ptr<std::vector<uint8_t>> hk, ho, hw;
  if (any_val) {
    hk = read_all(keys, D, &rc);
    if (!rc) ho = read_all(offs, (uint64_t)D + nreq, &rc);
    if (!rc) hw = read_all(words, W, &rc);
    if (rc) return rc;
  }
  for (uint32_t j = 0; j < nreq; ++j) {
    Msg outs(3);
    int st = hbad[j] ? KA_E_ARG : KA_OK;
    if (!st) {
      const uint64_t k0 = hks[j], k1 = hks[j + 1], w0 = hws[j], w1 = hws[j + 1];
      if ((rc = output(keys, modes[0], k0, k1 - k0, hk, &outs[0])) ||
          (rc = output(offs, modes[1], k0 + j, k1 - k0 + 1, ho, &outs[1])) ||
          (rc = output(words, modes[2], w0, w1 - w0, hw, &outs[2]))) {
        msg_clear(outs);
        return rc;
      }
    }
    tickets[j] = make_ticket(sys, si, std::move(outs), st);
  }
  return KA_OK;
}

// ---- exclusive_scan_u32 and affine_u32 ---------------------------------------------
// The scan's response is y; the affine stage's is x itself (in_out): a request
// that sent a reference gets it back updated in place, as from ka_send.
int run_elementwise(Actor* a, bool scan, const std::vector<Input>& in, ka_ticket** tickets) {
  System* sys = a->sys;
  const uint32_t si = a->stream;
  const uint32_t nreq = (uint32_t)in.size();
  std::vector<uint64_t> off(nreq + 1, 0);
  for (uint32_t j = 0; j < nreq; ++j) off[j + 1] = off[j] + in[j].n;
  const uint64_t n = off[nreq];
  if (n >= (1ull << 32)) return set_error(KA_E_ARG, "a batch holds fewer than 2^32 values");
  Refs made;
  Ref *x = nullptr, *y = nullptr, *roff = nullptr;
  int rc = made.make(sys, n, si, &x);
  if (!rc && scan) rc = made.make(sys, n, si, &y);
  if (!rc && scan) rc = made.make(sys, nreq + 1ull, si, &roff);
  if (rc) return rc;
  const uint32_t out_arg = scan ? 1 : 0;
  const uint32_t mode = a->sig[out_arg].a.out_mode;
  {
    CmdEnv env(sys, si);
    if ((rc = gather(sys, si, in, off, static_cast<uint32_t*>(x->ptr)))) return rc;
    if (scan) {
      std::vector<uint32_t> hoff(off.begin(), off.end());
      Input tab;
      tab.host = hoff.data();
      tab.n = nreq + 1ull;
      if ((rc = gather(sys, si, {tab}, {0}, static_cast<uint32_t*>(roff->ptr)))) return rc;
      rc = launch_segmented_scan(env, static_cast<uint32_t*>(x->ptr), static_cast<uint32_t*>(y->ptr), n,
                                 static_cast<uint32_t*>(roff->ptr), nreq);
    } else {
      uint32_t pa = 0, pb = 0;
      std::memcpy(&pa, a->sig[1].init.data(), 4);
      std::memcpy(&pb, a->sig[2].init.data(), 4);
      rc = launch_affine(env, static_cast<uint32_t*>(x->ptr), n, nullptr, 0, pa, pb);
      // in_out: a caller's reference is updated in place
      hipStream_t s = sys->streams[si]->s;
      for (uint32_t j = 0; !rc && j < nreq; ++j) {
        if (!in[j].ref || !in[j].n) continue;
        if ((rc = ref_use_on(in[j].ref, si, true))) break;
        in[j].ref->home = si;
        if (hipMemcpyAsync(in[j].ref->ptr, static_cast<uint32_t*>(x->ptr) + off[j], 4 * in[j].n,
                           hipMemcpyDeviceToDevice, s) != hipSuccess) {
          (void)hipGetLastError();
          rc = set_error(KA_E_DEVICE, "batch result copy");
        }
      }
    }
    if (rc) return rc;
  }
  Ref* res = scan ? y : x;
  std::shared_ptr<std::vector<uint8_t>> host;
  if (mode == KA_VAL) {
    host = read_all(res, n, &rc);
    if (rc) return rc;
  }
  for (uint32_t j = 0; j < nreq; ++j) {
    Msg outs(1);
    if (!scan && in[j].ref && mode == KA_REF) {  // the caller's own reference, updated
      ref_retain(in[j].ref);
      outs[0].mode = KA_REF;
      outs[0].dtype = KA_U32;
      outs[0].ref = in[j].ref;
    } else if ((rc = output(res, mode, off[j], in[j].n, host, &outs[0]))) {
      msg_clear(outs);
      return rc;
    }
    tickets[j] = make_ticket(sys, si, std::move(outs), KA_OK);
  }
  return KA_OK;
}

// The request's data: one uint32 element, a host value or a reference, in the
// mode the actor's first argument accepts (as ka_send matches it).
int one_input(const ka_request& r, uint32_t in_mode, Input* out) {
  if (r.nargs != 1 || !r.args) return set_error(KA_E_ARITY, "a batched request is one message element");
  const ka_value& v = r.args[0];
  if (v.mode != in_mode) return set_error(KA_E_TYPE, "message element does not match the signature's mode");
  Input x;
  if (v.mode == KA_VAL) {
    if (v.dtype != KA_U32) return set_error(KA_E_TYPE, "batched requests take uint32 data");
    if (v.count && !v.ptr) return set_error(KA_E_ARG, "VAL value without data");
    x.host = static_cast<const uint32_t*>(v.ptr);
    x.n = v.count;
  } else if (v.mode == KA_REF) {
    if (!v.ref) return set_error(KA_E_ARG, "REF value without a reference");
    if (v.ref->dtype != KA_U32) return set_error(KA_E_TYPE, "batched requests take uint32 data");
    x.ref = v.ref;
    int rc = ref_length(v.ref, &x.n);
    if (rc) return rc;
  } else {
    return set_error(KA_E_ARG, "unknown value mode");
  }
  *out = x;
  return KA_OK;
}

}  // namespace
}  // namespace ka

using namespace ka;

#define KA_GUARD_BEGIN try {
#define KA_GUARD_END                                      \
  }                                                       \
  catch (const std::bad_alloc&) {                         \
    return set_error(KA_E_OOM, "host allocation failed"); \
  }                                                       \
  catch (...) {                                           \
    return set_error(KA_E_DEVICE, "internal error");      \
  }

KA_API int ka_batch_run(ka_actor* actor, const ka_request* reqs, uint32_t nreq, ka_ticket** tickets) {
  KA_GUARD_BEGIN
  if (!actor || !tickets || (nreq && !reqs)) return set_error(KA_E_ARG, "null argument");
  System* sys = actor->sys;
  if (sys->destroyed.load()) return set_error(KA_E_STATE, "system was destroyed");
  if (nreq == 0) return KA_OK;
  int rc = sys->ensure_init();
  if (rc) return rc;
  if ((rc = sys->use_device())) return rc;
  const BuiltinKernel* bk = actor->composed ? nullptr : actor->bk;
  const bool mapped = actor->pre || actor->post;
  const std::string name = bk ? bk->name : "";
  bool batched = false;
  uint32_t value_bits = 0;
  if (bk && !mapped) {
    if (name == "wah_index") {
      uint32_t format = 0;  // the batched build writes the paper's form only
      if (actor->sig[1].init.size() >= 4) std::memcpy(&value_bits, actor->sig[1].init.data(), 4);
      if (actor->sig[1].init.size() >= 8) std::memcpy(&format, actor->sig[1].init.data() + 4, 4);
      const uint32_t req_bits = nreq > 1 ? 32u - (uint32_t)__builtin_clz(nreq - 1) : 0u;
      batched = format == 0 && value_bits >= 1 && value_bits + req_bits <= 32;
    } else if (name == "exclusive_scan_u32") {
      batched = true;
    } else if (name == "affine_u32") {
      batched = actor->sig[1].init.size() >= 4 && actor->sig[2].init.size() >= 4;
    }
  }
  if (batched) {
    std::vector<Input> in(nreq);
    for (uint32_t j = 0; j < nreq; ++j)
      if ((rc = one_input(reqs[j], actor->sig[0].a.in_mode, &in[j]))) return rc;
    std::vector<ka_ticket*> t(nreq, nullptr);
    std::lock_guard<std::mutex> g(actor->mu);  // one message at a time, in order of arrival
    if (name == "wah_index")
      rc = run_wah(actor, value_bits, in, t.data());
    else
      rc = run_elementwise(actor, name == "exclusive_scan_u32", in, t.data());
    if (rc) {
      for (auto* x : t)
        if (x) ka_ticket_release(x);
      return rc;
    }
    for (uint32_t j = 0; j < nreq; ++j) tickets[j] = t[j];
    return KA_OK;
  }
  // no batched form: the requests one after another
  std::vector<ka_ticket*> t(nreq, nullptr);
  for (uint32_t j = 0; j < nreq; ++j) {
    if ((rc = ka_send(actor, reqs[j].args, reqs[j].nargs, &t[j]))) {
      for (uint32_t i = 0; i < j; ++i) ka_ticket_release(t[i]);
      return rc;
    }
  }
  for (uint32_t j = 0; j < nreq; ++j) tickets[j] = t[j];
  return KA_OK;
  KA_GUARD_END
}
