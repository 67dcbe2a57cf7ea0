// The built-in program: kernel names, their signatures and the adapters that
// turn bound arguments into launches (Sec. 3.2: a program maps kernel names
// to kernels).
#include "runtime_internal.hpp"

namespace ka {
namespace {

uint64_t cap_same(uint32_t, uint64_t n, const std::vector<Bound>&) { return n; }
uint64_t cap_wah(uint32_t i, uint64_t n, const std::vector<Bound>&) {
  // (in skeys, in srows, out keys[D <= n], out offsets[D+1], out words[W <= 2n])
  if (i == 2) return n ? n : 1;
  if (i == 3) return n + 1;
  return n ? 2 * n : 1;
}
// (in values; in req_off[nreq+1]; priv value_bits; out keys[D <= n];
//  out offsets[D + nreq]; out words[W <= 2n]; out key_start[nreq+1]; out word_start[nreq+1])
uint64_t cap_batch(uint32_t i, uint64_t n, const std::vector<Bound>& args) {
  const uint64_t slots = args[1].len;  // nreq + 1
  const uint64_t nreq = slots ? slots - 1 : 0;
  switch (i) {
    case 3: return n ? n : 1;
    case 4: return std::max<uint64_t>(n + nreq, 1);
    case 5: return n ? 2 * n : 1;
    default: return std::max<uint64_t>(slots, 1);
  }
}
// (in values; priv value_bits; out keys[D <= n]; out offsets[D+1]; out words[W <= 2n])
uint64_t cap_wah_index(uint32_t i, uint64_t n, const std::vector<Bound>&) {
  if (i == 2) return n ? n : 1;
  if (i == 3) return n + 1;
  return n ? 2 * n : 1;
}
// wah_decode: (in words; priv format, ngroups; out groups[ngroups])
uint64_t cap_decode(uint32_t, uint64_t, const std::vector<Bound>& args) {
  return std::max<uint64_t>(args[1].priv[1], 1);
}
// wah_combine: (in a; in b; priv op, in_format, out_format, ngroups; out words[<= 2 ngroups])
uint64_t cap_combine(uint32_t, uint64_t, const std::vector<Bound>& args) { return 2 * args[2].priv[3] + 1; }
bool len_decode(uint32_t i) { return i == 2; }
bool len_combine(uint32_t i) { return i == 3; }
bool len_host(uint32_t) { return false; }
bool len_batch(uint32_t i) { return i >= 3; }
bool len_compact(uint32_t i) { return i == 1; }
bool len_wah(uint32_t i) { return i >= 2; }

// affine_u32: (in_out x; priv a; priv b)
int run_affine(LaunchCtx& c) {
  Bound& x = (*c.args)[0];
  const uint64_t off = c.range ? c.range->offset[0] : 0;
  if (off > x.cap || c.n > x.cap - off) return c.env->fail(KA_E_ARG, "affine_u32: range exceeds the buffer");
  return launch_affine(*c.env, static_cast<uint32_t*>(x.ptr), c.n, c.d_n, off, (uint32_t)(*c.args)[1].priv[0],
                       (uint32_t)(*c.args)[2].priv[0]);
}

// exclusive_scan_u32: (in x; out y)
int run_scan(LaunchCtx& c) {
  Bound& in = (*c.args)[0];
  Bound& out = (*c.args)[1];
  if (c.n > in.cap || c.n > out.cap) return c.env->fail(KA_E_ARG, "exclusive_scan_u32: range exceeds a buffer");
  int rc = launch_exclusive_scan(*c.env, static_cast<const uint32_t*>(in.ptr), static_cast<uint32_t*>(out.ptr), c.n,
                                 c.d_n);
  return rc;
}

// compact_nonzero_u32: (in x; out y) -- y's length is written on the device
int run_compact(LaunchCtx& c) {
  Bound& in = (*c.args)[0];
  Bound& out = (*c.args)[1];
  if (c.n > in.cap || c.n > out.cap) return c.env->fail(KA_E_ARG, "compact_nonzero_u32: range exceeds a buffer");
  return launch_compact_nonzero(*c.env, static_cast<const uint32_t*>(in.ptr), static_cast<uint32_t*>(out.ptr), c.n,
                                c.d_n, const_cast<uint64_t*>(out.d_len));
}

// radix_sort_rows_u32: (in keys; out skeys; out srows)
int run_sort_rows(LaunchCtx& c) {
  Bound& k = (*c.args)[0];
  Bound& sk = (*c.args)[1];
  Bound& sr = (*c.args)[2];
  if (c.n > k.cap || c.n > sk.cap || c.n > sr.cap)
    return c.env->fail(KA_E_ARG, "radix_sort_rows_u32: range exceeds a buffer");
  return launch_radix_sort_pairs(*c.env, static_cast<const uint32_t*>(k.ptr), nullptr, static_cast<uint32_t*>(sk.ptr),
                                 static_cast<uint32_t*>(sr.ptr), c.n, 0, c.d_n);
}

// radix_sort_pairs_u32: (in keys; in rows; out skeys; out srows)
int run_sort_pairs(LaunchCtx& c) {
  Bound& k = (*c.args)[0];
  Bound& r = (*c.args)[1];
  Bound& sk = (*c.args)[2];
  Bound& sr = (*c.args)[3];
  if (c.n > k.cap || c.n > r.cap || c.n > sk.cap || c.n > sr.cap)
    return c.env->fail(KA_E_ARG, "radix_sort_pairs_u32: range exceeds a buffer");
  return launch_radix_sort_pairs(*c.env, static_cast<const uint32_t*>(k.ptr), static_cast<const uint32_t*>(r.ptr),
                                 static_cast<uint32_t*>(sk.ptr), static_cast<uint32_t*>(sr.ptr), c.n, 0, c.d_n);
}

// wah_encode_sorted: (in skeys; in srows; out keys; out offsets; out words)
int run_wah(LaunchCtx& c) {
  auto& a = *c.args;
  if (c.n > a[0].cap || c.n > a[1].cap) return c.env->fail(KA_E_ARG, "wah_encode_sorted: range exceeds an input");
  if (a[2].cap < c.n || a[3].cap < c.n + 1 || a[4].cap < 2 * c.n)
    return c.env->fail(KA_E_ARG, "wah_encode_sorted: outputs need capacities n, n+1 and 2n");
  return launch_wah_encode(*c.env, static_cast<const uint32_t*>(a[0].ptr), static_cast<const uint32_t*>(a[1].ptr), c.n,
                           static_cast<uint32_t*>(a[2].ptr), static_cast<uint32_t*>(a[3].ptr),
                           static_cast<uint32_t*>(a[4].ptr), const_cast<uint64_t*>(a[2].d_len),
                           const_cast<uint64_t*>(a[3].d_len), const_cast<uint64_t*>(a[4].d_len), nullptr, 32, nullptr, 32,
                           c.d_n);
}

// wah_index: (in values; priv value_bits [, format]; out keys; out offsets;
// out words) -- parts 1-6 of Sec. 4.1 in one actor: the stable sort of
// (value, row) pairs, then the encoder.  value_bits 1..16: every value is below
// 2^value_bits, the sort runs ceil(value_bits / 8) passes over uint16 sort
// keys; 17..31: values below 2^value_bits, the sort of uint32 keys; 0 or 32:
// any uint32 value.  A value at or above 2^value_bits voids the result (every
// output length 0).  format: 0 the paper's form (one literal per non-empty
// group), 1 canonical WAH (runs of full groups as 1-fills), 2 PLWAH.
int run_wah_index(LaunchCtx& c) {
  auto& a = *c.args;
  Env& env = *c.env;
  const uint64_t n = c.n;
  const uint32_t bits = (uint32_t)a[1].priv[0];
  if (bits > 32) return env.fail(KA_E_ARG, "wah_index: value_bits must be 0..32");
  if (n > a[0].cap) return env.fail(KA_E_ARG, "wah_index: range exceeds the values");
  if (a[2].cap < n || a[3].cap < n + 1 || a[4].cap < 2 * n)
    return env.fail(KA_E_ARG, "wah_index: outputs need capacities n, n+1 and 2n");
  if (n >= (1ull << 30)) return env.fail(KA_E_ARG, "wah_index: n must be below 2^30");
  const uint32_t* values = static_cast<const uint32_t*>(a[0].ptr);
  uint32_t* keys = static_cast<uint32_t*>(a[2].ptr);
  uint32_t* offsets = static_cast<uint32_t*>(a[3].ptr);
  uint32_t* words = static_cast<uint32_t*>(a[4].ptr);
  uint64_t* lk = const_cast<uint64_t*>(a[2].d_len);
  uint64_t* lo = const_cast<uint64_t*>(a[3].d_len);
  uint64_t* lw = const_cast<uint64_t*>(a[4].d_len);
  const uint32_t fmt = (uint32_t)a[1].priv[1];
  const uint64_t* d_n = c.d_n;  // the count on the device (n is then the capacity)
  if (fmt > 2) return env.fail(KA_E_ARG, "wah_index: format must be 0 (paper), 1 (canonical) or 2 (PLWAH)");
  if (fmt == 2 && n > 31ull * 0x1FFFFFFull)
    return env.fail(KA_E_ARG, "wah_index: PLWAH fill lengths (25 bits) cover at most 31 * (2^25 - 1) rows");
  if (n == 0) return launch_wah_encode(env, nullptr, nullptr, 0, keys, offsets, words, lk, lo, lw);
  int rc;
  if (fmt != 0) {  // canonical WAH or PLWAH: the sorted pairs' group list, then the format's encoder
    uint32_t* reject = static_cast<uint32_t*>(env.scratch(4));
    if (!reject) return env.fail(KA_E_OOM, "wah_index: scratch");
    if (bits >= 1 && bits <= 16) {
      uint16_t* sk = static_cast<uint16_t*>(env.scratch(2 * n));
      uint32_t* sr = static_cast<uint32_t*>(env.scratch(4 * n));
      if (!sk || !sr) return env.fail(KA_E_OOM, "wah_index: scratch");
      if ((rc = launch_radix_sort_rows16(env, values, sk, sr, n, bits, reject, 0, d_n))) return rc;
      return launch_wah_encode_format16(env, sk, sr, n, fmt, keys, offsets, words, lk, lo, lw, reject, d_n);
    }
    uint32_t* sk = static_cast<uint32_t*>(env.scratch(4 * n));
    uint32_t* sr = static_cast<uint32_t*>(env.scratch(4 * n));
    if (!sk || !sr) return env.fail(KA_E_OOM, "wah_index: scratch");
    if ((rc = launch_zero_u32(env, reject))) return rc;
    if ((rc = launch_radix_sort_pairs(env, values, nullptr, sk, sr, n, 0, d_n))) return rc;
    if (bits >= 17 && bits <= 31 && (rc = launch_reject_above(env, sort_plan_keys_or(env), bits, reject))) return rc;
    return launch_wah_encode_format(env, sk, sr, n, fmt, keys, offsets, words, lk, lo, lw, reject, d_n);
  }
  if (bits >= 1 && bits <= 16) {
    uint32_t* reject = static_cast<uint32_t*>(env.scratch(4));
    uint16_t* sk = static_cast<uint16_t*>(env.scratch(2 * n));
    uint32_t* sr = static_cast<uint32_t*>(env.scratch(4 * n));
    if (!reject || !sk || !sr) return env.fail(KA_E_OOM, "wah_index: scratch");
    if ((rc = launch_radix_sort_rows16(env, values, sk, sr, n, bits, reject, 0, d_n))) return rc;
    return launch_wah_encode16(env, sk, sr, n, keys, offsets, words, lk, lo, lw, reject, 0, d_n);
  }
  uint32_t* sk = static_cast<uint32_t*>(env.scratch(4 * n));
  uint32_t* sr = static_cast<uint32_t*>(env.scratch(4 * n));
  if (!sk || !sr) return env.fail(KA_E_OOM, "wah_index: scratch");
  if ((rc = launch_radix_sort_pairs(env, values, nullptr, sk, sr, n, 0, d_n))) return rc;
  const bool check = bits >= 17 && bits <= 31;
  return launch_wah_encode(env, sk, sr, n, keys, offsets, words, lk, lo, lw, nullptr, 32,
                           check ? sort_plan_keys_or(env) : nullptr, check ? bits : 32u, d_n);
}

// wah_lookup: (in queries; in keys; out slots) -- slots[i] = the index d of
// queries[i] in the lookup table keys (ascending), or 0xFFFFFFFF (Sec. 4.1
// part 6 read back).
int run_lookup(LaunchCtx& c) {
  auto& a = *c.args;
  if (c.n > a[0].cap || c.n > a[2].cap) return c.env->fail(KA_E_ARG, "wah_lookup: range exceeds a buffer");
  return launch_wah_lookup(*c.env, static_cast<const uint32_t*>(a[1].ptr), a[1].d_len ? a[1].cap : a[1].len,
                           a[1].d_len, static_cast<const uint32_t*>(a[0].ptr), c.n, static_cast<uint32_t*>(a[2].ptr),
                           c.d_n);
}

// wah_decode: (in words; priv format, ngroups; out groups) -- one bitmap as
// one 31-bit word per group (group g: rows 31 g .. 31 g + 30); the output
// length is ngroups, or 0 if the words describe more groups.
int run_decode(LaunchCtx& c) {
  auto& a = *c.args;
  Env& env = *c.env;
  const uint32_t fmt = (uint32_t)a[1].priv[0];
  const uint64_t ng = a[1].priv[1];
  if (fmt > 2) return env.fail(KA_E_ARG, "wah_decode: format must be 0, 1 or 2");
  if (ng >= (1ull << 32) || ng > a[2].cap) return env.fail(KA_E_ARG, "wah_decode: ngroups exceeds the output");
  if (c.n > a[0].cap) return env.fail(KA_E_ARG, "wah_decode: range exceeds the words");
  uint32_t* reject = static_cast<uint32_t*>(env.scratch(4));
  if (!reject) return env.fail(KA_E_OOM, "wah_decode: scratch");
  int rc;
  if ((rc = launch_zero_u32(env, reject))) return rc;
  if ((rc = launch_wah_decode(env, static_cast<const uint32_t*>(a[0].ptr), c.n, c.d_n, fmt, (uint32_t)ng,
                              static_cast<uint32_t*>(a[2].ptr), reject)))
    return rc;
  return launch_len_unless(env, const_cast<uint64_t*>(a[2].d_len), ng, reject);
}

// wah_combine: (in a; in b; priv op, in_format, out_format, ngroups; out words)
// -- AND (op 0) or OR (op 1) of two bitmaps over ngroups groups, encoded in
// out_format; the output length is 0 if an input describes more groups.
int run_combine(LaunchCtx& c) {
  auto& a = *c.args;
  Env& env = *c.env;
  const uint32_t op = (uint32_t)a[2].priv[0], fin = (uint32_t)a[2].priv[1], fout = (uint32_t)a[2].priv[2];
  const uint64_t ng = a[2].priv[3];
  if (op > 1 || fin > 2 || fout > 2) return env.fail(KA_E_ARG, "wah_combine: op 0..1, formats 0..2");
  if (ng >= (1ull << 31) || 2 * ng + 1 > a[3].cap) return env.fail(KA_E_ARG, "wah_combine: ngroups exceeds the output");
  if (fout == 2 && ng > 0x1FFFFFFull) return env.fail(KA_E_ARG, "wah_combine: PLWAH fills cover at most 2^25 - 1 groups");
  uint32_t* reject = static_cast<uint32_t*>(env.scratch(4));
  if (!reject) return env.fail(KA_E_OOM, "wah_combine: scratch");
  int rc;
  if ((rc = launch_zero_u32(env, reject))) return rc;
  return launch_wah_combine(env, static_cast<const uint32_t*>(a[0].ptr), a[0].d_len ? a[0].cap : a[0].len, a[0].d_len,
                            static_cast<const uint32_t*>(a[1].ptr), a[1].d_len ? a[1].cap : a[1].len, a[1].d_len, fin,
                            (uint32_t)ng, op, fout, static_cast<uint32_t*>(a[3].ptr), const_cast<uint64_t*>(a[3].d_len),
                            reject);
}

// wah_index_batch: (in values; in req_off; priv value_bits [, largest request + 1];
//                   out keys; out offsets; out words; out key_start; out word_start)
int run_batch(LaunchCtx& c) {
  auto& a = *c.args;
  if (a[1].d_len) return c.env->fail(KA_E_ARG, "wah_index_batch: the request table's length must be known on the host");
  if (a[1].len < 2) return c.env->fail(KA_E_ARG, "wah_index_batch: the request table needs nreq + 1 >= 2 entries");
  if (a[1].len - 1 > 0xFFFFFFFFull) return c.env->fail(KA_E_ARG, "wah_index_batch: too many requests");
  const uint32_t nreq = (uint32_t)(a[1].len - 1);
  if (c.n > a[0].cap) return c.env->fail(KA_E_ARG, "wah_index_batch: range exceeds the values");
  if (a[3].cap < c.n || a[4].cap < c.n + nreq || a[5].cap < 2 * c.n || a[6].cap < nreq + 1ull ||
      a[7].cap < nreq + 1ull)
    return c.env->fail(KA_E_ARG, "wah_index_batch: outputs need capacities n, n+nreq, 2n, nreq+1, nreq+1");
  return launch_wah_batch(*c.env, static_cast<const uint32_t*>(a[0].ptr), c.n, static_cast<const uint32_t*>(a[1].ptr),
                          nreq, (uint32_t)a[2].priv[0], static_cast<uint32_t*>(a[3].ptr),
                          static_cast<uint32_t*>(a[4].ptr), static_cast<uint32_t*>(a[5].ptr),
                          static_cast<uint32_t*>(a[6].ptr), static_cast<uint32_t*>(a[7].ptr),
                          const_cast<uint64_t*>(a[3].d_len), const_cast<uint64_t*>(a[4].d_len),
                          const_cast<uint64_t*>(a[5].d_len), const_cast<uint64_t*>(a[6].d_len),
                          const_cast<uint64_t*>(a[7].d_len), 0,
                          a[2].priv[1] ? (uint32_t)(a[2].priv[1] - 1) : kMaxReqUnknown);
}

std::vector<BuiltinKernel> make_registry() {
  std::vector<BuiltinKernel> r;
  r.push_back({"affine_u32", {{KA_IN_OUT, KA_U32}, {KA_PRIV, KA_U32}, {KA_PRIV, KA_U32}}, cap_same, len_host, false,
               run_affine});
  r.push_back({"exclusive_scan_u32", {{KA_IN, KA_U32}, {KA_OUT, KA_U32}}, cap_same, len_host, false, run_scan});
  r.push_back({"compact_nonzero_u32", {{KA_IN, KA_U32}, {KA_OUT, KA_U32}}, cap_same, len_compact, false,
               run_compact});
  r.push_back({"radix_sort_rows_u32", {{KA_IN, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}}, cap_same, len_host, false,
               run_sort_rows});
  r.push_back({"radix_sort_pairs_u32",
               {{KA_IN, KA_U32}, {KA_IN, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}},
               cap_same,
               len_host,
               false,
               run_sort_pairs});
  r.push_back({"wah_encode_sorted",
               {{KA_IN, KA_U32}, {KA_IN, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}},
               cap_wah,
               len_wah,
               false,
               run_wah});
  r.push_back({"wah_index",
               {{KA_IN, KA_U32}, {KA_PRIV, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}, {KA_OUT, KA_U32}},
               cap_wah_index,
               len_wah,
               false,
               run_wah_index});
  r.push_back({"wah_lookup", {{KA_IN, KA_U32}, {KA_IN, KA_U32}, {KA_OUT, KA_U32}}, cap_same, len_host, false,
               run_lookup});
  r.push_back({"wah_decode", {{KA_IN, KA_U32}, {KA_PRIV, KA_U32}, {KA_OUT, KA_U32}}, cap_decode, len_decode, false,
               run_decode});
  r.push_back({"wah_combine",
               {{KA_IN, KA_U32}, {KA_IN, KA_U32}, {KA_PRIV, KA_U32}, {KA_OUT, KA_U32}},
               cap_combine,
               len_combine,
               false,
               run_combine});
  r.push_back({"wah_index_batch",
               {{KA_IN, KA_U32},
                {KA_IN, KA_U32},
                {KA_PRIV, KA_U32},
                {KA_OUT, KA_U32},
                {KA_OUT, KA_U32},
                {KA_OUT, KA_U32},
                {KA_OUT, KA_U32},
                {KA_OUT, KA_U32}},
               cap_batch,
               len_batch,
               true,
               run_batch});
  return r;
}

}  // namespace

const std::vector<BuiltinKernel>& builtin_kernels() {
  static const std::vector<BuiltinKernel> reg = make_registry();
  return reg;
}

const BuiltinKernel* find_builtin(const char* name) {
  if (!name) return nullptr;
  for (const auto& k : builtin_kernels())
    if (std::string(k.name) == name) return &k;
  return nullptr;
}

}  // namespace ka
