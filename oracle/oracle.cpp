// CPU oracle for the kernel-actor pipelines.
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header, table or helper with the HIP implementation, and the product path
// never calls it.
//
// Everything here is plain, sequential and unblocked, written to be checked by
// eye against the paper ("OpenCL Actors -- Adding Data Parallelism to
// Actor-based Programming with CAF", arXiv 1709.07781):
//
//  * WAH bitmap index, Sec. 4.1: values are tagged with their input position,
//    sorted by value, cut into chunk ids and literals, given fills, the fills and
//    literals are interleaved and the zero entries removed by a stream
//    compaction ("fuseFillsLiterals"), and a lookup table maps each distinct
//    value to its bitmap.  The six parts are separate functions below, called
//    in that order by ora_wah_index.
//  * Exclusive prefix sum (phase 2 of the stream compaction in Sec. 4.1) and
//    stream compaction of zero entries (Sec. 4.1).
//  * The affine stage x <- a*x + b (mod 2^32), the per-stage workload of the
//    kernel-stage overhead experiments (Sec. 3.6, Sec. 5.2-5.3).
//
// Word conventions where the paper is silent (each is a reading of the text):
//  * a literal has bit 31 clear; bit b (0..30) stands for row 31*g + b of its
//    31-row group g (least significant bit first);
//  * a fill has bit 31 set, bit 30 holds the fill bit (always 0 here), and bits
//    29..0 count the 31-row groups it covers;
//  * every non-empty group is one literal (the fill/literal pair structure of
//    fuseFillsLiterals, whose only compaction predicate is "zero"), runs of
//    empty groups before a literal become one 0-fill, counted from group 0, and
//    a bitmap ends at its last literal (no trailing fill).
//
// Encoder formats (the paper names fills "homogeneous blocks" compressed into
// one word and lists PLWAH as future work; the paper-structured form above has
// only 0-fills).  Two more formats follow the published definitions of WAH and
// PLWAH, in the same bit layout:
//  * canonical WAH: a run of groups whose 31 rows are all set ("full" groups)
//    is one 1-fill, bit 31 and bit 30 set, bits 29..0 the run length; 0-fills
//    as above;
//  * PLWAH: canonical WAH with 25-bit fill lengths (bits 24..0); bits 29..25 of
//    a fill hold a position p.  When the group right after a fill (same value,
//    next group) is a literal that differs from the fill's groups in exactly
//    one bit -- one bit set after a 0-fill, one of its 31 bits clear after a
//    1-fill -- that literal is folded into the fill with p = 1 + that bit's
//    index; p = 0 means no folded literal.
//
// Query path (the index is built to be searched: Sec. 4.1 keeps a lookup table
// from values to bitmaps; Sec. 4.2 names interactive searches and queries):
// lookup of values in the table, decoding of one bitmap (any format) into one
// 31-bit word per group, and AND / OR of two bitmaps, re-encoded.
//
// Return codes: 0 on success, -1 on a bad argument, -2 if a fill length would
// not fit its field (30 bits: unreachable for 32-bit row ids; 25 bits in PLWAH:
// more than 31 * (2^25 - 1) rows).

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

namespace {

constexpr uint32_t kGroupRows = 31;           // rows per WAH group
constexpr uint32_t kFillFlag = 0x80000000u;   // bit 31: word is a fill
constexpr uint32_t kMaxFillLen = 0x3FFFFFFFu; // bits 29..0
constexpr uint32_t kOneFill = 0x40000000u;    // bit 30: the fill bit
constexpr uint32_t kFull = 0x7FFFFFFFu;       // a group with all 31 rows set
constexpr uint32_t kPlwahMaxLen = 0x1FFFFFFu; // PLWAH: bits 24..0
constexpr uint32_t kPlwahPosShift = 25;       // PLWAH: position in bits 29..25

enum { kFormatPaper = 0, kFormatCanonical = 1, kFormatPlwah = 2 };

int popcount31(uint32_t x) {
  int c = 0;
  for (int b = 0; b < 31; ++b) c += (x >> b) & 1u;
  return c;
}

// Index (0..30) of the only set bit of x, of the only clear bit when `clear`.
uint32_t odd_bit(uint32_t x, bool clear) {
  for (uint32_t b = 0; b < 31; ++b)
    if (((x >> b) & 1u) != (clear ? 1u : 0u)) return b;
  return 31;
}

// A fill word of `len` groups in `format` (fill bit `one`), with folded
// position p (PLWAH only); -2 in *rc if len does not fit.
uint32_t fill_word(uint32_t format, bool one, uint64_t len, uint32_t p, int* rc) {
  const uint64_t lim = format == kFormatPlwah ? kPlwahMaxLen : kMaxFillLen;
  if (len > lim) *rc = -2;
  return kFillFlag | (one ? kOneFill : 0u) | (p << kPlwahPosShift) | static_cast<uint32_t>(len & lim);
}

// One bitmap given as its non-empty groups (ascending group ids c[0..m) with
// their literals lit[0..m)) encoded in `format`, appended to out.
int encode_bitmap(const uint32_t* c, const uint32_t* lit, uint64_t m, uint32_t format,
                  std::vector<uint32_t>& out) {
  int rc = 0;
  int64_t prev = -1;  // group id of the last group written (-1: none yet)
  uint64_t i = 0;
  while (i < m) {
    const int64_t gap = static_cast<int64_t>(c[i]) - prev - 1;
    if (gap < 0) return -1;
    if (format != kFormatPaper && lit[i] == kFull) {
      // a run of full groups with consecutive ids: one 1-fill
      uint64_t run = 1;
      while (i + run < m && c[i + run] == c[i] + run && lit[i + run] == kFull) ++run;
      if (gap > 0) out.push_back(fill_word(format, false, gap, 0, &rc));
      const uint64_t nx = i + run;
      uint32_t p = 0;
      if (format == kFormatPlwah && nx < m && c[nx] == c[i] + run && popcount31(lit[nx]) == 30)
        p = 1 + odd_bit(lit[nx], true);
      out.push_back(fill_word(format, true, run, p, &rc));
      prev = static_cast<int64_t>(c[i] + run - 1) + (p ? 1 : 0);
      i = nx + (p ? 1 : 0);
      continue;
    }
    if (format == kFormatPlwah && gap > 0 && popcount31(lit[i]) == 1) {
      out.push_back(fill_word(format, false, gap, 1 + odd_bit(lit[i], false), &rc));
    } else {
      if (gap > 0) out.push_back(fill_word(format, false, gap, 0, &rc));
      out.push_back(lit[i]);
    }
    prev = c[i];
    ++i;
  }
  return rc;
}

}  // namespace

extern "C" {

// Parts 1 and 2 (Sec. 4.1): tag each value with its input position and sort by
// value.  Ties keep input order (a stable sort), which is what keeps the rows
// of one value ascending.  rows == nullptr means rows 0..n-1.
int ora_sort_pairs(const uint32_t* keys, const uint32_t* rows, uint64_t n,
                   uint32_t* skeys, uint32_t* srows) {
  if (n && (!keys || !skeys || !srows)) return -1;
  std::vector<uint64_t> perm(n);
  std::iota(perm.begin(), perm.end(), uint64_t{0});
  std::stable_sort(perm.begin(), perm.end(),
                   [&](uint64_t a, uint64_t b) { return keys[a] < keys[b]; });
  for (uint64_t j = 0; j < n; ++j) {
    skeys[j] = keys[perm[j]];
    srows[j] = rows ? rows[perm[j]] : static_cast<uint32_t>(perm[j]);
  }
  return 0;
}

// Part 3 (Sec. 4.1): chunk ids and literals.  In the sorted (value, row)
// sequence a group is a maximal run with the same value and the same chunk id
// row / 31.  Each group yields its value, its chunk id and its literal, the OR
// of 1 << (row % 31) over its rows.  Outputs hold n entries; *k receives the
// number of groups.
int ora_wah_groups(const uint32_t* skeys, const uint32_t* srows, uint64_t n,
                   uint32_t* gkey, uint32_t* gchunk, uint32_t* glit, uint64_t* k) {
  if (!k || (n && (!skeys || !srows || !gkey || !gchunk || !glit))) return -1;
  uint64_t g = 0;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t chunk = srows[i] / kGroupRows;
    const uint32_t bit = 1u << (srows[i] % kGroupRows);
    const bool same = g > 0 && gkey[g - 1] == skeys[i] && gchunk[g - 1] == chunk;
    if (same) {
      glit[g - 1] |= bit;
    } else {
      gkey[g] = skeys[i];
      gchunk[g] = chunk;
      glit[g] = bit;
      ++g;
    }
  }
  *k = g;
  return 0;
}

// Part 4 (Sec. 4.1): fills.  The fill in front of group g covers the empty
// groups between the previous group of the same value (or group -1 when g is
// the first group of its value) and g.  A gap of zero gives the word 0, which
// the compaction of part 5 removes.
int ora_wah_fills(const uint32_t* gkey, const uint32_t* gchunk, uint64_t k, uint32_t* gfill) {
  if (k && (!gkey || !gchunk || !gfill)) return -1;
  for (uint64_t g = 0; g < k; ++g) {
    const bool first_of_value = (g == 0) || gkey[g - 1] != gkey[g];
    const int64_t prev = first_of_value ? -1 : static_cast<int64_t>(gchunk[g - 1]);
    const int64_t gap = static_cast<int64_t>(gchunk[g]) - prev - 1;
    if (gap < 0) return -1;  // groups of one value must have increasing chunk ids
    if (gap > kMaxFillLen) return -2;
    gfill[g] = gap > 0 ? (kFillFlag | static_cast<uint32_t>(gap)) : 0u;
  }
  return 0;
}

// Part 5a, "prepare_index" (Sec. 4.1): interleave fills and literals into a
// 2k-entry index, the fill of each group in front of its literal.
int ora_wah_interleave(const uint32_t* gfill, const uint32_t* glit, uint64_t k, uint32_t* index) {
  if (k && (!gfill || !glit || !index)) return -1;
  for (uint64_t g = 0; g < k; ++g) {
    index[2 * g] = gfill[g];
    index[2 * g + 1] = glit[g];
  }
  return 0;
}

// Part 5b, stream compaction (Sec. 4.1): keep the non-zero entries in order.
int ora_compact_nonzero(const uint32_t* in, uint64_t m, uint32_t* out, uint64_t* kept) {
  if (!kept || (m && (!in || !out))) return -1;
  uint64_t w = 0;
  for (uint64_t i = 0; i < m; ++i)
    if (in[i] != 0) out[w++] = in[i];
  *kept = w;
  return 0;
}

// Part 6 (Sec. 4.1): lookup table.  keys[d] is the d-th distinct value in
// ascending order and offsets[d] the position of its first word among the
// compacted words; offsets[D] = W.  The position of group g's first word is the
// number of non-zero index entries in front of index[2g].
int ora_wah_table(const uint32_t* gkey, const uint32_t* index, uint64_t k,
                  uint32_t* keys, uint32_t* offsets, uint64_t* D) {
  if (!D || !offsets || (k && (!gkey || !index || !keys))) return -1;
  uint64_t d = 0, kept = 0;
  for (uint64_t g = 0; g < k; ++g) {
    if (g == 0 || gkey[g - 1] != gkey[g]) {
      keys[d] = gkey[g];
      offsets[d] = static_cast<uint32_t>(kept);
      ++d;
    }
    kept += (index[2 * g] != 0) + (index[2 * g + 1] != 0);
  }
  offsets[d] = static_cast<uint32_t>(kept);
  *D = d;
  return 0;
}

// The whole index build: parts 1..6 in the paper's order.
// keys needs n entries, offsets n + 1, words 2n.
int ora_wah_index(const uint32_t* values, uint64_t n, uint32_t* keys, uint32_t* offsets,
                  uint32_t* words, uint64_t* D, uint64_t* W) {
  if (!D || !W || !offsets || (n && (!values || !keys || !words))) return -1;
  std::vector<uint32_t> skeys(n), srows(n), gkey(n), gchunk(n), glit(n), gfill(n), index(2 * n);
  uint64_t k = 0;
  int rc = ora_sort_pairs(values, nullptr, n, skeys.data(), srows.data());
  if (!rc) rc = ora_wah_groups(skeys.data(), srows.data(), n, gkey.data(), gchunk.data(), glit.data(), &k);
  if (!rc) rc = ora_wah_fills(gkey.data(), gchunk.data(), k, gfill.data());
  if (!rc) rc = ora_wah_interleave(gfill.data(), glit.data(), k, index.data());
  if (!rc) rc = ora_compact_nonzero(index.data(), 2 * k, words, W);
  if (!rc) rc = ora_wah_table(gkey.data(), index.data(), k, keys, offsets, D);
  return rc;
}

// Parts 3..6 from an already sorted (value, row) sequence.
int ora_wah_encode_sorted(const uint32_t* skeys, const uint32_t* srows, uint64_t n, uint32_t* keys,
                          uint32_t* offsets, uint32_t* words, uint64_t* D, uint64_t* W) {
  if (!D || !W || !offsets || (n && (!skeys || !srows || !keys || !words))) return -1;
  std::vector<uint32_t> gkey(n), gchunk(n), glit(n), gfill(n), index(2 * n);
  uint64_t k = 0;
  int rc = ora_wah_groups(skeys, srows, n, gkey.data(), gchunk.data(), glit.data(), &k);
  if (!rc) rc = ora_wah_fills(gkey.data(), gchunk.data(), k, gfill.data());
  if (!rc) rc = ora_wah_interleave(gfill.data(), glit.data(), k, index.data());
  if (!rc) rc = ora_compact_nonzero(index.data(), 2 * k, words, W);
  if (!rc) rc = ora_wah_table(gkey.data(), index.data(), k, keys, offsets, D);
  return rc;
}

// The index in an encoder format, from the groups of part 3 (value, group id,
// literal; sorted by value, then group id): each value's groups are encoded
// as one bitmap (see encode_bitmap), keys and offsets as in part 6.
int ora_wah_encode_groups(const uint32_t* gkey, const uint32_t* gchunk, const uint32_t* glit, uint64_t k,
                          uint32_t format, uint32_t* keys, uint32_t* offsets, uint32_t* words, uint64_t* D,
                          uint64_t* W) {
  if (!D || !W || !offsets || format > kFormatPlwah || (k && (!gkey || !gchunk || !glit || !keys || !words)))
    return -1;
  std::vector<uint32_t> out;
  uint64_t d = 0, g = 0;
  int rc = 0;
  while (g < k) {
    uint64_t e = g;
    while (e < k && gkey[e] == gkey[g]) ++e;
    keys[d] = gkey[g];
    offsets[d] = static_cast<uint32_t>(out.size());
    ++d;
    const int r = encode_bitmap(gchunk + g, glit + g, e - g, format, out);
    if (r == -1) return -1;
    if (r) rc = r;
    g = e;
  }
  offsets[d] = static_cast<uint32_t>(out.size());
  std::copy(out.begin(), out.end(), words);
  *D = d;
  *W = out.size();
  return rc;
}

// The whole index build in an encoder format: parts 1-3, then the format's
// encoding of each value's groups.  keys needs n entries, offsets n + 1,
// words 2n.
int ora_wah_index_format(const uint32_t* values, uint64_t n, uint32_t format, uint32_t* keys, uint32_t* offsets,
                         uint32_t* words, uint64_t* D, uint64_t* W) {
  if (!D || !W || !offsets || format > kFormatPlwah || (n && (!values || !keys || !words))) return -1;
  std::vector<uint32_t> skeys(n), srows(n), gkey(n), gchunk(n), glit(n);
  uint64_t k = 0;
  int rc = ora_sort_pairs(values, nullptr, n, skeys.data(), srows.data());
  if (!rc) rc = ora_wah_groups(skeys.data(), srows.data(), n, gkey.data(), gchunk.data(), glit.data(), &k);
  if (!rc) rc = ora_wah_encode_groups(gkey.data(), gchunk.data(), glit.data(), k, format, keys, offsets, words, D, W);
  return rc;
}

// Lookup (part 6's table read back): slots[i] = d with keys[d] == queries[i],
// or 0xFFFFFFFF when the value has no bitmap.  keys ascending.
int ora_wah_lookup(const uint32_t* keys, uint64_t D, const uint32_t* queries, uint64_t q, uint32_t* slots) {
  if ((D && !keys) || (q && (!queries || !slots))) return -1;
  for (uint64_t i = 0; i < q; ++i) {
    const uint32_t* p = std::lower_bound(keys, keys + D, queries[i]);
    slots[i] = (p != keys + D && *p == queries[i]) ? static_cast<uint32_t>(p - keys) : 0xFFFFFFFFu;
  }
  return 0;
}

// Decodes one bitmap's words (any format) into ngroups 31-bit group words:
// groups[g] has bit b set iff row 31 g + b is in the bitmap.  -1 if the words
// describe more than ngroups groups.
int ora_wah_decode(const uint32_t* words, uint64_t m, uint32_t format, uint64_t ngroups, uint32_t* groups) {
  if (format > kFormatPlwah || (m && !words) || (ngroups && !groups)) return -1;
  for (uint64_t g = 0; g < ngroups; ++g) groups[g] = 0;
  uint64_t g = 0;
  for (uint64_t i = 0; i < m; ++i) {
    const uint32_t w = words[i];
    if (!(w & kFillFlag)) {
      if (g >= ngroups) return -1;
      groups[g++] = w;
      continue;
    }
    const bool one = (w & kOneFill) != 0;
    const uint64_t len = format == kFormatPlwah ? (w & kPlwahMaxLen) : (w & kMaxFillLen);
    const uint32_t p = format == kFormatPlwah ? (w >> kPlwahPosShift) & 31u : 0u;
    if (g + len + (p ? 1 : 0) > ngroups) return -1;
    for (uint64_t j = 0; j < len; ++j) groups[g++] = one ? kFull : 0u;
    if (p) groups[g++] = one ? (kFull & ~(1u << (p - 1))) : (1u << (p - 1));
  }
  return 0;
}

// AND (op 0) or OR (op 1) of two bitmaps in format `in_format` over ngroups
// groups: decoded, combined group by group, and the non-empty groups of the
// result encoded as one bitmap in `out_format`.  out needs 2 * ngroups words;
// *m_out receives the word count.
int ora_wah_combine(const uint32_t* a, uint64_t ma, const uint32_t* b, uint64_t mb, uint32_t in_format,
                    uint64_t ngroups, uint32_t op, uint32_t out_format, uint32_t* out, uint64_t* m_out) {
  if (op > 1 || out_format > kFormatPlwah || !m_out || (ngroups && !out)) return -1;
  std::vector<uint32_t> ga(ngroups), gb(ngroups);
  int rc = ora_wah_decode(a, ma, in_format, ngroups, ga.data());
  if (!rc) rc = ora_wah_decode(b, mb, in_format, ngroups, gb.data());
  if (rc) return rc;
  std::vector<uint32_t> c, lit;
  for (uint64_t g = 0; g < ngroups; ++g) {
    const uint32_t x = op == 0 ? (ga[g] & gb[g]) : (ga[g] | gb[g]);
    if (x) {
      c.push_back(static_cast<uint32_t>(g));
      lit.push_back(x);
    }
  }
  std::vector<uint32_t> res;
  rc = encode_bitmap(c.data(), lit.data(), c.size(), out_format, res);
  if (rc == -1) return rc;
  std::copy(res.begin(), res.end(), out);
  *m_out = res.size();
  return rc;
}

// Exclusive prefix sum in uint32 arithmetic (wraps mod 2^32): out[0] = 0,
// out[i] = in[0] + ... + in[i-1].
int ora_exclusive_scan(const uint32_t* in, uint64_t m, uint32_t* out) {
  if (m && (!in || !out)) return -1;
  uint32_t acc = 0;
  for (uint64_t i = 0; i < m; ++i) {
    const uint32_t v = in[i];
    out[i] = acc;
    acc += v;
  }
  return 0;
}

// The affine chain: stage s maps x to a[s] * x + b[s] in uint32 arithmetic.
int ora_affine_chain(uint32_t* x, uint64_t m, const uint32_t* a, const uint32_t* b, uint32_t stages) {
  if ((m && !x) || (stages && (!a || !b))) return -1;
  for (uint32_t s = 0; s < stages; ++s)
    for (uint64_t i = 0; i < m; ++i) x[i] = a[s] * x[i] + b[s];
  return 0;
}

}  // extern "C"
