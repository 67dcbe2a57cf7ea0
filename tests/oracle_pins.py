"""Pins that tie the CPU oracle to the paper and to mathematics, not to itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with something the paper or the mathematics fixes:

* hand-derived worked examples under ``tests/golden`` (Sec. 4.1 conventions);
* a brute-force encoder written from the definition of a WAH-compressed bitmap
  (one dense bitmap per distinct value, cut into 31-row groups), which shares
  no step with the oracle's sort-based six-part pipeline;
* a decoder written from the word format: decode(encode(v)) must give back the
  indicator bitmap of every value;
* closed forms (single row, constant input, all-distinct input, alternating
  chunks, constant scan input, composed affine maps and their inverses);
* invariants (each row in exactly one bitmap, popcounts add up to n, no zero
  words, W <= 2k <= 2n, sorted keys, offsets ending at W);
* other libraries (numpy's stable argsort, cumsum and boolean masks).

``tests/test_oracle_mutants.py`` plants plausible mistakes in copies of the
oracle and checks that some pin here fails for each.
"""
from __future__ import annotations

import json
import os

import numpy as np

import workloads

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FILL = 0x80000000


# --- independent helpers (definitions, not the oracle's steps) ----------------------

def decode_bitmap(words, n: int) -> np.ndarray:
    """Dense bitmap of n rows from one value's WAH words (word-format definition)."""
    bits = np.zeros(n, dtype=bool)
    g = 0
    for w in (int(x) for x in words):
        if w & FILL:
            length = w & 0x3FFFFFFF
            assert length >= 1, "fill of length 0"
            if w & 0x40000000:
                bits[31 * g: min(n, 31 * (g + length))] = True
            g += length
        else:
            for b in range(31):
                if (w >> b) & 1:
                    r = 31 * g + b
                    assert r < n, f"literal bit for row {r} >= n={n}"
                    bits[r] = True
            g += 1
    return bits


def brute_force_index(v: np.ndarray):
    """WAH index from the definition: for each distinct value x ascending, the
    bitmap [v == x] cut into 31-row groups; each non-empty group is a literal,
    each run of empty groups before a literal is one 0-fill, no trailing fill."""
    v = np.asarray(v, dtype=np.uint32)
    n = v.size
    ngroups = (n + 30) // 31
    keys, offsets, words = [], [0], []
    for x in sorted(set(int(t) for t in v)):
        bm = np.zeros(ngroups * 31, dtype=np.uint64)
        bm[:n] = (v == x)
        grp = bm.reshape(ngroups, 31) if ngroups else bm.reshape(0, 31)
        lits = (grp << np.arange(31, dtype=np.uint64)).sum(axis=1)
        run = 0
        for lit in (int(t) for t in lits):
            if lit == 0:
                run += 1
            else:
                if run:
                    words.append(FILL | run)
                words.append(lit)
                run = 0
        keys.append(x)
        offsets.append(len(words))
    return (np.array(keys, dtype=np.uint32), np.array(offsets, dtype=np.uint32),
            np.array(words, dtype=np.uint32))


FMT_PAPER, FMT_CANONICAL, FMT_PLWAH = 0, 1, 2
FULL = 0x7FFFFFFF


def decode_groups_format(words, fmt: int) -> list[int]:
    """The 31-bit group words one bitmap's words stand for, from the word
    layout of each format: a literal is one group; a fill is `length` groups
    of 0 or all 31 bits (bit 30); in PLWAH the length has 25 bits and a
    non-zero position p in bits 29..25 adds one group that differs from the
    fill's groups in bit p - 1."""
    out = []
    for w in (int(x) for x in words):
        if not w & FILL:
            out.append(w)
            continue
        one = bool(w & 0x40000000)
        length = w & (0x1FFFFFF if fmt == FMT_PLWAH else 0x3FFFFFFF)
        pos = (w >> 25) & 31 if fmt == FMT_PLWAH else 0
        assert length >= 1, "fill of length 0"
        out += [FULL if one else 0] * length
        if pos:
            out.append(FULL ^ (1 << (pos - 1)) if one else 1 << (pos - 1))
    return out


def dense_groups(bits: np.ndarray) -> list[int]:
    """31-bit group words of a boolean row vector (rows beyond it are 0)."""
    n = bits.size
    ng = (n + 30) // 31
    padded = np.zeros(ng * 31, dtype=np.uint64)
    padded[:n] = bits
    grp = padded.reshape(ng, 31) if ng else padded.reshape(0, 31)
    return [int(t) for t in (grp << np.arange(31, dtype=np.uint64)).sum(axis=1)]


def definition_bitmap_words(groups: list[int], fmt: int) -> list[int]:
    """One bitmap from the definition of each format, in two steps: first
    run-length encode the group sequence (trailing empty groups dropped):
    a run of empty groups is a 0-fill, a run of full groups a 1-fill (canonical
    and PLWAH; the paper form keeps full groups as literals), every other
    group a literal; then, for PLWAH, fold a literal that differs from the
    fill just before it in one bit into that fill."""
    while groups and groups[-1] == 0:
        groups = groups[:-1]
    words, i = [], 0
    while i < len(groups):
        g = groups[i]
        homog = g == 0 or (g == FULL and fmt != FMT_PAPER)
        if homog:
            j = i
            while j < len(groups) and groups[j] == g:
                j += 1
            words.append(("fill", g == FULL, j - i))
            i = j
        else:
            words.append(("lit", g))
            i += 1
    out, k = [], 0
    while k < len(words):
        w = words[k]
        if w[0] == "lit":
            out.append(w[1])
            k += 1
            continue
        _, one, length = w
        pos = 0
        if fmt == FMT_PLWAH and k + 1 < len(words) and words[k + 1][0] == "lit":
            diff = words[k + 1][1] ^ (FULL if one else 0)
            if bin(diff).count("1") == 1:
                pos = diff.bit_length()
                k += 1
        limit = 0x1FFFFFF if fmt == FMT_PLWAH else 0x3FFFFFFF
        assert length <= limit
        out.append(FILL | (0x40000000 if one else 0) | (pos << 25) | length)
        k += 1
    return out


def definition_index_format(v: np.ndarray, fmt: int):
    """The index of v in format fmt from the definition (dense bitmap per value)."""
    v = np.asarray(v, dtype=np.uint32)
    keys, offsets, words = [], [0], []
    for x in sorted(set(int(t) for t in v)):
        words += definition_bitmap_words(dense_groups(v == x), fmt)
        keys.append(x)
        offsets.append(len(words))
    return (np.array(keys, dtype=np.uint32), np.array(offsets, dtype=np.uint32),
            np.array(words, dtype=np.uint32))


def check_invariants(v: np.ndarray, keys, offsets, words):
    """Properties any correct index of v has, whatever the encoder."""
    v = np.asarray(v, dtype=np.uint32)
    n = v.size
    keys, offsets, words = (np.asarray(a, dtype=np.uint32) for a in (keys, offsets, words))
    D, W = keys.size, words.size
    assert offsets.size == D + 1 and int(offsets[0]) == 0 and int(offsets[-1]) == W
    assert np.all(np.diff(offsets.astype(np.int64)) > 0), "each value has at least one word"
    assert np.all(np.diff(keys.astype(np.int64)) > 0), "keys strictly increasing"
    np.testing.assert_array_equal(keys, np.unique(v))
    assert not np.any(words == 0), "no zero words"
    fills = (words & FILL) != 0
    assert not np.any(words[fills] & 0x40000000), "only 0-fills"
    assert np.all((words[fills] & 0x3FFFFFFF) >= 1), "fill length >= 1"
    lits = ~fills
    # popcount of all literals adds up to n (0-fills carry no set bits)
    pc = np.unpackbits(words[lits].view(np.uint8)).sum() if lits.any() else 0
    assert int(pc) == n
    covered = np.zeros(n, dtype=np.int64)
    ngroups = (n + 30) // 31
    k = 0
    for d in range(D):
        wd = words[offsets[d]:offsets[d + 1]]
        # a bitmap ends with a literal and never has two fills in a row
        assert not (int(wd[-1]) & FILL)
        f = (wd & FILL) != 0
        assert not np.any(f[1:] & f[:-1])
        bm = decode_bitmap(wd, n)
        np.testing.assert_array_equal(bm, v == keys[d])
        covered += bm
        # #literals = #distinct 31-row groups the value touches
        rows = np.nonzero(v == keys[d])[0]
        nl = int(np.count_nonzero(~f))
        assert nl == np.unique(rows // 31).size
        k += nl
        assert int(np.count_nonzero(bm)) == rows.size
    assert np.all(covered == 1), "each row in exactly one bitmap"
    assert W <= 2 * k <= 2 * n
    assert k <= D * max(ngroups, 1)


def _load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    if "values" in g:
        v = np.array(g["values"], dtype=np.uint32)
    elif "values_sparse" in g:
        s = g["values_sparse"]
        v = np.full(s["n"], s["default"], dtype=np.uint32)
        for r, x in s["set"]:
            v[r] = x
    else:
        v = None
    return g, v


def _hex(a):
    return np.array([int(x, 16) for x in a], dtype=np.uint32)


# --- pins -------------------------------------------------------------------------

def pin_golden_indexes(o):
    for name in ("wah_small_two_values.json", "wah_fills_and_tail.json", "wah_long_fill_max_key.json"):
        g, v = _load_golden(name)
        keys, offs, words = o.wah_index(v)
        np.testing.assert_array_equal(keys, np.array(g["keys"], dtype=np.uint32), err_msg=name)
        np.testing.assert_array_equal(offs, np.array(g["offsets"], dtype=np.uint32), err_msg=name)
        np.testing.assert_array_equal(words, _hex(g["words"]), err_msg=name)


def pin_golden_fuse_stages(o):
    g, _ = _load_golden("fuse_fills_literals_stages.json")
    gk = np.array(g["gkey"], dtype=np.uint32)
    gc = np.array(g["gchunk"], dtype=np.uint32)
    np.testing.assert_array_equal(o.wah_fills(gk, gc), _hex(g["gfill"]))
    idx = o.wah_interleave(_hex(g["gfill"]), _hex(g["glit"]))
    np.testing.assert_array_equal(idx, _hex(g["index"]))
    np.testing.assert_array_equal(o.compact_nonzero(idx), _hex(g["compacted"]))
    tk, to = o.wah_table(gk, idx)
    np.testing.assert_array_equal(tk, np.array(g["table_keys"], dtype=np.uint32))
    np.testing.assert_array_equal(to, np.array(g["table_offsets"], dtype=np.uint32))


def pin_brute_force_small(o):
    kinds = ("uniform1024", "all_equal", "distinct", "reverse", "alternating_chunks", "sparse_hot",
             "high_bits", "zipf")
    sizes = list(range(0, 70)) + [93, 124, 125, 127, 128, 255, 256, 257, 500, 1000, 1023, 1024, 1025]
    for kind in kinds:
        for n in sizes:
            v = workloads.structured(kind, n, seed=n + 17)
            if kind in ("uniform1024",):
                v = v % np.uint32(max(1, n // 7 + 1))  # small alphabets to get long runs too
            got = o.wah_index(v)
            exp = brute_force_index(v)
            for a, b, what in zip(got, exp, ("keys", "offsets", "words")):
                np.testing.assert_array_equal(a, b, err_msg=f"{what} {kind} n={n}")


def pin_decode_and_invariants(o):
    for kind in workloads.STRUCTURED_KINDS:
        for n in (0, 1, 30, 31, 32, 61, 62, 63, 64, 500, 4096, 4097):
            v = workloads.structured(kind, n, seed=3 * n + 1)
            check_invariants(v, *o.wah_index(v))


def pin_closed_forms(o):
    # a single row r of value x: [fill(floor(r/31)) if r >= 31] + [1 << (r % 31)]
    for n in (1, 31, 32, 100, 1000):
        for r in sorted({0, 30, 31, n - 1, n // 2}):
            if r >= n:
                continue
            v = np.zeros(n, dtype=np.uint32)
            v[r] = 9
            keys, offs, words = o.wah_index(v)
            exp9 = ([FILL | (r // 31)] if r >= 31 else []) + [1 << (r % 31)]
            np.testing.assert_array_equal(words[offs[-2]:offs[-1]], np.array(exp9, dtype=np.uint32))
    # constant input: floor(n/31) full literals and a partial tail, no fills
    for n in (1, 30, 31, 32, 62, 63, 1000, 31 * 40):
        keys, offs, words = o.wah_index(np.full(n, 3, dtype=np.uint32))
        exp = [0x7FFFFFFF] * (n // 31) + ([(1 << (n % 31)) - 1] if n % 31 else [])
        np.testing.assert_array_equal(keys, [3])
        np.testing.assert_array_equal(offs, [0, len(exp)])
        np.testing.assert_array_equal(words, np.array(exp, dtype=np.uint32))
    # all distinct v[r] = r: D = n, W = n + #{r >= 31}
    for n in (1, 31, 32, 200):
        keys, offs, words = o.wah_index(np.arange(n, dtype=np.uint32))
        assert keys.size == n and words.size == n + max(0, n - 31)
    # v[r] = floor(r/31) mod 2: alternating full literals and length-1 fills
    for n in (62, 93, 100, 31 * 9 + 5):
        v = ((np.arange(n) // 31) % 2).astype(np.uint32)
        keys, offs, words = o.wah_index(v)
        ng = (n + 30) // 31
        tail = (1 << (n % 31)) - 1 if n % 31 else 0x7FFFFFFF
        lit = lambda g: tail if g == ng - 1 else 0x7FFFFFFF
        exp0 = [lit(g) if i == 0 else x for i, g in enumerate(range(0, ng, 2)) for x in
                ([lit(g)] if i == 0 else [FILL | 1, lit(g)])]
        exp1 = [x for g in range(1, ng, 2) for x in [FILL | 1, lit(g)]]
        np.testing.assert_array_equal(words, np.array(exp0 + exp1, dtype=np.uint32))
    # n <= 31: never a fill
    for n in range(1, 32):
        v = workloads.structured("u32", n, seed=n) % np.uint32(5)
        _, _, words = o.wah_index(v.astype(np.uint32))
        assert not np.any(words & FILL)


def pin_empty(o):
    keys, offs, words = o.wah_index(np.zeros(0, dtype=np.uint32))
    assert keys.size == 0 and words.size == 0
    np.testing.assert_array_equal(offs, [0])


def pin_sort_pairs(o):
    for kind in ("uniform1024", "u32", "all_equal", "distinct", "reverse", "zipf", "all_max", "high_bits"):
        for n in (0, 1, 2, 255, 256, 257, 5000):
            v = workloads.structured(kind, n, seed=n + 5)
            sk, sr = o.sort_pairs(v)
            perm = np.argsort(v, kind="stable")
            np.testing.assert_array_equal(sk, v[perm])
            np.testing.assert_array_equal(sr, perm.astype(np.uint32))
            # explicit rows follow their keys
            rows = workloads.u32(n + 99, n)
            sk2, sr2 = o.sort_pairs(v, rows)
            np.testing.assert_array_equal(sk2, v[perm])
            np.testing.assert_array_equal(sr2, rows[perm])
    # brute-force counting sort on a tiny alphabet
    v = workloads.uniform_values(11, 300, 4)
    sk, sr = o.sort_pairs(v)
    exp_rows = [r for x in range(4) for r in range(300) if v[r] == x]
    np.testing.assert_array_equal(sr, np.array(exp_rows, dtype=np.uint32))


def pin_exclusive_scan(o):
    for n in (0, 1, 2, 1000, 4097):
        x = workloads.u32(n + 3, n)
        got = o.exclusive_scan(x)
        exp = np.zeros(n, dtype=np.uint64)
        if n:
            exp[1:] = np.cumsum(x.astype(np.uint64))[:-1]
        np.testing.assert_array_equal(got, (exp & np.uint64(0xFFFFFFFF)).astype(np.uint32))
    # constant c: out[i] = i*c mod 2^32 (wraps)
    c = 0xDEADBEEF
    got = o.exclusive_scan(np.full(3000, c, dtype=np.uint32))
    exp = (np.arange(3000, dtype=np.uint64) * np.uint64(c)) & np.uint64(0xFFFFFFFF)
    np.testing.assert_array_equal(got, exp.astype(np.uint32))


def pin_compact(o):
    for n in (0, 1, 7, 1000, 4097):
        x = workloads.u32(n + 1, n)
        x[workloads.uniform_values(n + 2, n, 3) == 0] = 0
        np.testing.assert_array_equal(o.compact_nonzero(x), x[x != 0])
    np.testing.assert_array_equal(o.compact_nonzero(np.zeros(10, np.uint32)), np.zeros(0, np.uint32))
    y = np.array([0, 0, 5, 0, 7], dtype=np.uint32)
    np.testing.assert_array_equal(o.compact_nonzero(y), [5, 7])


def _inv_odd(a: int) -> int:
    """Inverse of an odd a mod 2^32 by Newton iteration x <- x(2 - a x)."""
    x = a  # correct to 3 bits for odd a
    for _ in range(5):
        x = (x * (2 - a * x)) & 0xFFFFFFFF
    return x


def pin_affine(o):
    a, b = workloads.affine_params(123, 8)
    x = workloads.u32(7, 5000)
    y = o.affine_chain(x, a, b)
    # closed-form composition: (A, B) <- (a A, a B + b) applied once
    A, B = 1, 0
    for ai, bi in zip(a.tolist(), b.tolist()):
        A, B = (ai * A) & 0xFFFFFFFF, (ai * B + bi) & 0xFFFFFFFF
    exp = (x.astype(np.uint64) * np.uint64(A) + np.uint64(B)) & np.uint64(0xFFFFFFFF)
    np.testing.assert_array_equal(y, exp.astype(np.uint32))
    # invertibility: undo the stages in reverse order
    z = y.astype(np.uint64)
    for ai, bi in zip(reversed(a.tolist()), reversed(b.tolist())):
        z = ((z - np.uint64(bi)) * np.uint64(_inv_odd(ai))) & np.uint64(0xFFFFFFFF)
    np.testing.assert_array_equal(z.astype(np.uint32), x)


def pin_stage_composition(o):
    """fuse(msg) = move(count(prepare(msg))): the staged parts compose to the full build."""
    for kind in ("uniform1024", "zipf", "alternating_chunks", "distinct"):
        v = workloads.structured(kind, 3001, seed=4)
        sk, sr = o.sort_pairs(v)
        gk, gc, gl = o.wah_groups(sk, sr)
        gf = o.wah_fills(gk, gc)
        idx = o.wah_interleave(gf, gl)
        words = o.compact_nonzero(idx)
        tk, to = o.wah_table(gk, idx)
        full = o.wah_index(v)
        np.testing.assert_array_equal(words, full[2])
        np.testing.assert_array_equal(tk, full[0])
        np.testing.assert_array_equal(to, full[1])
        enc = o.wah_encode_sorted(sk, sr)
        for a, b in zip(enc, full):
            np.testing.assert_array_equal(a, b)
        assert words.size <= idx.size  # compaction never grows the index


def pin_golden_formats(o):
    g, v = _load_golden("wah_formats_fills_and_tail.json")
    for fmt, name in ((FMT_CANONICAL, "canonical"), (FMT_PLWAH, "plwah")):
        keys, offs, words = o.wah_index_format(v, fmt)
        np.testing.assert_array_equal(keys, np.array(g["keys"], dtype=np.uint32))
        np.testing.assert_array_equal(offs, np.array(g[name]["offsets"], dtype=np.uint32), err_msg=name)
        np.testing.assert_array_equal(words, _hex(g[name]["words"]), err_msg=name)


def pin_formats_brute_force(o):
    """Canonical WAH and PLWAH (and the paper form through the same entry)
    against the definition encoder, over structured layouts and sizes that
    cross group edges; full runs come from all-equal, alternating and sorted
    inputs."""
    kinds = ("all_equal", "alternating_chunks", "presorted", "uniform1024", "distinct", "sparse_hot", "zipf")
    sizes = list(range(0, 70)) + [92, 93, 94, 124, 155, 186, 500, 1000, 1023, 1025]
    for fmt in (FMT_PAPER, FMT_CANONICAL, FMT_PLWAH):
        for kind in kinds:
            for n in sizes:
                v = workloads.structured(kind, n, seed=n + 29)
                if kind == "uniform1024":
                    v = v % np.uint32(max(1, n // 40 + 1))
                got = o.wah_index_format(v, fmt)
                exp = definition_index_format(v, fmt)
                for a, b, what in zip(got, exp, ("keys", "offsets", "words")):
                    np.testing.assert_array_equal(a, b, err_msg=f"{what} fmt={fmt} {kind} n={n}")


def pin_formats_decode(o):
    """decode(encode(v)) gives every value's rows back in each format, and each
    encoding is in its normal form: no full literal in canonical WAH and PLWAH,
    no two adjacent fills of one kind (unless the first holds a folded
    literal), and in PLWAH no fill followed by a literal that differs from it
    in one bit."""
    for kind in workloads.STRUCTURED_KINDS:
        for n in (0, 1, 30, 31, 32, 62, 63, 93, 124, 500, 4097):
            v = workloads.structured(kind, n, seed=5 * n + 2)
            for fmt in (FMT_CANONICAL, FMT_PLWAH):
                keys, offs, words = o.wah_index_format(v, fmt)
                np.testing.assert_array_equal(keys, np.unique(v))
                assert offs[0] == 0 and offs[-1] == words.size
                for d in range(keys.size):
                    wd = [int(x) for x in words[offs[d]:offs[d + 1]]]
                    groups = decode_groups_format(wd, fmt)
                    ref = dense_groups(v == keys[d])
                    assert groups == ref[:len(groups)] and not any(ref[len(groups):]), (kind, n, fmt, d)
                    assert FULL not in wd, "a full group left as a literal"
                    for a, b in zip(wd, wd[1:]):
                        if a & FILL and b & FILL:  # (a PLWAH fill with a folded literal ends its run)
                            assert (a ^ b) & 0x40000000 or (fmt == FMT_PLWAH and (a >> 25) & 31), \
                                "two adjacent fills of one kind"
                        if fmt == FMT_PLWAH and a & FILL and not b & FILL:
                            diff = b ^ (FULL if a & 0x40000000 else 0)
                            assert bin(diff).count("1") != 1 or (a >> 25) & 31, "literal not folded"


def pin_formats_closed_forms(o):
    # constant input of n = 31 m + t rows: one 1-fill of m groups, then the
    # tail literal; PLWAH folds a 30-row tail (its clear bit is bit 30, p = 31)
    for m, t in ((0, 5), (1, 0), (1, 30), (3, 7), (40, 30), (40, 0)):
        n = 31 * m + t
        v = np.full(n, 4, dtype=np.uint32)
        tail = [(1 << t) - 1] if t else []
        can = ([0xC0000000 | m] if m else []) + tail
        np.testing.assert_array_equal(o.wah_index_format(v, FMT_CANONICAL)[2], np.array(can, dtype=np.uint32))
        pl = ([0xC0000000 | (31 << 25) | m] if m and t == 30 else can)
        np.testing.assert_array_equal(o.wah_index_format(v, FMT_PLWAH)[2], np.array(pl, dtype=np.uint32))
    # a single row r: PLWAH writes one word, a fill with p = r % 31 + 1, when r >= 31
    for r in (0, 30, 31, 100, 31 * 1000 + 17):
        v = np.zeros(r + 1, dtype=np.uint32)
        v[r] = 8
        _, offs, words = o.wah_index_format(v, FMT_PLWAH)
        exp = [FILL | ((r % 31 + 1) << 25) | (r // 31)] if r >= 31 else [1 << r]
        np.testing.assert_array_equal(words[offs[-2]:offs[-1]], np.array(exp, dtype=np.uint32))
    # all distinct values: one word per value in PLWAH
    for n in (1, 31, 32, 500):
        _, _, words = o.wah_index_format(np.arange(n, dtype=np.uint32), FMT_PLWAH)
        assert words.size == n
    # alternating groups of two values: 1-fills of length 1 between 0-fills of length 1
    n = 31 * 6
    v = ((np.arange(n) // 31) % 2).astype(np.uint32)
    _, _, words = o.wah_index_format(v, FMT_CANONICAL)
    exp = [0xC0000001, FILL | 1, 0xC0000001, FILL | 1, 0xC0000001] + [FILL | 1, 0xC0000001] * 3
    np.testing.assert_array_equal(words, np.array(exp, dtype=np.uint32))


def pin_plwah_length_field(o):
    """PLWAH fill lengths have 25 bits: a gap of 2^25 - 1 groups fits, 2^25 is
    refused; canonical WAH takes it (30 bits)."""
    ok = o.wah_encode_groups([1], [(1 << 25) - 1], [1], FMT_PLWAH)[2]
    np.testing.assert_array_equal(ok, np.array([FILL | (1 << 25) | ((1 << 25) - 1)], dtype=np.uint32))
    try:
        o.wah_encode_groups([1], [1 << 25], [1], FMT_PLWAH)
    except RuntimeError:
        pass
    else:
        raise AssertionError("a 2^25-group PLWAH fill was accepted")
    can = o.wah_encode_groups([1], [1 << 25], [1], FMT_CANONICAL)[2]
    np.testing.assert_array_equal(can, np.array([FILL | (1 << 25), 1], dtype=np.uint32))


def pin_lookup(o):
    keys = np.unique(workloads.uniform_values(3, 500, 3000))
    q = np.concatenate([keys[::7], np.array([0, 1, 2999, 3000, 0xFFFFFFFF], dtype=np.uint32),
                        workloads.uniform_values(4, 300, 3100)]).astype(np.uint32)
    got = o.wah_lookup(keys, q)
    pos = {int(k): i for i, k in enumerate(keys)}
    exp = [pos.get(int(x), 0xFFFFFFFF) for x in q]
    np.testing.assert_array_equal(got, np.array(exp, dtype=np.uint32))
    np.testing.assert_array_equal(o.wah_lookup(np.zeros(0, np.uint32), q[:3]), [0xFFFFFFFF] * 3)


def pin_decode_groups(o):
    for fmt in (FMT_PAPER, FMT_CANONICAL, FMT_PLWAH):
        for kind in ("zipf", "all_equal", "alternating_chunks", "sparse_hot", "presorted"):
            n = 2000
            v = workloads.structured(kind, n, seed=11)
            keys, offs, words = o.wah_index_format(v, fmt)
            ng = (n + 30) // 31
            for d in range(0, keys.size, max(1, keys.size // 9)):
                got = o.wah_decode(words[offs[d]:offs[d + 1]], fmt, ng)
                np.testing.assert_array_equal(got, np.array(dense_groups(v == keys[d]), dtype=np.uint32))
    try:
        o.wah_decode(np.array([FILL | 5, 1], np.uint32), FMT_PAPER, 5)
    except RuntimeError:
        pass
    else:
        raise AssertionError("a bitmap longer than ngroups was decoded")


def pin_combine(o):
    """AND / OR of two bitmaps: the decoded result is the bitwise AND / OR of
    the rows, its words are the definition encoding of that row set, and the
    usual identities hold (x AND x = x, x OR x = x, commutativity)."""
    n = 31 * 300 + 11
    ng = (n + 30) // 31
    for kind in ("zipf", "alternating_chunks", "presorted", "sparse_hot"):
        v = workloads.structured(kind, n, seed=21)
        for fmt in (FMT_PAPER, FMT_CANONICAL, FMT_PLWAH):
            keys, offs, words = o.wah_index_format(v, fmt)
            pick = [0, keys.size // 2, keys.size - 1]
            bms = [words[offs[d]:offs[d + 1]] for d in pick]
            rows = [v == keys[d] for d in pick]
            # an OR of several values is a range-like set: many full groups
            for i, j in ((0, 1), (1, 2), (0, 2), (1, 1)):
                for op, f in ((0, np.logical_and), (1, np.logical_or)):
                    for out_fmt in (FMT_PAPER, FMT_CANONICAL, FMT_PLWAH):
                        got = o.wah_combine(bms[i], bms[j], fmt, ng, op, out_fmt)
                        exp = definition_bitmap_words(dense_groups(f(rows[i], rows[j])), out_fmt)
                        np.testing.assert_array_equal(got, np.array(exp, dtype=np.uint32),
                                                      err_msg=f"{kind} fmt={fmt} op={op} out={out_fmt}")
                        sym = o.wah_combine(bms[j], bms[i], fmt, ng, op, out_fmt)
                        np.testing.assert_array_equal(got, sym)
            same = o.wah_combine(bms[0], bms[0], fmt, ng, 0, fmt)
            np.testing.assert_array_equal(same, bms[0])


ALL_PINS = [pin_golden_indexes, pin_golden_fuse_stages, pin_brute_force_small, pin_decode_and_invariants,
            pin_closed_forms, pin_empty, pin_sort_pairs, pin_exclusive_scan, pin_compact, pin_affine,
            pin_stage_composition, pin_golden_formats, pin_formats_brute_force, pin_formats_decode, pin_formats_closed_forms,
            pin_plwah_length_field, pin_lookup, pin_decode_groups, pin_combine]
