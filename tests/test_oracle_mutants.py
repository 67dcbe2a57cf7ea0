"""The pins have teeth: each plausible mistake planted in a copy of the oracle
(on the CPU) makes at least one pin fail."""
import os
import subprocess
import tempfile

import pytest

import oracle
from oracle.build import SRC
from oracle_pins import ALL_PINS

# (name, original text, mutated text): dropped terms, wrong signs or indexes,
# transposed operands, wrong constants.
MUTANTS = [
    ("gap_off_by_one", "gchunk[g]) - prev - 1;", "gchunk[g]) - prev;"),
    ("msb_first_bits", "1u << (srows[i] % kGroupRows)", "1u << (30 - srows[i] % kGroupRows)"),
    ("group_of_32_rows", "kGroupRows = 31;", "kGroupRows = 32;"),
    ("unstable_ties", "return keys[a] < keys[b];", "return keys[a] < keys[b] || (keys[a] == keys[b] && a > b);"),
    ("leading_fill_from_0", "first_of_value ? -1 :", "first_of_value ? 0 :"),
    ("fill_across_values", "(g == 0) || gkey[g - 1] != gkey[g];", "(g == 0);"),
    ("keep_trailing_zero", "if (in[i] != 0) out[w++]", "if (in[i] != 0 || i + 1 == m) out[w++]"),
    ("inclusive_scan", "out[i] = acc;\n    acc += v;", "acc += v;\n    out[i] = acc;"),
    ("offsets_plus_one", "offsets[d] = static_cast<uint32_t>(kept);\n      ++d;",
     "offsets[d] = static_cast<uint32_t>(kept + 1);\n      ++d;"),
    ("affine_transposed", "a[s] * x[i] + b[s]", "a[s] * (x[i] + b[s])"),
    ("literal_before_fill", "index[2 * g] = gfill[g];\n    index[2 * g + 1] = glit[g];",
     "index[2 * g] = glit[g];\n    index[2 * g + 1] = gfill[g];"),
    ("one_fill_flag", "kFillFlag = 0x80000000u;", "kFillFlag = 0xC0000000u;"),
    ("chunks_merged", "gkey[g - 1] == skeys[i] && gchunk[g - 1] == chunk", "gkey[g - 1] == skeys[i]"),
    ("rows_are_ranks", ": static_cast<uint32_t>(perm[j]);", ": static_cast<uint32_t>(j);"),
    ("table_counts_zeros", "kept += (index[2 * g] != 0) + (index[2 * g + 1] != 0);", "kept += 2;"),
    ("groups_by_key_only_in_literal", "glit[g - 1] |= bit;", "glit[g - 1] = bit;"),
    # encoder formats and the query path
    ("one_fill_without_fill_bit", "kFillFlag | (one ? kOneFill : 0u)", "kFillFlag | (one ? 0u : 0u)"),
    ("full_run_ignores_adjacency", "c[i + run] == c[i] + run && lit[i + run] == kFull",
     "lit[i + run] == kFull"),
    ("one_fold_position_no_plus_one", "p = 1 + odd_bit(lit[nx], true);", "p = odd_bit(lit[nx], true);"),
    ("zero_fold_any_small_literal", "gap > 0 && popcount31(lit[i]) == 1", "gap > 0 && popcount31(lit[i]) <= 2"),
    ("fold_keeps_literal_group", "prev = static_cast<int64_t>(c[i] + run - 1) + (p ? 1 : 0);",
     "prev = static_cast<int64_t>(c[i] + run - 1);"),
    ("plwah_30_bit_lengths", "format == kFormatPlwah ? kPlwahMaxLen : kMaxFillLen;\n  if (len > lim)",
     "kMaxFillLen;\n  if (len > lim)"),
    ("fold_after_one_fill_of_29", "popcount31(lit[nx]) == 30", "popcount31(lit[nx]) >= 29"),
    ("decode_position_off_by_one", "one ? (kFull & ~(1u << (p - 1))) : (1u << (p - 1))",
     "one ? (kFull & ~(1u << p)) : (1u << p)"),
    ("lookup_insertion_point", "(p != keys + D && *p == queries[i]) ?", "(p != keys + D) ?"),
    ("combine_or_as_and", "op == 0 ? (ga[g] & gb[g]) : (ga[g] | gb[g])", "(ga[g] & gb[g])"),
    ("canonical_keeps_full_literals", "if (format != kFormatPaper && lit[i] == kFull) {",
     "if (format == kFormatPlwah && lit[i] == kFull) {"),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, name, orig, mut, tmp_path):
    assert source.count(orig) == 1, f"mutation anchor for {name} not unique/found"
    src = tmp_path / "mutant.cpp"
    src.write_text(source.replace(orig, mut))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(src), "-o", str(lib)], check=True)
    o = oracle.Oracle(str(lib))
    failed = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except (AssertionError, RuntimeError) as e:  # RuntimeError: oracle reported an error
            failed.append(pin.__name__)
            break
    assert failed, f"no pin catches mutant {name}"
