"""Plants plausible mistakes in copies of the oracle (on the CPU) and checks
that the pins catch every one.  Each mutant runs in its own process, since a
wrong index may crash instead of giving a wrong value."""
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, text in oracle.c, replacement, which occurrence: 0 first, -1 last)
MUTANTS = [
    ("min_becomes_max", "if (a < b) return a;\n  if (b < a) return b;",
     "if (a < b) return b;\n  if (b < a) return a;", 0),
    ("int64_times_becomes_plus", "r = a * b;", "r = a + b;", 0),
    ("fp64_times_becomes_plus", "r = a * b;", "r = a + b;", -1),
    ("fp64_plus_becomes_minus", "r = a + b;\n    memcpy(dst, &r, 8);\n  }\n}",
     "r = a - b;\n    memcpy(dst, &r, 8);\n  }\n}", 0),
    ("dropped_first_term", "for (int64_t ea = arp[i]; ea", "for (int64_t ea = arp[i] + 1; ea", 0),
    ("wrong_inner_row", "for (int64_t eb = brp[k]; eb < brp[k + 1]; ++eb)",
     "for (int64_t eb = brp[k % (i + 1)]; eb < brp[k % (i + 1) + 1]; ++eb)", 0),
    ("operands_swapped", "i, arp, aci, (const char*)av, brp, bci,\n                                   (const char*)bv",
     "i, brp, bci, (const char*)bv, arp, aci,\n                                   (const char*)av", 0),
    ("first_product_from_zero", "memcpy(slot, p, (size_t)vs);",
     "memset(slot, 0, (size_t)vs); sr_add(sr, slot, slot, p);", 0),
    ("rows_not_sorted", "qsort(s->touched", "if (0) qsort(s->touched", 0),
    ("delete_ignored", "if (present) {\n          memmove(wc + pos, wc + pos + 1",
     "if (0) {\n          memmove(wc + pos, wc + pos + 1", 0),
    ("add_overwrites", "if (bop[t] == ORC_OP_SET) memcpy(", "if (1) memcpy(", 0),
    ("batch_order_reversed", "int64_t t = order[u];", "int64_t t = order[first[i] + first[i + 1] - 1 - u];", 0),
    ("changed_means_length_change", "changed[i] = (uint8_t)diff;", "changed[i] = (uint8_t)(len != len0);", 0),
    ("bool_or_becomes_xor", "r = a | b;", "r = a ^ b;", 0),
    ("bool_and_becomes_or", "r = a & b;", "r = a | b;", 0),
    ("bool_words_truncated", "case ORC_OR_AND_U32: return 4;", "case ORC_OR_AND_U32: return 2;", 0),
    ("transpose_keeps_column", "tci[o] = i;", "tci[o] = ci[e];", 0),
    ("transpose_rows_reversed", "for (int32_t i = 0; i < nrows; ++i) {\n    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {\n      int64_t o",
     "for (int32_t i = nrows - 1; i >= 0; --i) {\n    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {\n      int64_t o", 0),
    ("transpose_value_shifted", "(const char*)v + (size_t)vs * (size_t)e, (size_t)vs);",
     "(const char*)v + (size_t)vs * (size_t)(e > 0 ? e - 1 : 0), (size_t)vs);", 0),
    ("axpby_beta_ignored", "sr_mul(sr, t2, beta, (const char*)xv + (size_t)vs * (size_t)b);",
     "memcpy(t2, (const char*)xv + (size_t)vs * (size_t)b, (size_t)vs);", 0),
    ("axpby_overlap_keeps_c", "sr_add(sr, d, t1, t2);", "memcpy(d, t1, (size_t)vs);", 0),
    ("axpby_x_only_scaled_by_alpha", "sr_mul(sr, d, beta,", "sr_mul(sr, d, alpha,", 0),
    ("axpby_x_only_dropped", "        dci[out] = xci[b];\n        ++b;\n      }\n      ++out;",
     "        dci[out] = xci[b];\n        ++b;\n        continue;\n      }\n      ++out;", 0),
    ("bloom_bits_mod_32", "((uint32_t)k % ORC_BLOOM_L)", "((uint32_t)k % 32)", 0),
    ("pattern_without_a_bstar", "if (mark[j] != i) { mark[j] = i; touched[nt++] = j; }\n      }\n    }\n    /* A' B*",
     "(void)j;\n      }\n    }\n    /* A' B*", 0),
    ("filter_ignores_fstar", "uint64_t x = fs[e];", "uint64_t x = 0; (void)fs;", 0),
    ("filter_and_instead_of_or", "acc |= x;", "acc &= x;", 0),
    ("masked_merge_keeps_deleted", "if (zp[b]) src = (const char*)zv + (size_t)vs * (size_t)b;",
     "src = zp[b] ? (const char*)zv + (size_t)vs * (size_t)b\n                    : (a < xrp[i + 1] && xci[a] == j) ? (const char*)xv + (size_t)vs * (size_t)a : NULL;", 0),
    ("changed_ignores_values", "(size_t)vs) != 0;\n        ++a; ++b;", "(size_t)vs) != 0 && 0;\n        ++a; ++b;", 0),
]


def _mutate(src, old, new, which):
    if which == 0:
        pos = src.find(old)
    else:
        pos = src.rfind(old)
    assert pos >= 0, old
    return src[:pos] + new + src[pos + len(old):]


@pytest.mark.parametrize("name,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, old, new, which):
    src = open(os.path.join(oracle.HERE, "oracle.c")).read()
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "oracle.c"), "w").write(_mutate(src, old, new, which))
        open(os.path.join(d, "oracle.h"), "w").write(open(os.path.join(oracle.HERE, "oracle.h")).read())
        so = oracle.build(os.path.join(d, "libmut.so"), d)
        code = ("import sys; sys.path[:0] = [%r, %r]\n"
                "import oracle, pins\n"
                "L = oracle.lib(%r)\n"
                "for p in pins.ALL_PINS:\n"
                "    try:\n"
                "        p(L)\n"
                "    except AssertionError:\n"
                "        print('caught by', p.__name__); sys.exit(3)\n"
                "sys.exit(0)\n") % (ROOT, os.path.join(ROOT, "tests"), so)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
        assert r.returncode != 0, f"mutant {name} passed every pin"
