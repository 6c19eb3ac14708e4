"""Plant plausible mistakes in copies of the oracle and check that the pins
catch every one of them (the unmodified copy must pass).  Runs on the CPU
only; each variant runs in a child process so a crashing variant cannot take
the test run down."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    ("ceil_to_floor", "(num_lo + d - 1) / d", "(num_lo) / d"),
    ("upper_bound_off_by_one", "((D + eps + 1) * scale - 1) / d", "((D + eps + 1) * scale) / d"),
    ("cap_off_by_one", "if (D + eps + 1 >= cap)", "if (D + eps >= cap)"),
    ("lower_end_tiebreak", "A = lo + (hi - lo) / 2;", "A = lo;"),
    ("upper_end_tiebreak", "A = lo + (hi - lo) / 2;", "A = hi;"),
    ("clamped_midpoint", "    return A < 0 ? 0 : (uint64_t)A;",
     "    if (lo < 0)\n        A = hi / 2;\n    return A < 0 ? 0 : (uint64_t)A;"),
    ("min_slope_of_full_reach", "uint32_t got = cone(k, s, e, eps, F, &lo, &hi);",
     "uint32_t got = cone(k, s, nb, eps, F, &lo, &hi);"),
    ("min_chain_skips_first_anchor", "        uint32_t s = 0;\n        while (reach[s] < bound[m])",
     "        uint32_t s = bound[m] > 1 ? 1 : 0;\n        while (reach[s] < bound[m])"),
    ("min_reach_one_short", "        reach[s] = cone(k, s, nb, eps, F, &lo, &hi);",
     "        reach[s] = cone(k, s, nb, eps, F, &lo, &hi);\n        if (reach[s] > s + 1 && reach[s] < nb) reach[s]--;"),
    ("residual_sign", "u128 code = (uint64_t)(key + eps - pred);", "u128 code = (uint64_t)(pred + eps - key);"),
    ("offset_dropped", "(u128)(j - starts[base + t])", "(u128)(j)"),
    ("decoder_search", "if (get_le(st + 2ull * u, 2) <= j)", "if (get_le(st + 2ull * u, 2) < j)"),
    ("bit_order", "slab[p / 8] |= (uint8_t)(1u << (p % 8));", "slab[p / 8] |= (uint8_t)(1u << (7 - p % 8));"),
    ("anchor_not_relative", "put_le(sa + (uint64_t)ab * u, anchors[base + u] - first, ab);",
     "put_le(sa + (uint64_t)ab * u, anchors[base + u], ab);"),
    ("width_off_by_one", "while ((1ull << w) < values)", "while ((1ull << w) <= values)"),
    ("byte_width_step", "if (v < (1ull << 8)) return 1;", "if (v <= (1ull << 8)) return 1;"),
    ("delta_transposed", "i128 D = (i128)k[e] - (i128)anchor;", "i128 D = (i128)anchor - (i128)k[e];"),
    ("stride_unaligned", "const uint64_t res_stride = align16((B * (uint64_t)w + 7) / 8);",
     "const uint64_t res_stride = (B * (uint64_t)w + 7) / 8;"),
    ("dir_count", "put_le(d + 12, nb - 1, 2);", "put_le(d + 12, nb, 2);"),
    ("opt_start_not_raised", "#define LO(i) ((i) == s ? ((i128)k[s] - E > first ? (i128)k[s] - E : first) * scale",
     "#define LO(i) ((i) == s ? ((i128)k[s] - E) * scale"),
    ("opt_ceil_as_floor", "i128 l = ceil_div(LO(e) - UP(i), (i128)(e - i));",
     "i128 l = floor_div(LO(e) - UP(i), (i128)(e - i));"),
    ("opt_pairs_with_start_only", "            for (uint32_t i = s; i < e; i++) {\n                i128 l = ceil_div",
     "            for (uint32_t i = s; i < s + 1; i++) {\n                i128 l = ceil_div"),
    ("opt_cap_eps_once", "if ((i128)k[e] - (i128)k[s] + 2 * E + 1 >= cap)", "if ((i128)k[e] - (i128)k[s] + E + 1 >= cap)"),
    ("opt_intercept_low_end", "i128 C = g + (h - g) / 2;", "i128 C = g;"),
    ("opt_slope_low_end", "i128 A = e > s + 1 ? lo + (hi - lo) / 2 : 0;", "i128 A = e > s + 1 ? lo : 0;"),
    ("opt_fraction_dropped", "(((u128)slopes[base + t] * (u128)(j - starts[base + t]) + fracs[base + t]) >> F)",
     "(((u128)slopes[base + t] * (u128)(j - starts[base + t])) >> F)"),
    ("opt_fraction_width", "static int frac_bytes(uint32_t F) { return F == 0 ? 0 : F <= 8 ? 1 : F <= 16 ? 2 : 4; }",
     "static int frac_bytes(uint32_t F) { return F == 0 ? 0 : F <= 8 ? 1 : 4; }"),
]

RUNNER = (
    "import sys; sys.path[:0] = [{root!r}, {tests!r}]\n"
    "import oracle, oracle_pins\n"
    "bad = oracle_pins.run_quick(oracle.Ref({lib!r}))\n"
    "print(bad or 'all-pass'); sys.exit(1 if bad else 0)\n"
)


def _variant(tmp_path, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "lcref.c")).read()
    if old is not None:
        assert src.count(old) == 1, f"mutation site for {name} not unique/found"
        src = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    c.write_text(src)
    lib = str(tmp_path / f"lib{name}.so")
    oracle.build(force=True, src=str(c), out=lib)
    code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
    return subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)


def test_unmodified_copy_passes(tmp_path):
    r = _variant(tmp_path, "unmodified", None, None)
    assert r.returncode == 0, r.stdout + r.stderr


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    r = _variant(tmp_path, name, old, new)
    assert r.returncode != 0, f"mutant {name} passed every pin"
    print(name, "caught by", r.stdout.strip() or r.returncode)
