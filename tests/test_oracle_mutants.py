"""Plant plausible mistakes in copies of the oracle (on the CPU) and check
that the pins reject every one of them: a dropped term, a wrong index, a
wrong comparison, a transposed operand."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "d4_stride": ("default: return i >= 4 ? x[i - 4] : 0u;", "default: return i >= 4 ? x[i - 3] : 0u;"),
    "d1_stride": ("case ORC_D1: return i >= 1 ? x[i - 1] : 0u;", "case ORC_D1: return i >= 2 ? x[i - 2] : 0u;"),
    "d2_stride": ("case ORC_D2: return i >= 2 ? x[i - 2] : 0u;", "case ORC_D2: return i >= 1 ? x[i - 1] : 0u;"),
    "dm_reference": ("return q >= 1 ? x[4u * q - 1u] : 0u;", "return q >= 1 ? x[4u * q - 2u] : 0u;"),
    "inverse_dropped": ("out[i] += orc_reference(out, i, mode);", "out[i] += orc_reference(out, i, ORC_D4);"),
    "d2_steps": ("u[2] = t[2] + t[0]; u[3] = t[3] + t[1];\n      t[0] = u[0] + v[2];",
                 "u[2] = t[2] + t[1]; u[3] = t[3] + t[1];\n      t[0] = u[0] + v[2];"),
    "d1_steps": ("t[0] = u[0]; t[1] = u[1] + u[0]; t[2] = u[2] + u[1]; t[3] = u[3] + u[2];",
                 "t[0] = u[0]; t[1] = u[1] + u[0]; t[2] = u[2] + u[0]; t[3] = u[3] + u[2];"),
    "dm_steps": ("for (int c = 0; c < 4; ++c) t[c] += v[3];\n      break;\n    case ORC_D2:",
                 "for (int c = 0; c < 4; ++c) t[c] += v[c];\n      break;\n    case ORC_D2:"),
    "lane_word_index": ("get32(w + 4u * (4u * m + j))", "get32(w + 4u * (4u * j + m))"),
    "width_compare": ("(uint64_t)d[i] >= ((uint64_t)1 << b)", "(uint64_t)d[i] > ((uint64_t)1 << b)"),
    "width_drops_last": ("orc_width(d + 128u * k, 128u)", "orc_width(d + 128u * k, 127u)"),
    "pack_lane_order": ("d[128u * k + 4u * q + j]", "d[128u * k + 32u * j + q]"),
    "merge_advance": ("else if (b[j] < a[i]) ++j;", "else if (b[j] < a[i]) ++i;"),
    "alg1_straddle_shift": ("<< (32u - i)) & M;", "<< (31u - i)) & M;"),
    "alg1_dropped_prefix": ("default: /* D4: t + v */\n      for (int c = 0; c < 4; ++c) t[c] += v[c];",
                            "default: /* D4: t + v */\n      for (int c = 0; c < 4; ++c) t[c] += 0;"),
    "b32_mask": ("uint64_t mask = (b == 32u) ? 0xFFFFFFFFull", "uint64_t mask = (b == 32u) ? 0x7FFFFFFFull"),
    "tail_offset": ("out[128u * v.nb + i] = get32(v.tail + 4u * i);\n  return ORC_OK;\n}\n\n/* The vector",
                    "out[128u * v.nb + i] = get32(v.tail);\n  return ORC_OK;\n}\n\n/* The vector"),
    "extract_shift": ("return (uint32_t)((window >> s) & mask);", "return (uint32_t)((window >> (s + 1)) & mask);"),
    "fp_tie_smaller": ("if (k == 0 || cost < best) { best = cost;", "if (k == 0 || cost <= best) { best = cost;"),
    "fp_cost_seven": ("(uint64_t)c * (b - bp + 8u);", "(uint64_t)c * (b - bp + 7u);"),
    "fp_exception_strict": ("if ((uint64_t)d[i] >= ((uint64_t)1 << bp)) ++c;", "if ((uint64_t)d[i] > ((uint64_t)1 << bp)) ++c;"),
    "fp_patch_shift": ("out[128u * k + m[o + e]] += (uint32_t)((uint64_t)high << bp);",
                       "out[128u * k + m[o + e]] += (uint32_t)((uint64_t)high << (bp + 1u));"),
    "fp_page_256": ("#define ORC_PAGE 512u", "#define ORC_PAGE 256u"),
    "fp_reader_drift": ("  r->have -= d;\n", "  r->have -= d - (d > 1u);\n"),
    "fp_array_pad": ("if (cnt[e]) pages += 4u + 4u * (size_t)e * ((cnt[e] + 31u) / 32u);",
                     "if (cnt[e]) pages += 4u + 4u * (size_t)e * ((cnt[e] + 127u) / 128u) * 4u;"),
    "hyb_rule_strict": ("return n >= (universe + B - 1u) / B;", "return n > (universe + B - 1u) / B;"),
    "hyb_rule_floor": ("return n >= (universe + B - 1u) / B;", "return n >= universe / B;"),
    "hyb_probe_msb_first": ("((bits[j][x / 32u] >> (x % 32u)) & 1u)", "((bits[j][x / 32u] >> (31u - x % 32u)) & 1u)"),
    "hyb_first_bitmap_skipped": ("for (uint32_t j = 0; j < nbm; ++j) {\n      uint64_t c = 0;",
                                 "for (uint32_t j = 1; j < nbm; ++j) {\n      uint64_t c = 0;"),
    "hyb_and_drops_one": ("for (uint32_t j = 1; j < nbm; ++j) a &= bits[j][w];",
                          "for (uint32_t j = 2; j < nbm; ++j) a &= bits[j][w];"),
    "hyb_extract_offset": ("out[cur++] = (uint32_t)(32u * w + b);", "out[cur++] = (uint32_t)(32u * w + 31u - b);"),
}


def battery():
    """Run the pins; return the names of those that failed."""
    failed = []
    checks = [
        ("fig1c", pins.test_fig1c_bytes_are_one_lane_stream),
        ("fig2", pins.test_fig2_interleaved_layout),
        ("b32", pins.test_b32_block_is_raw_words),
        ("b0", pins.test_b0_block_repeats_seed),
        ("mixed", pins.test_mixed_widths_all_values),
        ("width_floor", pins.test_width_floor_strictly_increasing),
        ("plain_pair", pins.test_intersect_matches_numpy_set_routine),
        ("k_invariants", pins.test_intersect_k_invariants),
        ("random_subsets", pins.test_intersect_random_subsets_of_12),
    ]
    for b in (0, 1, 7, 18, 31, 32):
        checks.append((f"alg1_b{b}", lambda b=b: pins.test_random_access_matches_alg1_walk(b)))
        checks.append((f"round_trip_b{b}", lambda b=b: pins.test_round_trip_per_width(b)))
    for n in (129, 2049):
        checks.append((f"edge_{n}", lambda n=n: pins.test_round_trip_edge_lengths(n)))
    for s in range(2):
        checks.append((f"formula_{s}", lambda s=s: pins.test_bits_per_block_formula_and_widths(s)))
    checks.append(("ap", lambda: pins.test_arithmetic_progression_closed_form(7, 3)))
    for p in (0, 127):
        checks.append((f"jump_{p}", lambda p=p: pins.test_width_reaches_every_position(p)))
    checks.append(("sec5_steps", pins.test_sec5_worked_prefix_steps))
    checks.append(("table3", pins.test_table3_relative_delta_sizes))
    checks.append(("modes_ap", lambda: pins.test_modes_arithmetic_progression_widths(7, 3)))
    for name in pins.MODES:
        checks.append((f"modes_alg1_{name}", lambda n=name: pins.test_modes_random_access_matches_alg1_walk(n, 17)))
        checks.append((f"modes_rt_{name}", lambda n=name: pins.test_modes_round_trip(n, 2049)))
    checks.append(("fig3_choice", pins.test_fig3_fastpfor_choice))
    checks.append(("fig3_bytes", pins.test_fig3_fastpfor_stream_bytes))
    checks.append(("fp_tie", pins.test_fastpfor_tie_goes_to_larger_width))
    for i, (blk, want) in enumerate([([5] * 128, (3, 3, 0)), ([0] * 127 + [1 << 31], (32, 0, 1)),
                                     ([7] * 120 + [1 << 20] * 8, (21, 3, 8))]):
        checks.append((f"fp_hand_{i}", lambda blk=blk, want=want: pins.test_fastpfor_choice_by_hand(blk, want)))
    for mode in (pins.oracle.D4, pins.oracle.D1):
        checks.append((f"fp_pages_{mode}", lambda m=mode: pins.test_fastpfor_stream_size_and_pages(m, 128 * 700)))
    rule_cases = [(128, 1024, 8, True), (127, 1024, 8, False), (32, 1000, 32, True), (31, 1000, 32, False),
                  (5, 41, 8, False)]
    checks.append(("hyb_rule", lambda: [pins.test_hyb_bitmap_rule(*c) for c in rule_cases]))
    checks.append(("hyb_hand", pins.test_hyb_all_bitmaps_and_mixed_by_hand))
    for sd in range(12):
        checks.append((f"hyb_sets_{sd}", lambda sd=sd: pins.test_hyb_equals_set_intersection(sd)))
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, oracle.OracleError, ValueError, IndexError):
            failed.append(name)
    return failed


def test_unmutated_oracle_passes_battery():
    assert battery() == []


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / f"lib{name}.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(path)])
    with oracle.use_variant(str(so)):
        failed = battery()
    assert failed, f"mutant {name} survived every pin"
