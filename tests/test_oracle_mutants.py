"""Planted mistakes in a copy of the oracle must each fail some pin.

Every mutant is a plausible slip (a wrong shift, a dropped term, a swapped
symbol, a relaxed padding rule, an off-by-one offset). The oracle source is
copied to a temporary directory, edited there and compiled with gcc; the
checked-in oracle is never modified.
"""
import os

import pytest

import oracle
from oracle import build as obuild
import test_oracle as pins

MUTANTS = {
    "enc_second_shift": ("(s[i + 1] / 16));\n        p[o++] = oracle_B(alphabet, ((s[i + 1] * 4)",
                         "(s[i + 1] / 8));\n        p[o++] = oracle_B(alphabet, ((s[i + 1] * 4)"),
    "enc_drop_third_term": ("+ (s[i + 2] / 64));", ");"),
    "table_swap_62_63": ('"+/";', '"/+";'),
    "url_swap": ("if (v == 62) return (uint8_t)'-';", "if (v == 62) return (uint8_t)'_';"),
    "tail1_shift": ("p[o++] = oracle_B(alphabet, (s[i] * 16) % 64);",
                    "p[o++] = oracle_B(alphabet, (s[i] * 4) % 64);"),
    "drop_one_pad": ("        }\n        p[o++] = '=';\n    }\n    return o;", "        }\n    }\n    return o;"),
    "dec_first_byte": ("(uint8_t)((a * 4) + (b / 16));\n        if (c[i + 2]",
                       "(uint8_t)((a * 4) + (b / 8));\n        if (c[i + 2]"),
    "dec_third_byte": ("(uint8_t)(((cc * 64) % 256) + d);\n    }", "(uint8_t)(((cc * 16) % 256) + d);\n    }"),
    "pad_slot2_relaxed": ("if (i == n - 2 && c[n - 1] == '=') return 1;", "if (i == n - 2) return 1;"),
    "no_length_check": ("if (bad < 0 && n % 4 != 0) bad = n;\n    if (bad >= 0) {\n        *err_off",
                        "if (bad >= 0) {\n        *err_off"),
    "offset_off_by_one": ("if (!oracle_char_ok(c, n, i, inv)) return i;",
                          "if (!oracle_char_ok(c, n, i, inv)) return i + 1;"),
    "dec_no_early_stop": ("        if (c[i + 2] == '=') return o;\n", ""),
    # whitespace-tolerant decode (Appendix B)
    "ws_also_tab": ("if (v == ' ' || v == '\\n' || v == '\\r') continue;",
                    "if (v == ' ' || v == '\\n' || v == '\\r' || v == '\\t') continue;"),
    "ws_no_cr": ("if (v == ' ' || v == '\\n' || v == '\\r') continue;", "if (v == ' ' || v == '\\n') continue;"),
    "ws_stripped_offsets": ("if (len < 0) *err_off = (*err_off >= m) ? n : pos[*err_off];",
                            "if (len < 0) *err_off = (*err_off >= m) ? n : *err_off;"),
    "ws_length_error_at_m": ("if (len < 0) *err_off = (*err_off >= m) ? n : pos[*err_off];",
                             "if (len < 0) *err_off = (*err_off >= m) ? m : pos[*err_off];"),
    # Appendix A strict checks and the unpadded mode
    "strict_two_pad_bits": ("if ((inv[c[n - 3]] * 16) % 256 != 0)", "if ((inv[c[n - 3]] * 64) % 256 != 0)"),
    "strict_one_pad_bits": ("if ((inv[c[n - 2]] * 64) % 256 != 0)", "if ((inv[c[n - 2]] * 16) % 256 != 0)"),
    "nopad_accepts_len_mod4_1": ("    if (bad < 0 && n % 4 == 1) bad = n;\n    if (bad >= 0) { *err_off = bad; return -1; }",
                                 "    if (bad >= 0) { *err_off = bad; return -1; }"),
    "nopad_second_byte": ("p[o++] = (uint8_t)(((b * 16) % 256) + (cc / 4));\n        }\n    }\n    return o;",
                          "p[o++] = (uint8_t)(((b * 16) % 256) + (cc / 2));\n        }\n    }\n    return o;"),
    # batch loops
    "batch_encode_ignores_flags": ("dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD);",
                                   "dst + out_off[i],\n                                   ORACLE_STD);"),
    "batch_decode_ignores_flags": ("flags ? flags[i] : ORACLE_STD, &err_off[i]);", "ORACLE_STD, &err_off[i]);"),
    "batch_output_at_input_offset": ("in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD);",
                                     "in_off[i + 1] - in_off[i], dst + in_off[i],\n                                   flags ? flags[i] : ORACLE_STD);"),
}

PIN_TESTS = [
    lambda t1: pins.test_table1_alphabet(t1),
    lambda t1: pins.test_base64url_variant(t1),
    lambda t1: pins.test_example_encode_R0lG(),
    lambda t1: pins.test_example_decode_gif(),
    lambda t1: pins.test_appendix_c_example(),
    lambda t1: pins.test_standard_examples_named_for_this_codec(),
    lambda t1: pins.test_length_law(),
    lambda t1: pins.test_padding_readings(),
    lambda t1: pins.test_rejection_sweep_all_256_bytes(t1, oracle.STD),
    lambda t1: pins.test_rejection_sweep_all_256_bytes(t1, oracle.URL),
    lambda t1: pins.test_all_one_and_two_byte_tails(t1, oracle.URL),
    lambda t1: pins.test_single_injected_offset_is_exact(),
    lambda t1: pins.test_whitespace_strip_and_decode(),
    lambda t1: pins.test_whitespace_mode_classifies_every_byte_value(),
    lambda t1: pins.test_appendix_a_strict_checks(),
    lambda t1: pins.test_appendix_a_strict_accepts_exactly_the_canonical_texts(t1, oracle.STD),
    lambda t1: pins.test_nopad_variants(),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, table1):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "b64_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    so = obuild.build(out=str(tmp_path / "liboracle_mut.so"), src=str(mut),
                      extra_flags=["-Wno-unused-variable", "-Wno-unused-but-set-variable"])
    caught = []
    with oracle.using(so):
        for k, t in enumerate(PIN_TESTS):
            try:
                t(table1)
            except AssertionError:
                caught.append(k)
    assert caught, f"no pin caught mutant {name}"


def test_unmutated_copy_passes_all_pins(tmp_path, table1):
    so = obuild.build(out=str(tmp_path / "liboracle_copy.so"))
    with oracle.using(so):
        for t in PIN_TESTS:
            t(table1)
    assert os.path.exists(so)
