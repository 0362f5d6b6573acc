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
    # encoding: group value, 6-bit fields, padding
    "enc_field_mask": ("return (v >> (18 - 6 * k)) & 63u;", "return (v >> (18 - 6 * k)) & 31u;"),
    "enc_field_shift": ("return (v >> (18 - 6 * k)) & 63u;", "return (v >> (18 - 5 * k)) & 63u;"),
    "enc_group_little_endian": ("v = (v << 8) | (k < avail ? s[k] : 0u);",
                                "v = (v >> 8) | ((k < avail ? s[k] : 0u) << 16);"),
    "enc_drop_third_byte": ("for (int k = 0; k < 3; k++) v = (v << 8)", "for (int k = 0; k < 2; k++) v = (v << 8)"),
    "enc_missing_bytes_not_zero": ("(k < avail ? s[k] : 0u)", "(k < avail ? s[k] : 0xffu)"),
    "table_swap_62_63": ('"+/";', '"/+";'),
    "url_swap": ("if (v == 62) return (uint8_t)'-';", "if (v == 62) return (uint8_t)'_';"),
    "drop_one_pad": ("p[o++] = k <= avail ?", "p[o++] = k <= avail + 1 ?"),
    "one_field_short": ("p[o++] = k <= avail ?", "p[o++] = k < avail ?"),
    # decoding: group value, byte order, padding, validation
    "dec_field_shift": ("v = (v << 6) | (c[i + k] == '='", "v = (v << 5) | (c[i + k] == '='"),
    "dec_bytes_little_endian": ("for (int k = 0; k < 3; k++) p[o++] = (uint8_t)(v >> (16 - 8 * k));",
                                "for (int k = 0; k < 3; k++) p[o++] = (uint8_t)(v >> (8 * k));"),
    "dec_pads_not_dropped": ("return oracle_decode_quads(c, 0, n, p, inv) - oracle_pads(c, n);",
                             "return oracle_decode_quads(c, 0, n, p, inv);"),
    "pad_slot2_relaxed": ("if (i == n - 2 && c[n - 1] == '=') return 1;", "if (i == n - 2) return 1;"),
    "no_length_check": ("if (bad < 0 && n % 4 != 0) bad = n;\n    if (bad >= 0) {\n        *err_off",
                        "if (bad >= 0) {\n        *err_off"),
    "offset_off_by_one": ("if (!oracle_char_ok(c, n, i, inv)) return i;",
                          "if (!oracle_char_ok(c, n, i, inv)) return i + 1;"),
    # whitespace-tolerant decode (Appendix B)
    "ws_also_tab": ("if (v == ' ' || v == '\\n' || v == '\\r') continue;",
                    "if (v == ' ' || v == '\\n' || v == '\\r' || v == '\\t') continue;"),
    "ws_no_cr": ("if (v == ' ' || v == '\\n' || v == '\\r') continue;", "if (v == ' ' || v == '\\n') continue;"),
    "ws_stripped_offsets": ("if (len < 0) *err_off = (*err_off >= m) ? n : pos[*err_off];",
                            "if (len < 0) *err_off = (*err_off >= m) ? n : *err_off;"),
    "ws_length_error_at_m": ("if (len < 0) *err_off = (*err_off >= m) ? n : pos[*err_off];",
                             "if (len < 0) *err_off = (*err_off >= m) ? m : pos[*err_off];"),
    # Appendix A strict checks and the unpadded mode
    "strict_two_pad_bits": ("(inv[c[n - 3]] & 15) != 0", "(inv[c[n - 3]] & 3) != 0"),
    "strict_one_pad_bits": ("(inv[c[n - 2]] & 3) != 0", "(inv[c[n - 2]] & 15) != 0"),
    "nopad_accepts_len_mod4_1": ("    if (bad < 0 && n % 4 == 1) bad = n;\n    if (bad >= 0) { *err_off = bad; return -1; }",
                                 "    if (bad >= 0) { *err_off = bad; return -1; }"),
    "nopad_tail_one_byte_short": ("for (int64_t k = 0; k < r - 1; k++) p[o++]", "for (int64_t k = 0; k < r - 2; k++) p[o++]"),
    # batch loops (packed and gather forms)
    "batch_encode_ignores_flags": ("in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD);",
                                   "in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   ORACLE_STD);"),
    "batch_decode_ignores_flags": ("in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD, &err_off[i]);",
                                   "in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   ORACLE_STD, &err_off[i]);"),
    "batch_output_at_input_offset": ("in_off[i + 1] - in_off[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD);",
                                     "in_off[i + 1] - in_off[i], dst + in_off[i],\n                                   flags ? flags[i] : ORACLE_STD);"),
    "gather_encode_ignores_flags": ("in_len[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD);",
                                    "in_len[i], dst + out_off[i],\n                                   ORACLE_STD);"),
    "gather_decode_ignores_flags": ("in_len[i], dst + out_off[i],\n                                   flags ? flags[i] : ORACLE_STD, &err_off[i]);",
                                    "in_len[i], dst + out_off[i],\n                                   ORACLE_STD, &err_off[i]);"),
    "gather_encode_drops_last_byte": ("oracle_encode(src + in_begin[i], in_len[i],",
                                      "oracle_encode(src + in_begin[i], in_len[i] - (in_len[i] > 0),"),
    "gather_decode_at_packed_offset": ("oracle_decode(src + in_begin[i], in_len[i],",
                                       "oracle_decode(src + in_begin[0] + i, in_len[i],"),
    "mt_batch_range_skips_message": ("        w[t].begin = i;\n", "        w[t].begin = i + (t == 1 && i < N);\n"),
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
    lambda t1: pins.test_gather_forms_equal_single_calls(),
    lambda t1: pins.test_multithreaded_batch_wrappers_equal_plain(),
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
