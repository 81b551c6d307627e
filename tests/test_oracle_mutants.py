"""Every plausible mistake planted in the oracle must trip at least one pin.

Each case copies ``oracle/aes_oracle.c``, applies one textual change (a wrong
polynomial, a transposed operand, a wrong index or shift direction, a dropped
term, ...), compiles the copy into a temporary directory with gcc and runs the
whole pin suite of ``oracle_pins.py`` on it.  The committed oracle is never
modified.  A mutant that passes every pin would mean the pins cannot tell a
broken oracle from the real one.
"""
import os

import pytest

import oracle_pins
from oracle import oracle as oracle_mod

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "oracle", "aes_oracle.c")

MUTANTS = [
    # GF(2^8)
    ("wrong_polynomial", "#define AES_POLY 0x11Bu", "#define AES_POLY 0x11Du"),
    ("mul_uses_a_bits", "if (b & (1u << i))", "if (a & (1u << i))"),
    ("no_reduction", "if (term & 0x100u)\n            term ^= AES_POLY;",
     "if (term & 0x200u)\n            term ^= AES_POLY;"),
    ("inverse_exponent", "oracle_gf_pow(a, 254u)", "oracle_gf_pow(a, 253u)"),
    # affine maps
    ("affine_transposed", "s ^= row[(j - i + 8) % 8] & v[j];",
     "s ^= row[(i - j + 8) % 8] & v[j];"),
    ("affine_lsb_first", "v[k] = (x >> (7 - k)) & 1;", "v[k] = (x >> k) & 1;"),
    ("affine_constant", "SBOX_B[8]   = {0, 1, 1, 0, 0, 0, 1, 1}",
     "SBOX_B[8]   = {1, 1, 0, 0, 0, 1, 1, 0}"),
    ("affine_row", "SBOX_ROW[8] = {1, 1, 1, 1, 1, 0, 0, 0}",
     "SBOX_ROW[8] = {1, 1, 1, 1, 0, 0, 0, 1}"),
    ("inv_affine_constant", "INV_B[8]    = {0, 0, 0, 0, 0, 1, 0, 1}",
     "INV_B[8]    = {0, 0, 0, 0, 0, 1, 1, 0}"),
    ("inv_affine_row", "INV_ROW[8]  = {0, 1, 0, 1, 0, 0, 1, 0}",
     "INV_ROW[8]  = {0, 0, 1, 0, 1, 0, 0, 1}"),
    # key schedule
    ("rcon_off_by_one", "oracle_gf_pow(0x02, (unsigned)(j - 1))",
     "oracle_gf_pow(0x02, (unsigned)j)"),
    ("rotword_wrong_way", "uint8_t rot[4] = {t[1], t[2], t[3], t[0]};",
     "uint8_t rot[4] = {t[3], t[0], t[1], t[2]};"),
    ("no_rotword", "uint8_t rot[4] = {t[1], t[2], t[3], t[0]};",
     "uint8_t rot[4] = {t[0], t[1], t[2], t[3]};"),
    ("aes256_no_extra_subword", "} else if (nk > 6 && i % nk == 4) {",
     "} else if (nk > 8 && i % nk == 4) {"),
    ("schedule_wrong_lag", "w[i][b] = oracle_gf_add(w[i - nk][b], t[b]);",
     "w[i][b] = oracle_gf_add(w[i - 4][b], t[b]);"),
    # round steps
    ("shiftrows_wrong_way", "t[r][c] = st[r][(c + r) % 4];",
     "t[r][c] = st[r][(c + 4 - r) % 4];"),
    ("inv_shiftrows_wrong_way", "t[r][(c + r) % 4] = st[r][c];",
     "t[r][(c + 4 - r) % 4] = st[r][c];"),
    ("mix_matrix_transposed", "m[i][j] = row[(j - i + 4) % 4];",
     "m[i][j] = row[(i - j + 4) % 4];"),
    ("mix_row_swapped", "MIX_ROW[4]     = {2, 3, 1, 1}", "MIX_ROW[4]     = {3, 2, 1, 1}"),
    ("inv_mix_row_swapped", "INV_MIX_ROW[4] = {14, 11, 13, 9}",
     "INV_MIX_ROW[4] = {14, 9, 13, 11}"),
    ("state_transposed_on_load", "st[k % 4][k / 4] = in[k];", "st[k / 4][k % 4] = in[k];"),
    ("mix_in_final_round",
     "        if (r < nr)\n            mix_columns_with(st, MIX_ROW);",
     "        if (r <= nr)\n            mix_columns_with(st, MIX_ROW);"),
    ("decrypt_skips_inv_mix",
     "        if (r < nr)\n            mix_columns_with(st, INV_MIX_ROW);",
     "        if (r < 0)\n            mix_columns_with(st, INV_MIX_ROW);"),
    ("decrypt_last_key_wrong", "    add_round_key(st, rk);\n    store_state(out, st);",
     "    add_round_key(st, rk + 16);\n    store_state(out, st);"),
    ("one_round_short", "for (int r = 1; r <= nr; ++r) {", "for (int r = 1; r < nr; ++r) {"),
    # modes
    ("counter_little_endian", "blk[12] = (uint8_t)(ctr >> 24);\n    blk[13] = (uint8_t)(ctr >> 16);\n"
     "    blk[14] = (uint8_t)(ctr >> 8);\n    blk[15] = (uint8_t)ctr;",
     "blk[15] = (uint8_t)(ctr >> 24);\n    blk[14] = (uint8_t)(ctr >> 16);\n"
     "    blk[13] = (uint8_t)(ctr >> 8);\n    blk[12] = (uint8_t)ctr;"),
    ("counter_wraps_silently", "if ((uint64_t)ctr0 + nblocks > (1ull << 32))\n        return -3;",
     "if (0)\n        return -3;"),
    # GCM
    ("gcm_reduction_constant", "V[0] ^= 0xE1;", "V[0] ^= 0xE0;"),
    ("gcm_bit_order", "int xi = (X[i / 8] >> (7 - i % 8)) & 1;", "int xi = (X[i / 8] >> (i % 8)) & 1;"),
    ("gcm_lengths_in_bytes", "uint64_t abits = (uint64_t)aad_len * 8, cbits = (uint64_t)ct_len * 8;",
     "uint64_t abits = (uint64_t)aad_len, cbits = (uint64_t)ct_len;"),
    ("gcm_counter_starts_at_1", "int rc = oracle_ctr_xcrypt(key, key_bytes, iv, 2, in, out, nbytes);\n    if (rc)\n        return rc;\n    return gcm_tag",
     "int rc = oracle_ctr_xcrypt(key, key_bytes, iv, 1, in, out, nbytes);\n    if (rc)\n        return rc;\n    return gcm_tag"),
    ("gcm_j0_counter", "J0[15] = 1;", "J0[15] = 2;"),
    ("cbc_chains_plaintext", "cipher_block(rk, nr, box, x, out + off);\n        memcpy(chain, out + off, 16);",
     "cipher_block(rk, nr, box, x, out + off);\n        memcpy(chain, in + off, 16);"),
]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, source, name, old, new):
    assert source.count(old) == 1, "mutation anchor must match exactly once: " + name
    path = tmp_path / ("mutant_%s.c" % name)
    path.write_text(source.replace(old, new))
    lib = oracle_mod.load(oracle_mod.build(force=True, src=str(path),
                                           out=str(tmp_path / ("libm_%s.so" % name))))
    o = oracle_mod.Oracle(lib)
    failed = []
    for pin in oracle_pins.ALL_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError, IndexError):
            failed.append(pin.__name__)
    assert failed, "mutant %s passed every pin" % name
