"""The oracle's pins must catch plausible mistakes.

Each case copies the oracle's C sources, plants one mistake by text
substitution, builds the copy on the CPU and runs the pin suites
(test_oracle_aes.py, test_oracle_dpf.py, test_oracle_chacha.py,
test_oracle_batch.py) against it: they must fail.
"""
import os
import shutil
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
sys.path.insert(0, str(ROOT))
import oracle  # noqa: E402

MUTANTS = {
    "no_mixcolumns": ("aes_ref.c", "        mix_columns(s);\n", "\n"),
    "shiftrows_right": ("aes_ref.c", "t[c] = s[r][(c + r) % 4];", "t[c] = s[r][(c + 4 - r) % 4];"),
    "rcon_not_doubled": ("aes_ref.c", "rcon = gf_mul(rcon, 0x02);", "rcon = rcon;"),
    "counter_little_endian": ("dpf_ref.c", "blk[15 - i] = (uint8_t)", "blk[i] = (uint8_t)"),
    "child_index_lsb_first": ("dpf_ref.c", "expand(key, ch, d + 1, 2 * j + (uint64_t)c, shares);",
                              "expand(key, ch, d + 1, j + ((uint64_t)c << d), shares);"),
    "point_eval_lsb_first": ("dpf_ref.c", "int c = (int)((j >> (n - d)) & 1);\n        child(",
                             "int c = (int)((j >> (d - 1)) & 1);\n        child("),
    "control_bit_of_prf_output": ("dpf_ref.c", "xor16(out, p, cw(key, tbit(parent), c, d));",
                                  "xor16(out, p, cw(key, tbit(p), c, d));"),
    "no_party_sign": ("dpf_ref.c", "return key[1] ? (uint32_t)(0u - v) : v;", "return v;"),
    "beta_bytes_reversed": ("dpf_ref.c", "((beta >> (8 * i)) & 0xff)", "((beta >> (8 * (3 - i))) & 0xff)"),
    "offpath_cw_drops_term": ("dpf_ref.c", "C[1 - tau][cb][i] = R[i] ^ P[0][cb][i] ^ P[1][cb][i];",
                              "C[1 - tau][cb][i] = R[i] ^ P[1][cb][i];"),
    "control_bits_not_forced_apart": ("dpf_ref.c", "((P[1][c][0] & 1) ^ 1 ^ tbit(ns0))",
                                      "((P[1][c][0] & 1) ^ tbit(ns0))"),
    "answer_transposed": ("dpf_ref.c", "ans[k] += y[j] * table[j * dim + k];",
                          "ans[k] += y[j] * table[k * rows + j];"),
    "chacha_rotation_12_as_13": ("chacha_ref.c", "*b = rotl(*b, 12);", "*b = rotl(*b, 13);"),
    "chacha_no_feed_forward": ("chacha_ref.c", "uint32_t v = x[i] + init[i];", "uint32_t v = x[i];"),
    "chacha_wrong_diagonal": ("chacha_ref.c", "qr(x, 1, 6, 11, 12);", "qr(x, 1, 6, 11, 15);"),
    "chacha_nine_double_rounds": ("chacha_ref.c", "for (int i = 0; i < 10; i++) {", "for (int i = 0; i < 9; i++) {"),
    "chacha_key_not_doubled": ("dpf_ref.c", "memcpy(key + 16, s, 16);", "memset(key + 16, 0, 16);"),
    "chacha_child_same_half": ("dpf_ref.c", "memcpy(out, blk + 16 * (x % 4), 16);", "memcpy(out, blk, 16);"),
    "chacha_tree_uses_aes": ("dpf_ref.c", "or_prf_by(key[3], parent, (uint64_t)c, p);",
                             "or_prf_by(0, parent, (uint64_t)c, p);"),
    "bins_first_row_not_scaled": ("dpf_ref.c", "uint64_t first = b << jb->bin_log;", "uint64_t first = b;"),
    "bins_keys_bin_major": ("dpf_ref.c", "uint64_t b = i % jb->n_bins;", "uint64_t b = i / jb->n_clients;"),
    "slice_ignores_offset": ("dpf_ref.c", "const uint32_t y = or_eval_point(key, row0 + i);",
                             "const uint32_t y = or_eval_point(key, i);"),
    "answer_skips_last_row": ("dpf_ref.c", "for (uint64_t j = 0; j < rows; j++)\n        for (uint32_t k",
                              "for (uint64_t j = 0; j + 1 < rows; j++)\n        for (uint32_t k"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    fname, old, new = MUTANTS[name]
    for s in oracle.SOURCES + ("oracle.h",):
        shutil.copy(oracle.HERE / s, tmp_path / s)
    src = (tmp_path / fname).read_text()
    assert src.count(old) == 1, f"mutation site for {name} not found exactly once"
    (tmp_path / fname).write_text(src.replace(old, new))
    lib = oracle.build(out=tmp_path / "libmutant.so", src_dir=tmp_path, extra=("-w",))
    env = dict(os.environ, ORACLE_LIB_PATH=str(lib))
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
         str(ROOT / "tests" / "test_oracle_aes.py"), str(ROOT / "tests" / "test_oracle_dpf.py"),
         str(ROOT / "tests" / "test_oracle_chacha.py"), str(ROOT / "tests" / "test_oracle_batch.py")],
        env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake {name} passed every pin:\n{r.stdout[-2000:]}"
