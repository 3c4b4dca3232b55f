"""Planted mistakes in the CPU oracle are caught by its pins (no GPU).

Each mutant is a copy of ``oracle/ensei_oracle.c`` with one plausible bug
(a dropped term, a wrong sign, a wrong index, a transposed operand, a missing
reduction) compiled into a temporary library. The test asserts that at least
one pin of ``tests/pins.py`` fails on it, so the pins constrain every part of
the oracle rather than only its own restatement. The Python part of the oracle
(the error sampler's thresholds, ``oracle.cdt_table``) gets the same treatment:
a mutated copy of the function replaces it while the pins run.
"""
import os
import subprocess
import textwrap

import pytest

import oracle
from tests import pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ensei_oracle.c")
PY_SRC = os.path.join(ROOT, "oracle", "__init__.py")

MUTANTS = {
    "root_not_inverted": ("return inverse ? powmod(w, p - 2, p) : w;", "return w;"),
    "primitive_root_unchecked": ("if (ok) return g;", "return g;"),
    "intt_missing_scale": (
        "    uint64_t scale = inverse ? or_inverse((uint64_t)H * (uint64_t)W % p, p) : 1;\n    int64_t F = (int64_t)H * W;\n    uint64_t *powH",
        "    uint64_t scale = 1;\n    int64_t F = (int64_t)H * W;\n    uint64_t *powH",
    ),
    "row_uses_column_root": ("powW[(int64_t)i2 * k2 % W]", "powH[(int64_t)i2 * k2 % H]"),
    "direct_dft_wrong_index": ("powmod(wH, (uint64_t)i1 * k1, p)", "powmod(wH, (uint64_t)i1 * k2, p)"),
    "conv_correlation_not_convolution": ("int r1 = ((m1 - j1) % H + H) % H", "int r1 = ((m1 + j1) % H + H) % H"),
    "conv_weight_not_reduced": ("if (wv < 0) wv += (int64_t)p;\n                                int r1", "int r1"),
    "filter_transposed_in_grid": ("w_hat[t * F + a * W + b] = (uint32_t)v;", "w_hat[t * F + b * W + a] = (uint32_t)v;"),
    "splitmix_wrong_shift": ("z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;", "z = (z ^ (z >> 29)) * 0x94d049bb133111ebULL;"),
    "enc_counter_off_by_one": ("(ct_index0 + q) * (uint64_t)n + (uint64_t)j + 1)", "(ct_index0 + q) * (uint64_t)n + (uint64_t)j)"),
    "enc_counter_channel_major": ("uint64_t q = (uint64_t)((b * F + f) * C + c)", "uint64_t q = (uint64_t)((b * C + c) * F + f)"),
    "enc_dropped_error": ("dot + (uint64_t)(int64_t)e[mi] + delta * (uint64_t)m[mi];", "dot + delta * (uint64_t)m[mi];"),
    "enc_wrong_key_sign": (
        "                    if (s[j] == 1) dot += a;\n                    else if (s[j] == -1) dot -= a;",
        "                    if (s[j] == 1) dot += a;\n                    else if (s[j] == -1) dot += a;",
    ),
    "delta_rounded_up": ("return (uint64_t)((((u128)1) << 64) / p);", "return (uint64_t)((((u128)1) << 64) / p + 1);"),
    "dec_truncates_not_rounds": ("u128 t = (u128)phi * p + (((u128)1) << 63);", "u128 t = (u128)phi * p;"),
    "dec_missing_final_mod": ("m[(b * C + c) * F + f] = (uint32_t)(v % p);", "m[(b * C + c) * F + f] = (uint32_t)v;"),
    "dec_phase_sign": ("return w[(int64_t)n * stride] - dot;", "return w[(int64_t)n * stride] + dot;"),
    "homconv_mask_on_word0": ("out[n * ostride] += or_delta(p)", "out[0] += or_delta(p)"),
    "homconv_weight_transposed": ("w_hat[(o * Cin + i) * F + f]", "w_hat[(i * Cout + o) * F + f]"),
    "homconv_mask_missing_delta": ("out[n * ostride] += or_delta(p) * (uint64_t)r", "out[n * ostride] += (uint64_t)r"),
    "homconv_wrong_word_stride": ("blk[(int64_t)j * Cin + i]", "blk[(int64_t)i * (n + 1) + j]"),
    "server_share_not_negated": ("s_b[k] = (uint32_t)((p - r[k] % p) % p);", "s_b[k] = (uint32_t)(r[k] % p);"),
    "homrec_on_word0": ("ct[((b * F + f) * (int64_t)(n + 1) + n) * C + c] += delta", "ct[((b * F + f) * (int64_t)(n + 1)) * C + c] += delta"),
    "homrec_missing_delta": ("+= delta * (uint64_t)s_hat[(b * C + c) * F + f];", "+= (uint64_t)s_hat[(b * C + c) * F + f];"),
    "homrec_share_index_transposed": ("s_hat[(b * C + c) * F + f]", "s_hat[(b * F + f) * C + c]"),
    "reshare_share_added": ("s_a_next[k] = (uint32_t)((u + p - s_b_next[k]) % p);", "s_a_next[k] = (uint32_t)((u + s_b_next[k]) % p);"),
    "seeded_counter_off_by_one": ("w[(int64_t)j * C] = or_splitmix64(seed_a, (ct_index0 + q) * (uint64_t)n + (uint64_t)j + 1);",
                                  "w[(int64_t)j * C] = or_splitmix64(seed_a, (ct_index0 + q) * (uint64_t)n + (uint64_t)j);"),
    "seeded_index_offset_dropped": ("w[(int64_t)j * C] = or_splitmix64(seed_a, (ct_index0 + q) * (uint64_t)n",
                                    "w[(int64_t)j * C] = or_splitmix64(seed_a, q * (uint64_t)n"),
    "seeded_b_words_transposed": ("w[(int64_t)n * C] = bw[(b * F + f) * C + c];", "w[(int64_t)n * C] = bw[(b * C + c) * F + f];"),
    "noise_counter_off_by_one": ("uint64_t u = or_splitmix64(seed_e, ct_index0 + q + 1);",
                                 "uint64_t u = or_splitmix64(seed_e, ct_index0 + q);"),
    "noise_field_shift": ("uint64_t v = (u >> 15) & ((1ULL << 48) - 1);", "uint64_t v = (u >> 16) & ((1ULL << 48) - 1);"),
    "noise_sign_from_low_bit": ("e[(b * C + c) * F + f] = (u >> 63) && mag ? -mag : mag;",
                                "e[(b * C + c) * F + f] = (u & 1) && mag ? -mag : mag;"),
    "noise_index_transposed": ("e[(b * C + c) * F + f] = (u >> 63)", "e[(b * F + f) * C + c] = (u >> 63)"),
    "reshare_square_dropped": ("uint64_t u = act == 1 ? mulmod(y, y, p) : y;", "uint64_t u = y;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    assert mutated != src
    c_path = tmp_path / f"{name}.c"
    so_path = tmp_path / f"lib_{name}.so"
    c_path.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp", str(c_path), "-o", str(so_path)], check=True)
    return oracle.Oracle(str(so_path))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    orc = _build(tmp_path, name, old, new)
    caught_by = None
    for check in pins.ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError, IndexError, OverflowError):
            caught_by = check.__name__
            break
    assert caught_by, f"planted mistake {name!r} passed every pin"


# Planted mistakes in the Python threshold table of the rounded-Gaussian
# sampler: rounding instead of the floor, the half-integer edge dropped, the
# sqrt(2) of the Gaussian's erf dropped, too little working precision.
PY_MUTANTS = {
    "cdt_rounds_not_floors": ("rounding=ROUND_FLOOR", 'rounding="ROUND_HALF_EVEN"'),
    "cdt_edge_not_half_integer": ("x = (Decimal(k) + Decimal(1) / 2) /", "x = Decimal(k) /"),
    "cdt_sigma_without_sqrt2": ("/ (sigma * Decimal(2).sqrt())", "/ sigma"),
    "cdt_low_precision": ("prec = 80", "prec = 12"),
}


def _mutated_cdt_table(old, new):
    src = open(PY_SRC).read()
    start = src.index("def cdt_table()")
    end = src.index("\ndef ", start + 1)
    fn = src[start:end]
    assert fn.count(old) == 1, f"mutation site {old!r} not found"
    ns = dict(vars(oracle))
    exec(textwrap.dedent(fn.replace(old, new)), ns)
    return ns["cdt_table"]


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_python_mutant_is_caught(monkeypatch, name):
    old, new = PY_MUTANTS[name]
    monkeypatch.setattr(oracle, "cdt_table", _mutated_cdt_table(old, new))
    orc = oracle.default()
    caught_by = None
    for check in pins.ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError, IndexError, OverflowError):
            caught_by = check.__name__
            break
    assert caught_by, f"planted mistake {name!r} passed every pin"
