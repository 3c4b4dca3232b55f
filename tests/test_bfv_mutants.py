"""Planted mistakes in the packed (BFV / RLWE) oracle are caught by its pins
(no GPU). Each mutant is a copy of ``oracle/ensei_bfv_oracle.c`` with one
plausible bug, compiled into a temporary library; some pin of
``tests/pins_bfv.py`` must fail on it."""
import os
import subprocess

import pytest

from oracle import bfv
from tests import pins_bfv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ensei_bfv_oracle.c")

MUTANTS = {
    "even_powers_of_psi": ("(uint64_t)(2 * k + 1) * j;", "(uint64_t)(2 * k) * j;"),
    "inverse_not_scaled": ("const uint64_t scale = inverse ? powm((uint64_t)n, m - 2, m) : 1;",
                           "const uint64_t scale = 1;"),
    "inverse_root_not_inverted": ("if (inverse) psi = powm(psi, m - 2, m);", ""),
    "psi_of_order_n": ("return powm(primitive_root(m), (m - 1) / two_n, m);",
                       "return powm(primitive_root(m), (m - 1) / (uint64_t)n, m);"),
    "primitive_root_unchecked": ("        if (ok) return g;", "        return g;"),
    "delta_floored": ("return (modulus_q(qs) + t / 2) / t; }", "return modulus_q(qs) / t; }"),
    "delta_of_one_limb": ("return (modulus_q(qs) + t / 2) / t; }", "return ((u128)qs[0] + t / 2) / t; }"),
    "filters_lifted_canonically": ("            else if (x > t / 2)\n                x = m - (t - x);",
                                   "            else if (0)\n                x = m - (t - x);"),
    "enc_dropped_error": ("c[i] = (uint32_t)((mulm(dl, u[i], m) + ei) % m);", "c[i] = (uint32_t)(mulm(dl, u[i], m) % m);"),
    "enc_error_sign": ("const uint64_t ei = e[i] < 0 ? m - (uint64_t)(-(int64_t)e[i]) % m : (uint64_t)e[i] % m;",
                       "const uint64_t ei = e[i] < 0 ? (uint64_t)(-(int64_t)e[i]) % m : m - (uint64_t)e[i] % m;"),
    "enc_unscaled_message": ("c[i] = (uint32_t)((mulm(dl, u[i], m) + ei) % m);", "c[i] = (uint32_t)((u[i] + ei) % m);"),
    "key_sign_dropped": ("c[j] = (uint32_t)(s[j] < 0 ? qs[l] - 1 : (uint64_t)s[j]);",
                         "c[j] = (uint32_t)(s[j] < 0 ? 1 : (uint64_t)s[j]);"),
    "a_counter_off_by_one": ("(uint64_t)k + 1) % m;", "(uint64_t)k) % m;"),
    "a_counter_limb_major": ("((ct_index0 + (uint64_t)i) * NLIMB + (uint64_t)l) * (uint64_t)n",
                             "((uint64_t)l * 1000 + (ct_index0 + (uint64_t)i)) * (uint64_t)n"),
    "dec_phase_sign": ("d[i * n + k] = (uint32_t)((w[n + k] + m - mulm(w[k], s_hat[l * n + k], m)) % m);",
                       "d[i * n + k] = (uint32_t)((w[n + k] + mulm(w[k], s_hat[l * n + k], m)) % m);"),
    "crt_wrong_order": ("const uint64_t h = mulm((r[1][i] + q1 - r[0][i] % q1) % q1, inv, q1);",
                        "const uint64_t h = mulm((r[0][i] % q1 + q1 - r[1][i]) % q1, inv, q1);"),
    "dec_truncates": ("mc[i] = (uint32_t)((((u128)phi[i] * t + (q - 1) / 2) / q) % t);",
                      "mc[i] = (uint32_t)((((u128)phi[i] * t) / q) % t);"),
    "pack_channel_block": ("const int64_t g = c / P, j = c % P, k = f / Fp, slot = j * Fp + f % Fp;\n"
                           "                v[((b * G + g) * K + k) * n + slot] = x_hat",
                           "const int64_t g = c % G, j = c / G, k = f / Fp, slot = j * Fp + f % Fp;\n"
                           "                v[((b * G + g) * K + k) * n + slot] = x_hat"),
    "filters_transposed": ("= w_hat[((int64_t)o * Cin + c) * F + f];", "= w_hat[((int64_t)c * Cout + o) * F + f];"),
    "homconv_mask_on_a": ("if (w == 1) acc = (acc + mask_enc", "if (w == 0) acc = (acc + mask_enc"),
    "homconv_last_vector_dropped": ("for (int g = 0; g < G; ++g) {", "for (int g = 0; g + 1 < G; ++g) {"),
    "fold_one_block": ("for (int64_t j = 0; j < P; ++j) acc +=", "for (int64_t j = 0; j < 1; ++j) acc +="),
    "rerand_counter_off_by_one": ("(uint64_t)n +\n                                                             (uint64_t)j + 1);",
                                  "(uint64_t)n +\n                                                             (uint64_t)j);"),
    "rerand_bound_not_doubled": ("(((z >> 32) * (2 * B + 1)) >> 32)", "(((z >> 32) * (B + 1)) >> 32)"),
    "rerand_a_without_e1": ("wa[k] = (uint32_t)((wa[k] + mulm(pa[k], rho[k], m) + e1[k]) % m);",
                            "wa[k] = (uint32_t)((wa[k] + mulm(pa[k], rho[k], m)) % m);"),
    "rerand_b_with_a_key": ("wb[k] = (uint32_t)((wb[k] + mulm(pb[k], rho[k], m) + e2[k]) % m);",
                            "wb[k] = (uint32_t)((wb[k] + mulm(pa[k], rho[k], m) + e2[k]) % m);"),
    "rerand_flood_on_a": ("const uint32_t *rho = h + (i * 3) * (int64_t)n, *e1 = rho + n, *e2 = e1 + n;",
                          "const uint32_t *rho = h + (i * 3) * (int64_t)n, *e2 = rho + n, *e1 = e2 + n;"),
    "mask_unscaled": ("            if (scaled)\n                x = mulm(dl, x, m);", "            if (scaled)\n                x = x;"),
}


def _build(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    assert mutated != src
    c_path = tmp_path / f"{name}.c"
    so_path = tmp_path / f"lib_{name}.so"
    c_path.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", str(c_path), "-o", str(so_path)],
                   check=True)
    o = bfv.BfvOracle(str(so_path))
    o.set_threads(8)
    return o


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    orc = _build(tmp_path, name, old, new)
    caught_by = None
    for check in pins_bfv.ALL_CHECKS:
        try:
            check(orc)
        except (AssertionError, ValueError, IndexError, OverflowError, StopIteration):
            caught_by = check.__name__
            break
    assert caught_by, f"planted mistake {name!r} passed every pin"
