"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch each one.

Every mutant is a one-line textual change of oracle.c, compiled into a temporary
library and run under the pin suite in a subprocess; the suite must fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "drop_last_start": ("for (int64_t s = 0; s <= last; ++s)", "for (int64_t s = 0; s < last; ++s)"),
    "drop_last_compare": ("for (uint64_t j = 0; j < m; ++j)\n        if (t[s + j] != p[j])",
                          "for (uint64_t j = 0; j + 1 < m; ++j)\n        if (t[s + j] != p[j])"),
    "reversed_pattern_index": ("if (t[s + j] != p[j])", "if (t[s + j] != p[m - 1 - j])"),
    "report_one_based": ("pos[count] = s;", "pos[count] = s + 1;"),
    "hist_seven_bit": ("hist[t[s]]++;", "hist[t[s] & 0x7f]++;"),
    "freq_descending": ("return fa < fb ? -1 : 1;", "return fa < fb ? 1 : -1;"),
    "order_h_chain_swap": ("const uint64_t starts[3] = {4, 3, 2};", "const uint64_t starts[3] = {4, 2, 3};"),
    "alg4_or_instead_of_and": ("            found &= simd_compare(t, i, nvalid, p, j);\n            if (found == 0)",
                               "            found |= simd_compare(t, i, nvalid, p, j);\n            if (found == 0)"),
    "alg4_inverted_exit": ("        if (found == 0)\n            continue;", "        if (found != 0)\n            continue;"),
    "alg4_window_off_by_one": ("if (t[i + k + j] == p[j])", "if (t[i + k + j] == p[j ? j - 1 : 0])"),
    "bigram_row_for_backward": ("er = frac_of(bigram[(uint64_t)p[j] * 256 + p[j + 1]], col[p[j + 1]]);",
                                "er = frac_of(bigram[(uint64_t)p[j] * 256 + p[j + 1]], row[p[j]]);"),
    "bigram_max_of_neighbours": ("(frac_less(er, el) ? er : el)", "(frac_less(er, el) ? el : er)"),
    "bigram_ignores_conditionals": ("            if (left || right) {\n                frac_t el",
                                    "            if (0) {\n                frac_t el"),
    "nonoverlap_resume_early": ("            s += m;\n", "            s += m - 1 + (m == 1);\n"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found for {name}"
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "oracle_mutant.c"
    lib = tmp_path / "liboracle_mutant.so"
    csrc.write_text(mutated)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", str(lib), str(csrc)], check=True)
    env = dict(os.environ, ORACLE_LIB_OVERRIDE=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pin suite:\n{r.stdout[-2000:]}"
