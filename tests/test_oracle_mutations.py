"""Plant plausible mistakes in copies of the oracle (CPU only) and check that
the pin suite rejects every one of them.

Each mutant is a one-line change of the oracle source compiled into a temp
directory; the pins then run in a child process against that library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nnsemd_oracle.c")

MUTANTS = {
    # greedy protocol serving the farthest claimant first
    "farthest_first": ("    if (a->key < b->key) return -1;\n    if (a->key > b->key) return 1;",
                       "    if (a->key > b->key) return -1;\n    if (a->key < b->key) return 1;"),
    # argmin ties going to the largest supplier index
    "argmin_tie_last": ("if (k < best) { second = best;", "if (k <= best) { second = best;"),
    # claimant ties broken by the larger consumer index
    "claimant_tie_reversed": ("    return (a->j > b->j) - (a->j < b->j);\n}\n\nstatic int cmp_random",
                              "    return (a->j < b->j) - (a->j > b->j);\n}\n\nstatic int cmp_random"),
    # the cost charged with the squared distance under L2
    "cost_uses_key": ("R = R + f * dist_of_key(cl[e].key, metric);", "R = R + f * cl[e].key;"),
    # the consumer's demand never decreases
    "no_consumer_update": ("c[j] = c[j] - f;", "c[j] = c[j];"),
    # the printed inner-loop bound: the last claimant is never served
    "skip_last_claimant": ("for (int64_t e = lo; e < hi; ++e) {\n                if (!(s[i] > 0.0)) break;",
                           "for (int64_t e = lo; e < hi - 1; ++e) {\n                if (!(s[i] > 0.0)) break;"),
    # the supplier keeps serving after it is empty
    "serve_when_empty": ("if (!(s[i] > 0.0)) break;", "if (s[i] < 0.0) break;"),
    # one flow is sent the wrong way: f = max instead of min
    "flow_max": ("double f = s[i] < c[j] ? s[i] : c[j];", "double f = s[i] > c[j] ? s[i] : c[j];"),
    # near ties judged without the absolute rule at distance 0
    "near_tie_no_zero_rule": ("if (d1 == 0.0) return gap <= 1e-12;", ""),
    # near ties of the NNS step judged on squared keys instead of distances
    "near_tie_on_keys": ("near_tie(dist_of_key(best, metric), dist_of_key(second, metric))",
                         "near_tie(best, second)"),
    # a given D read with its columns mirrored (consumer j sees column n-1-j)
    "given_D_mirrored": ("if (g->D != NULL) return g->D[i * g->n + j];",
                         "if (g->D != NULL) return g->D[i * g->n + (g->n - 1 - j)];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-o",
                    str(lib), str(mut), "-lm"], check=True)
    env = dict(os.environ, NNSEMD_ORACLE_LIB=str(lib))
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"mutant {name} survived the pins:\n{res.stdout[-2000:]}"
