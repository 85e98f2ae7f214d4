"""The oracle's pins must be able to fail.

Each mutant below is a copy of the oracle's C source with one plausible
mistake planted (a dropped term, a loosened bound, an off-by-one, a wrong
tie rule).  The copy is compiled into a temporary folder and the oracle's pin
suite runs against it in a child process (ORACLE_LIBRARY points the oracle's
binding at the copy).  Every mutant must make at least one pin fail; a mutant
that survives means part of the oracle is unpinned.  Nothing here touches the
GPU library.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sba_oracle.c")

# (name, text in the source, replacement, replace every occurrence)
MUTANTS = [
    # the distance predicate says "near" for everything
    ("within_always_true",
     "    typedef unsigned __int128 u128;\n",
     "    typedef unsigned __int128 u128;\n    if (k > 0) return 1;\n", False),
    # interior branch loosened by a factor of 2 (distance bound sqrt(2) eps)
    ("within_interior_loose",
     "return (u128)k * (c * c) <= (u128)e2 * (u128)l2;",
     "return (u128)k * (c * c) <= 2 * (u128)e2 * (u128)l2;", False),
    # endpoint branch before a: always near
    ("within_endpoint_a_near",
     "if (t <= 0) return k * (wx * wx + wy * wy) <= e2;",
     "if (t <= 0) return 1;", False),
    # the eps/2 test of the centre-sampled cells checks eps instead
    ("half_ignored",
     "seg_within_k(px, py, x1, y1, x2, y2, eps, half ? 4 : 1)",
     "seg_within_k(px, py, x1, y1, x2, y2, eps, 1)", False),
    # far mismatches never counted
    ("far_never_counted",
     "if (!near_boundary(&a->ps, p, px, py, check_eps, half)) far++;",
     "(void)check_eps; (void)half;", True),
    # scan form: the cell left of a strip's x-range dropped (the "-1")
    ("boundary_range_off_by_one",
     "c0 = (int64_t)cdiv(lo, den * s) - 1;",
     "c0 = (int64_t)cdiv(lo, den * s);", False),
    # crossing rule: points on an edge counted as left of it
    ("crossing_tie_rule",
     "return (y2 > y1) ? (lhs < rhs) : (lhs > rhs);",
     "return (y2 > y1) ? (lhs <= rhs) : (lhs >= rhs);", False),
    # cell side: one too large (diagonal above eps)
    ("cell_side_too_large",
     "    return s;\n}\n\n/* ------------------------------------------------------------------ */\n"
     "/* geometry predicates",
     "    return s + 1;\n}\n\n/* ------------------------------------------------------------------ */\n"
     "/* geometry predicates", False),
]


@pytest.mark.parametrize("name,old,new,every", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new, every):
    src = open(SRC).read()
    assert old in src, f"mutation site of {name} not found in the oracle source"
    mutated = src.replace(old, new) if every else src.replace(old, new, 1)
    cfile = tmp_path / "oracle_mutant.c"
    cfile.write_text(mutated)
    so = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-w", "-fopenmp", "-fPIC", "-shared", "-o",
                    str(so), str(cfile), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIBRARY=str(so), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-p", "no:xdist", os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # 1: some pin failed; negative: the mutant crashed the suite (also caught)
    assert r.returncode == 1 or r.returncode < 0, (
        f"mutant {name} survived the oracle's pins (exit {r.returncode}):\n{r.stdout[-2000:]}")
