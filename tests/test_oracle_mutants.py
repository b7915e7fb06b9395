"""The pins have teeth: plausible mistakes planted in a copy of the oracle (on the
CPU) must each make at least one pin fail."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
import test_oracle_bruteforce as BF
import test_oracle_laws as LAWS

MUTANTS = {
    "weight uses the rank uniform": ("double weight = Wn + (wd + V) * dnu;",
                                     "double weight = Wn + (wd + U) * dnu;"),
    "dropped region corner": ("double weight = Wn + (wd + V) * dnu;",
                              "double weight = (wd + V) * dnu;"),
    "column width exponent sign": ("ldexp(P->u, nu - rho)", "ldexp(P->u, rho - nu)"),
    "row count uses the wrong index": ("double rmax = ldexp(1.0, nu);",
                                       "double rmax = ldexp(1.0, rho);"),
    "strict rank filter": ("if (weight <= xi && rank <= tau)", "if (weight <= xi && rank < tau)"),
    "partial last column skipped": ("if (xi < Wn + wd * dnu) break;",
                                    "if (xi < Wn + (wd + 1.0) * dnu) break;"),
    "partial last row skipped": ("if (tau < Rr + rd * drho) break;",
                                 "if (tau < Rr + (rd + 1.0) * drho) break;"),
    "Poisson count off by one": ("uint32_t n = 0;\n    while (n < DMSO_NPOIS",
                                 "uint32_t n = 1;\n    while (n < DMSO_NPOIS"),
    "bucket from the low hash bits": ("uint32_t b = (uint32_t)(((D->s >> 32) * (uint64_t)k) >> 32);",
                                      "uint32_t b = (uint32_t)(((D->s & 0xffffffffULL) * (uint64_t)k) >> 32);"),
    "bucket keeps the maximum": ("dart_less(D->rank, D->s, out_rank[b], out_s[b])",
                                 "dart_less(out_rank[b], out_s[b], D->rank, D->s)"),
}


def _pins(darts):
    """Run a selection of pins; return the names of those that fail."""
    failed = []
    checks = [
        ("rejection sampling", lambda: [BF.test_darthash_equals_rejection_sampling(darts, c) for c in range(8)]),
        ("inclusive boundaries", lambda: BF.test_boundaries_are_inclusive(darts)),
        ("first hitting dart", lambda: BF.test_minhash_is_first_hitting_dart(darts, 4)),
        ("Lemma 1 count", LAWS.test_lemma1_dart_count_is_poisson_phi_t),
        ("Lemma 1 uniformity", LAWS.test_lemma1_darts_are_uniform_under_x),
    ]
    for name, fn in checks:
        try:
            fn()
        except (AssertionError, StopIteration, IndexError):
            failed.append(name)
    return failed


@pytest.fixture(scope="module")
def darts():
    return BF.stream(BF.IDS, BF.T, BF.SEED, BF.NU, BF.RHO)


def test_unmutated_oracle_passes(darts):
    assert _pins(darts) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, darts, name):
    old, new = MUTANTS[name]
    src = open(O.SRC).read()
    assert src.count(old) >= 1, name
    src = src.replace(old, new)
    c = tmp_path / "mut.c"
    c.write_text(src)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", str(so), str(c), "-lm"])
    saved_lib, saved_path = O._lib, O.LIB
    try:
        O._lib = None
        O.LIB = str(so)
        # load the mutant without triggering a rebuild of the real oracle
        orig_build = O.build
        O.build = lambda force=False: str(so)
        O.lib()
        failed = _pins(darts)
    finally:
        O.build = orig_build
        O._lib, O.LIB = saved_lib, saved_path
    assert failed, f"no pin caught mutant '{name}'"
