"""The oracle's C code and the library's host-side constants code under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU only): the oracle's
brute-force, law, bottom-k, counter and tabulation pins rerun against a
sanitizer build of dms_oracle.c, and the constants code, built with the
sanitizers into a small driver, must print what the oracle derives."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PINS = ["test_oracle_bruteforce.py", "test_oracle_laws.py", "test_oracle_bottomk.py",
        "test_oracle_counters.py", "test_oracle_tabulation.py"]


def _runtime(name):
    path = subprocess.check_output(["gcc", "-print-file-name=" + name], text=True).strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip(f"{name} not available")
    return path


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    lib = O.build(force=True, sanitize=True)
    env = dict(os.environ)
    env["DMS_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = _runtime("libasan.so") + ":" + _runtime("libubsan.so")
    # the Python interpreter itself is not instrumented: leaks it holds at exit are not the oracle's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + [os.path.join(HERE, p) for p in PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out


def test_library_constants_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "spec_constants")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           os.path.join(HERE, "native", "spec_constants_driver.cpp"),
                           os.path.join(ROOT, "paper_2005_11547_amd", "csrc", "dms_constants.cpp"),
                           "-o", exe])
    cases = [(0, 1), (2005_11547, 331), (2005_11547, 1676), (2 ** 64 - 1, 8122), (7, 38166)]
    args = [str(v) for c in cases for v in c]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe] + args, capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.strip().split("\n")
    assert len(lines) == 6 * len(cases) + 1
    for n, (seed, t) in enumerate(cases):
        block = {ln.split(" ", 1)[0]: ln.split(" ")[1:] for ln in lines[6 * n:6 * n + 6]}
        keys = O.hash_keys(seed)
        assert [int(v) for v in block["keys"]] == [keys[x] for x in
                                                  ("key_r", "key_a", "key_u", "key_v", "key_s", "key_l")]
        assert [int(v) for v in block["pois"]] == list(O.poisson_thresholds())
        W, R, u = O.tables(t)
        assert [float.fromhex(v) for v in block["W"]] == list(np.asarray(W, dtype=float))
        assert [float.fromhex(v) for v in block["R"]] == list(np.asarray(R, dtype=float))
        assert float.fromhex(block["u"][0]) == u
        assert [int(v) for v in block["tab"]] == list(O.tab_tables(seed))
    assert [int(v) for v in lines[-1].split()] == [O.t_of_k(k) for k in range(1, 4097)]
