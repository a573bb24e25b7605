"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the oracle, driven through every configuration class, and the host
model tables of the library."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]


def _build_run(compiler, srcs, incs, extra, exe):
    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip("no " + compiler)
    cmd = [cc, *SAN, *["-I" + i for i in incs], *srcs, "-o", exe, *extra]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout, r.stderr[-3000:])
    return r.stdout


def test_oracle_clean_under_sanitizers(tmp_path):
    out = _build_run("gcc", [os.path.join(ROOT, "tests", "san_oracle_driver.c"),
                             os.path.join(ROOT, "oracle", "dbm_oracle.c")],
                     [os.path.join(ROOT, "oracle")], ["-std=c99", "-fopenmp", "-lm"],
                     str(tmp_path / "or_drv"))
    assert out.count("mass") == 4


def test_model_tables_clean_under_sanitizers(tmp_path):
    out = _build_run("g++", [os.path.join(ROOT, "tests", "san_model_driver.cpp"),
                             os.path.join(ROOT, "paper_2006_15932_amd", "csrc", "dbm_model.cpp")],
                     [os.path.join(ROOT, "include"),
                      os.path.join(ROOT, "paper_2006_15932_amd", "csrc")], ["-std=c++17"],
                     str(tmp_path / "model_drv"))
    lines = out.strip().splitlines()
    assert len(lines) == 12
    assert sum(" rc=0 " in l + " " for l in lines) == 3       # the regular parameter set
    assert sum("rc=-2" in l for l in lines) == 9               # singular sets rejected
