"""The CPU oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (host compilers only; no GPU code is built with a
sanitizer). Each driver exercises its side once at the toy parameters and
checks its results; the sanitizers abort on the first memory or undefined-
behaviour error. The host driver also compares the library's keys and
encryptions with the oracle's, linked in beside it."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    print(r.stdout[-4000:], r.stderr[-4000:])
    return r


@pytest.mark.slow
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "san_oracle")
    r = _run(["gcc", *SAN, "-fopenmp", os.path.join(HERE, "sanitize_oracle.c"),
              os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    assert r.returncode == 0
    env = dict(os.environ, OMP_NUM_THREADS="8")
    r = _run([exe, os.path.join(HERE, "golden", "philox4x32_10_kat.txt")], env=env, timeout=600)
    assert r.returncode == 0 and "0 failed checks" in r.stdout


@pytest.mark.slow
def test_host_code_under_sanitizers(tmp_path):
    obj = str(tmp_path / "oracle.o")
    exe = str(tmp_path / "san_host")
    r = _run(["gcc", *SAN, "-fopenmp", "-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", obj])
    assert r.returncode == 0
    r = _run(["g++", "-std=c++17", *SAN, os.path.join(HERE, "sanitize_host.cpp"),
              os.path.join(ROOT, "paper_2101_03403_amd", "csrc", "cemu_host.cpp"), obj,
              "-fopenmp", "-lpthread", "-lm", "-o", exe])
    assert r.returncode == 0
    r = _run([exe], timeout=300)
    assert r.returncode == 0 and "0 failed checks" in r.stdout
