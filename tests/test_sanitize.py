"""CPU sanitizer builds of the host-side C/C++ code (no GPU needed).

* The oracle with AddressSanitizer + UndefinedBehaviorSanitizer and its
  shared-face debug check (-DORC_FACE_CHECK), driven by tests/oracle_sanitize.c
  over many shapes, both bound modes, every lossless pipeline and damaged
  streams; a planted face mistake must be caught.
* The serving scheduler core (serve.h): the simulated-clock mock under
  ASan + UBSan, and a threaded stress driver (submitters, the scheduling loop
  and a poller on their own threads) under ThreadSanitizer and ASan.
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2507_11165_amd", "csrc")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1 exitcode=66")


def _run(cmd, timeout=300):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=ENV)


def _build_oracle_driver(tmp_path, src=None):
    exe = str(tmp_path / "oracle_sanitize")
    oracle_c = src or os.path.join(ORACLE, "hiz_oracle.c")
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off", "-DORC_FACE_CHECK", *ASAN,
                           "-I", ORACLE, os.path.join(ROOT, "tests", "oracle_sanitize.c"),
                           oracle_c, "-lm", "-o", exe])
    return exe


def test_oracle_under_asan_ubsan_with_face_check(tmp_path):
    r = _run([_build_oracle_driver(tmp_path)])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout


def test_face_check_catches_a_planted_mistake(tmp_path):
    # only the owning block quantizes: non-owners keep the raw prediction on
    # their +1 faces, so shared points disagree
    src = open(os.path.join(ORACLE, "hiz_oracle.c")).read()
    old = "                            buf[li] = xo;\n"
    assert src.count(old) == 1
    bad = tmp_path / "hiz_oracle.c"
    bad.write_text(src.replace(old, "                            buf[li] = owned ? xo : p;\n"))
    r = _run([_build_oracle_driver(tmp_path, str(bad))])
    assert r.returncode == 1 and "faces (compress)" in r.stderr, r.stdout + r.stderr


def test_scheduler_mock_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "serve_mock")
    subprocess.check_call(["g++", "-std=c++17", "-pthread", *ASAN, "-I", CSRC,
                           os.path.join(ROOT, "tests", "serve_mock.cpp"), "-o", exe])
    r = _run([exe, "3", "5000", "400", "4", "8", "600000000", "0.3", "7"])
    assert r.returncode == 0, r.stderr
    assert json.loads(r.stdout)["n"] == 400


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_threaded_scheduler_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / "serve_threads")
    subprocess.check_call(["g++", "-std=c++17", "-pthread", f"-fsanitize={san}",
                           "-fno-sanitize-recover=all", "-g", "-O1", "-I", CSRC,
                           os.path.join(ROOT, "tests", "serve_threads.cpp"), "-o", exe])
    r = _run([exe, "4", "200", "4", "8"])
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok 800"
