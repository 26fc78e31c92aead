"""The runtime's host-only code (CSR validation, size bounds, the int128 and
256-bit -> double conversions, the finalisation of exact sums; in
paper_1701_01772_amd/csrc/lge_hostmath.cpp) and the C oracle, built with g++
under AddressSanitizer and UndefinedBehaviorSanitizer and run through
tests/host_checks.cpp.  The checks compare the runtime with the oracle and
with values the arithmetic fixes; any sanitizer report aborts the run."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
    return r


@pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None, reason="no host compiler")
def test_host_code_under_sanitizers(tmp_path):
    objs = []
    for src, cc, std in ((os.path.join(ROOT, "paper_1701_01772_amd", "csrc", "lge_hostmath.cpp"), "g++", "-std=c++17"),
                         (os.path.join(HERE, "host_checks.cpp"), "g++", "-std=c++17"),
                         (os.path.join(ROOT, "oracle", "lge_oracle.c"), "gcc", "-std=c11")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = _run([cc, std] + SAN + ["-c", src, "-o", obj])
        assert r.returncode == 0, "compile failed: %s" % src
        objs.append(obj)
    exe = str(tmp_path / "host_checks")
    r = _run(["g++"] + SAN + objs + ["-o", exe, "-lpthread", "-lm"])
    assert r.returncode == 0, "link failed"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
