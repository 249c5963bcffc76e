"""The FP64 CPU oracle under the host address and undefined-behaviour
sanitizers: oracle/sanitize_main.c runs every entry of oracle/pmdg_ref.c once
on small inputs (two bricks with PMUTs, receive mode and receivers; absorbing
faces and a matched layer; trilinear hexahedra; the face matching of
Algorithm 3).  Built with gcc, without OpenMP, so that every loop runs on the
one instrumented thread."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_runs_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    src = [os.path.join(ROOT, "oracle", "sanitize_main.c"), os.path.join(ROOT, "oracle", "pmdg_ref.c")]
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas"]
    subprocess.check_call(cmd + src + ["-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "all entries ran" in r.stdout
