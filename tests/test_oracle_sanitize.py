"""The CPU oracle built with gcc's sanitizers (AddressSanitizer with leak
checks, UndefinedBehaviorSanitizer; ThreadSanitizer for the threaded
construction) and run over random small texts by tests/oracle_sanitize_main.c.
CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
SOURCES = [os.path.join(ORACLE, "bt_oracle.c"), os.path.join(ORACLE, "bt_par.c"),
           os.path.join(HERE, "oracle_sanitize_main.c")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_oracle_under_sanitizers(san):
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "ora_san")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
               "-fsanitize=" + san, "-fno-sanitize-recover=all", "-I", ORACLE, "-o", exe] + SOURCES
        subprocess.check_call(cmd)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1",
                   TSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "0 failures" in r.stdout
