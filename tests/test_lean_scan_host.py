"""The memory-lean probe scan's window loop (paper_2512_23314_amd/csrc/lean.hpp)
compiled for the host with g++ against a HIP stand-in (tests/host_emu) and run
on the CPU under AddressSanitizer and UBSan: rolled hashes against directly
computed ones, coverage of every window, the short key's leftmost occurrence,
and no access outside its array (a window at text position 0 once read the
byte before the text)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2512_23314_amd", "csrc")


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    out = str(tmp_path_factory.mktemp("lean_host") / "lean_scan_host")
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(HERE, "host_emu"), "-I", CSRC,
           os.path.join(HERE, "host_emu", "lean_scan_host.cpp"), "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_lean_chunk_on_host(binary, seed):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    r = subprocess.run([binary, str(seed)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "0 failing trials" in r.stdout
