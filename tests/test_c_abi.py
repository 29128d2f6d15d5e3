"""The C ABI used from a plain C99 program (tests/c_abi/host_check.c), compiled with gcc
against include/pcpf.h and linked to the built library: host calls only, no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2006_10967_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_host_calls_from_c(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libpcpf.so")):
        pytest.skip("libpcpf.so is not built")
    exe = str(tmp_path / "host_check")
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c_abi", "host_check.c"), "-o", exe,
           "-L", LIBDIR, "-lpcpf", "-Wl,-rpath," + LIBDIR, "-Wl,--allow-shlib-undefined", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("ok  ") == 16
