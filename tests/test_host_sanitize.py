"""The host engine under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): every library source and tests/sanitize_host.cpp are built
with the sanitizers on the host code only (the device code is compiled as
usual and never launched), and the program sweeps validation, sizes, the
host-side work-table construction and the multilevel set lists over seeded
valid and invalid configurations.  The build is cached under _build/ by the
hash of its sources and flags."""
import hashlib
import os
import subprocess

import pytest

from paper_1902_09699_amd import build as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize_host.cpp")
FLAGS = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _binary():
    srcs = [os.path.join(b.CSRC, s) for s in b.SOURCES] + [DRIVER]
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in srcs + [os.path.join(ROOT, "include", "sip.h"), os.path.join(b.CSRC, "sip_internal.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    out_dir = os.path.join(ROOT, "_build", "sanitize")
    exe = os.path.join(out_dir, f"host_check_{h.hexdigest()[:16]}")
    if not os.path.exists(exe):
        os.makedirs(out_dir, exist_ok=True)
        cmd = [b.hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", b.CSRC, *srcs, "-o", exe + ".tmp"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            pytest.fail("sanitizer build failed:\n" + res.stderr[-4000:])
        os.replace(exe + ".tmp", exe)
    return exe


def test_host_engine_under_address_and_ub_sanitizers():
    exe = _binary()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(res.stdout)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in res.stderr
    assert "runtime error" not in res.stderr
    assert "0 failed checks" in res.stdout
