"""The oracle and the host-side engine logic under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

tests/sanitize/oracle_driver.c runs every oracle entry point on small and
edge-case shapes (gcc, -fsanitize=address,undefined); tests/sanitize/
host_engine.cpp runs the engine's host logic (validation, storage rule,
workspace layouts, bridge schedules, batch sizing, the pool allocator,
shutdown) with the kernel entry points stubbed out (hipcc, the sanitizers on
the host pass only).  Each must exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    return r.returncode, r.stdout + r.stderr


def test_oracle_under_sanitizers(orc, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    poly, vinit = orc.joe_kuo_data()
    ndim = 64
    poly = np.ascontiguousarray(poly[:ndim], dtype=np.int64)
    vinit = np.ascontiguousarray(vinit[:ndim], dtype=np.int64)
    poly.tofile(tmp_path / "poly.bin")
    vinit.tofile(tmp_path / "vinit.bin")
    exe = str(tmp_path / "oracle_san")
    rc, out = _run(["gcc", *SAN, "-std=c11", os.path.join(HERE, "sanitize", "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "amq_oracle.c"), "-lm", "-o", exe])
    assert rc == 0, out
    rc, out = _run([exe, str(tmp_path / "poly.bin"), str(tmp_path / "vinit.bin"), str(ndim),
                    str(vinit.shape[1])], env=ENV, timeout=600)
    assert rc == 0 and "oracle checks passed" in out and "runtime error" not in out, out[-3000:]


def test_host_engine_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "host_engine_san")
    host_san = []
    for f in SAN[:3]:
        host_san += ["-Xarch_host", f]
    rc, out = _run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-std=c++17", "-O1", "-g", *host_san,
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1205_0106_amd", "csrc"),
                    os.path.join(HERE, "sanitize", "host_engine.cpp"), "-o", exe], timeout=900)
    assert rc == 0, out[-3000:]
    rc, out = _run([exe], env=ENV, timeout=600)
    assert rc == 0 and "host engine checks passed" in out and "runtime error" not in out, out[-3000:]
