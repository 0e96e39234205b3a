"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer builds (CPU only):
the oracle's C core with a driver of its own, and the library's host
runtime files (device code built unsanitised, -Xarch_host) linked with the
regular kernel objects and a driver that calls the entry points that need
no device.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1304_2062_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1304_2062_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracle_core_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    _run(["gcc", "-O1", "-g", *SAN, "-fopenmp", "-o", str(exe), os.path.join(HERE, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "cn_core.c"), "-lm"])
    r = _run([str(exe)], env=ENV)
    assert "worst cyclic residual" in r.stdout


HOST_FILES = ["se2n_runtime.hip", "se2n_batch_host.hip", "se2n_cnn_host.hip"]


@pytest.mark.skipif(shutil.which(HIPCC) is None and not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_runtime_under_sanitizers(tmp_path):
    kernels = [f for f in os.listdir(CSRC) if f.endswith(".hip") and f not in HOST_FILES]
    objs = [os.path.join(BUILD, f.replace(".hip", ".o")) for f in kernels]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (python -m paper_1304_2062_amd.build)")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wno-unused-command-line-argument"]
    host_san = [x for s in SAN for x in ("-Xarch_host", s)]
    procs = []
    for f in HOST_FILES:
        o = tmp_path / f.replace(".hip", ".o")
        procs.append((f, subprocess.Popen([HIPCC, *flags, *host_san, "-c", os.path.join(CSRC, f), "-o", str(o)],
                                          stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(str(o))
    for f, pr in procs:
        out, _ = pr.communicate()
        assert pr.returncode == 0, (f, out.decode()[-3000:])
    drv = tmp_path / "host_driver.o"
    _run(["g++", "-O1", "-g", "-std=c++17", *SAN, "-c", os.path.join(HERE, "host_driver.cpp"), "-o", str(drv)])
    exe = tmp_path / "host_san"
    _run([HIPCC, "--offload-arch=gfx950", *host_san, "-o", str(exe), str(drv), *objs])
    r = _run([str(exe)], env=ENV)
    assert "0 unexpected results" in r.stdout
