"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU calls):

* the oracle's C direct sums (oracle/csum.c) with gcc, against a plain loop and on the invalid
  arguments it must refuse (tests/sanitize/csum_driver.c);
* the library's C ABI built by hipcc with the sanitizers on the host side only, driven through
  the argument validation of every entry point, which fails before any HIP call
  (tests/sanitize/abi_driver.cpp).

A sanitizer report makes the program exit non-zero."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2407_06834_amd", "csrc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def test_oracle_direct_sum_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "csum_asan")
    r = _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
              "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "csum.c"),
              os.path.join(HERE, "csum_driver.c"), "-o", exe, "-lm"])
    assert r.returncode == 0, r.stderr
    r = _run([exe], env=SAN_ENV)
    assert r.returncode == 0 and "0 failures" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def test_abi_host_validation_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument", *san]
    srcs = [os.path.join(CSRC, f + ".hip") for f in ("api", "plan", "nfft", "pcg", "cnn", "mis")]
    srcs.append(os.path.join(HERE, "abi_driver.cpp"))
    objs, procs = [], []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([hipcc, *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
    for p in procs:
        out = p.communicate()[0].decode(errors="replace")
        assert p.returncode == 0, out
    exe = str(tmp_path / "abi_asan")
    r = _run([hipcc, "--offload-arch=gfx950", *san, *objs, "-o", exe])
    assert r.returncode == 0, r.stdout + r.stderr
    r = _run([exe], env=SAN_ENV)
    assert r.returncode == 0 and "0 failures" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
