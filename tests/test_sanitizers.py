"""Host-side AddressSanitizer and UndefinedBehaviorSanitizer builds (CPU only).

The FP64 oracle (plain C) is built with gcc and every one of its functions is
driven on small ragged inputs, empty skewers and invalid arguments
(tests/sanitize/oracle_sanitize.c), with leak detection on.  The library's
sources are built with hipcc with the sanitizers on the host side only, and
the host-side validation of every C entry point is driven with invalid and
empty arguments (tests/sanitize/abi_sanitize.cpp); those calls return before
any HIP call, so no GPU is needed (leak detection is off there: the HIP
runtime keeps its allocations until exit)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

pytestmark = pytest.mark.slow


def _run(exe, env_extra, timeout=120):
    env = dict(os.environ, **env_extra)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, f"{exe} failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D_DEFAULT_SOURCE",
           "-o", exe, os.path.join(HERE, "oracle_sanitize.c"),
           os.path.join(ROOT, "oracle", "lyaf_oracle.c"),
           os.path.join(ROOT, "oracle", "lyaf_instrument_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    out = _run(exe, {"OMP_NUM_THREADS": "2", "ASAN_OPTIONS": "detect_leaks=1"})
    assert "oracle_sanitize: ok" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_abi_host_validation_under_address_and_undefined_sanitizers(tmp_path):
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address",
             "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]
    csrc = os.path.join(ROOT, "paper_1105_4747_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    srcs.append(os.path.join(HERE, "abi_sanitize.cpp"))
    objs = []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], check=True, capture_output=True,
                       timeout=600)
        objs.append(obj)
    exe = str(tmp_path / "abi_sanitize")
    subprocess.run([HIPCC, "--offload-arch=gfx950",
                    "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-o", exe, *objs],
                   check=True, capture_output=True, timeout=300)
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert "abi_sanitize: ok" in out
