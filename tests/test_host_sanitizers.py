"""The host plan builder (window placement, support rows, segment and coverage lists,
workspace layout) under AddressSanitizer and UndefinedBehaviorSanitizer: the library's
sources and tests/host_plan_driver.cpp built with host-side sanitizers (the device code
unoptimised, as it never runs here), then every supported shape, precision, LED grid,
multiplexing and flag combination and a set of malformed problems through
elfpie_workspace_bytes.  A sanitizer report aborts the driver.  CPU only; the build is
cached in tests/_build by a hash of the sources."""
import hashlib
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2209_14671_amd", "csrc")
DRIVER = os.path.join(HERE, "host_plan_driver.cpp")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")


def sources():
    files = [DRIVER, os.path.join(ROOT, "include", "elfpie.h")]
    files += sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp")))
    return files


def build():
    h = hashlib.sha256()
    for f in sources():
        h.update(open(f, "rb").read())
    out_dir = os.path.join(HERE, "_build")
    exe = os.path.join(out_dir, "host_plan_driver_" + h.hexdigest()[:16])
    if os.path.exists(exe):
        return exe
    os.makedirs(out_dir, exist_ok=True)
    for old in os.listdir(out_dir):
        if old.startswith("host_plan_driver_"):
            os.remove(os.path.join(out_dir, old))
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xarch_device", "-O0", "-Xarch_device", "-g0",
           "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, "elfpie.hip"), DRIVER,
           "-L", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib"), "-lrocprofiler-sdk-roctx",
           "-o", exe + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    if res.returncode != 0:
        raise RuntimeError(f"sanitizer build failed:\n{res.stderr[-4000:]}")
    os.replace(exe + ".tmp", exe)
    return exe


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_plan_builder_is_clean_under_asan_and_ubsan():
    exe = build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert res.returncode == 0
    assert "problems 0" in out
