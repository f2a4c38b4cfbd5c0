"""Host code under sanitizers (CPU only).

* The FP64 oracle, built with gcc -fsanitize=address,undefined (no recovery,
  leak detection on), driven through every entry point on small seeded
  inputs by tests/san/oracle_driver.c, which also checks the adjoint
  identities of the projector pair and the sketches.
* libimask's host code (validation, workspace and table sizing, batch
  buffers, the launch-shape table, host draws, step-size rules), built with
  hipcc and the sanitizers on the host side only (each -fsanitize= right
  after -Xarch_host: the GPU code is built as usual), driven by
  tests/san/host_driver.cpp; nothing reaches a device.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_sanitizer_build(tmp_path, sources, out):
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-std=gnu11", *sources, "-o", out, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0 and "asan" in (res.stderr + res.stdout).lower():
        pytest.skip("gcc has no sanitizer runtime here")
    assert res.returncode == 0, res.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _gcc_sanitizer_build(tmp_path, [os.path.join(ROOT, "tests", "san", "oracle_driver.c"),
                                    os.path.join(ROOT, "oracle", "imask_oracle.c")], exe)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok")
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr


HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SANITIZERS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                   "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_library_host_code_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2412_10249_amd", "csrc")
    exe = str(tmp_path / "host_san")
    cmd = [HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", *HOST_SANITIZERS, "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "kernels.hip"), os.path.join(csrc, "api.hip"),
           os.path.join(ROOT, "tests", "san", "host_driver.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")  # the HIP runtime keeps its allocations
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.strip().endswith("ok")
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
