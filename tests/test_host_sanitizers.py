"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers in tests/sanitize/: the input generator's ray caster with the C
form of the dithering oracle (gcc), and the library's host code (api.cpp,
compiled by hipcc with the sanitizers on the host side only and linked with
the device objects of the regular build) exercised through the host-side
argument checks and workspace arithmetic that run without a GPU.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")


def test_generator_and_dithering_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "gen_oracle"
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-ffp-contract=off",
                           os.path.join(SAN, "gen_oracle_driver.c"), os.path.join(ROOT, "gen", "raycast.c"),
                           os.path.join(ROOT, "oracle", "fs_dither.c"), "-o", str(exe), "-lm"])
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.startswith("ok")


def test_library_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    objs = [os.path.join(ROOT, "_build", n + ".o") for n in ("step", "aux", "scan", "sample", "aniso")]
    if not os.path.exists(hipcc) or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs hipcc and the regular build's device objects (python -m paper_1910_00572_amd.build)")
    api = tmp_path / "api_san.o"
    # sanitizers on the host side only (-Xarch_host before each option)
    subprocess.check_call([hipcc, "-x", "hip", "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                           "-I", os.path.join(ROOT, "include"), "-c",
                           os.path.join(ROOT, "paper_1910_00572_amd", "csrc", "api.cpp"), "-o", str(api)])
    exe = tmp_path / "host_abi"
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-I", os.path.join(ROOT, "include"),
                           "-x", "c", os.path.join(SAN, "host_abi_driver.c"), "-x", "none", str(api), *objs,
                           "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=ENV, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout
