"""The oracle (plain C) and the library's host FP64 geometry (C++) built with
AddressSanitizer and UndefinedBehaviorSanitizer -- host code only, gcc / g++ --
and run on seeded cases through every entry point (tests/native/)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-ffp-contract=off"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_oracle")
    subprocess.run(["gcc", "-std=c99", *FLAGS, "-I", os.path.join(ROOT, "oracle"), "-o", exe,
                    os.path.join(ROOT, "tests", "native", "asan_oracle.c"),
                    os.path.join(ROOT, "oracle", "sphbuf_oracle.c"), "-lm"], check=True)
    _run(exe)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_geometry_under_sanitizers(tmp_path):
    exe = str(tmp_path / "asan_geometry")
    subprocess.run(["g++", "-std=c++17", *FLAGS, "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2406_16786_amd", "csrc"), "-o", exe,
                    os.path.join(ROOT, "tests", "native", "asan_geometry.cpp"),
                    os.path.join(ROOT, "paper_2406_16786_amd", "csrc", "geometry.cpp")], check=True)
    _run(exe)
