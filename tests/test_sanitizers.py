"""AddressSanitizer + UndefinedBehaviorSanitizer builds of host code (CPU): the library's
posting-list codec and quantisers, and the FP64 oracle, each driven by a small program
under tests/sanitize/ that checks its own results. The library's device-facing runtime and
the serving loop need the HIP runtime and a GPU, and GPU sanitizers are not available, so
they are covered by the GPU tests instead."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1", "-std=c++17"]

cxx = shutil.which("g++")
pytestmark = pytest.mark.skipif(cxx is None, reason="no C++ compiler")


def build_and_run(tmp_path, name, sources, extra=()):
    exe = str(tmp_path / name)
    subprocess.run([cxx, *SAN, *extra, *sources, "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")


def test_library_host_codec_and_quantisers_under_asan_ubsan(tmp_path):
    csrc = os.path.join(ROOT, "paper_2511_22460_amd", "csrc")
    build_and_run(tmp_path, "host_codec",
                  [os.path.join(HERE, "host_codec_main.cpp"), os.path.join(csrc, "codec.cpp"),
                   os.path.join(csrc, "quant.cpp")],
                  ["-I", csrc, "-I", os.path.join(ROOT, "include")])


def test_oracle_under_asan_ubsan(tmp_path):
    build_and_run(tmp_path, "oracle",
                  [os.path.join(HERE, "oracle_main.cpp"), os.path.join(ROOT, "oracle", "oracle.cpp")],
                  ["-fopenmp"])
