"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the BVH builder with an invariant-checking driver, and the FP64
oracle with its pins run against a sanitizer build of the same source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
       "-fno-sanitize-recover=all"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip("no %s in this toolchain" % name)
    return p


def test_bvh_builder_under_sanitizers(tmp_path):
    exe = str(tmp_path / "bvh_check")
    subprocess.check_call(["g++"] + SAN + [os.path.join(ROOT, "tests", "sanitize", "bvh_check.cpp"),
                                           os.path.join(ROOT, "paper_2606_14173_amd", "csrc", "bvh_build.cpp"),
                                           "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "ALL OK" in r.stdout


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++"] + SAN + ["-fopenmp", "-shared", "-fPIC", "-o", lib,
                                           os.path.join(ROOT, "oracle", "hpt_oracle.cpp")])
    env = dict(os.environ)
    pre = [_runtime("libasan.so"), _runtime("libubsan.so")] + ([env["LD_PRELOAD"]] if env.get("LD_PRELOAD") else [])
    env.update(HPT_ORACLE_LIB=lib, LD_PRELOAD=":".join(pre), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    pins = ["tests/test_oracle_pins.py", "tests/test_point_emitter_pins.py", "tests/test_nee_pins.py",
            "tests/test_principled_pins.py"]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] + pins,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    print(r.stdout[-3000:], r.stderr[-4000:])
    assert r.returncode == 0, "oracle pins failed under the sanitizers"
    # the sanitizer build was the one loaded
    chk = subprocess.run([sys.executable, "-c", "import oracle._lib as L; L.lib(); import os; "
                          "print([l for l in open('/proc/self/maps') if 'liboracle_san' in l][:1])"],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert "liboracle_san" in chk.stdout
