"""Host sanitizer builds of the FP64 oracle (CPU only): every oracle routine
runs once on small inputs (tests/sanitize/oracle_driver.c) under
AddressSanitizer + UndefinedBehaviorSanitizer (gcc), and under
ThreadSanitizer over its OpenMP loops (clang with the LLVM OpenMP runtime
and its Archer tool, which tells ThreadSanitizer about OpenMP's
synchronisation).  A planted race in a tiny OpenMP program must be reported,
so a clean oracle run means something."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")
ORACLE = os.path.join(ROOT, "oracle", "oracle.c")
LLVM = "/opt/rocm/lib/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")


def _run(exe, env_extra, tmp):
    env = dict(os.environ, OMP_NUM_THREADS="4", **env_extra)
    return subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300, cwd=tmp)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "orc_asan")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-std=c11", "-D_GNU_SOURCE",
                    "-o", exe, DRIVER, ORACLE, "-lm"], check=True, capture_output=True)
    r = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}, tmp_path)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "clean" in r.stdout


def _tsan_build(src, exe):
    subprocess.run([CLANG, "-O1", "-g", "-fsanitize=thread", "-fopenmp", "-std=c11",
                    "-D_GNU_SOURCE", "-o", exe, *src, "-lm",
                    "-Wl,-rpath," + os.path.join(LLVM, "lib")], check=True, capture_output=True)


TSAN_ENV = {"OMP_TOOL_LIBRARIES": ARCHER,
            "TSAN_OPTIONS": "halt_on_error=1:ignore_noninstrumented_modules=1:report_mutex_bugs=0"}


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                    reason="clang with the LLVM OpenMP runtime and Archer not available")
def test_oracle_openmp_loops_under_tsan(tmp_path):
    planted = tmp_path / "race.c"
    planted.write_text("#include <stdio.h>\nint main(void){long s=0;\n#pragma omp parallel for\n"
                       "for(int i=0;i<100000;++i) s+=i;\nprintf(\"%ld\\n\",s);return 0;}\n")
    _tsan_build([str(planted)], str(tmp_path / "race"))
    r = _run(str(tmp_path / "race"), TSAN_ENV, tmp_path)
    assert r.returncode != 0 and "data race" in r.stderr, "the planted race was not reported"
    exe = str(tmp_path / "orc_tsan")
    _tsan_build([DRIVER, ORACLE], exe)
    r = _run(exe, TSAN_ENV, tmp_path)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "clean" in r.stdout
