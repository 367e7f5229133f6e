"""The oracle, the host planner (csrc/ss_plan.cpp) and the serving arena's allocator (csrc/ss_arena.h)
built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only) and driven over random and
edge-case inputs (tests/sanitize/drive.cpp): empty pairs, thresholds beyond the length, unequal
lengths, sub-maze widths, threaded batches, plans of every slice width.  Any memory error or
undefined behaviour aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
HIPCC = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not (os.path.exists(CLANG) and os.path.exists(CLANGXX) and os.path.exists(HIPCC)):
        pytest.skip("ROCm clang toolchain not found")
    d = tmp_path_factory.mktemp("san")
    objs = []
    o = str(d / "oracle.o")
    subprocess.check_call([CLANG, "-O1", "-g", "-fPIC", *SAN, "-c", os.path.join(ROOT, "oracle", "ss_oracle.c"),
                           "-o", o])
    objs.append(o)
    o = str(d / "ss_plan.o")
    # the host planner (host code only), every sanitizer flag scoped to the host pass
    host_san = [x for f in SAN for x in ("-Xarch_host", f)]
    subprocess.check_call([HIPCC, "--offload-host-only", "-x", "hip", "-O1", "-std=c++17", "-fPIC", "-Xarch_host", "-g",
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1910_09020_amd", "csrc"),
                           *host_san, "-c", os.path.join(ROOT, "paper_1910_09020_amd", "csrc", "ss_plan.cpp"),
                           "-o", o])
    objs.append(o)
    o = str(d / "drive.o")
    subprocess.check_call([CLANGXX, "-O1", "-g", "-std=c++17", *SAN, "-I",
                           os.path.join(ROOT, "paper_1910_09020_amd", "csrc"), "-c",
                           os.path.join(ROOT, "tests", "sanitize", "drive.cpp"), "-o", o])
    objs.append(o)
    exe = str(d / "drive")
    subprocess.check_call([CLANGXX, *SAN, *objs, "-o", exe, "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lpthread"])
    return exe


def test_oracle_and_planner_clean_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized drive: ok" in r.stdout


def test_the_sanitizers_are_live(tmp_path):
    """A heap overflow planted in a tiny host program built with the same flags is reported (the
    sanitizer runtime is really in the builds above)."""
    if not os.path.exists(CLANGXX):
        pytest.skip("ROCm clang toolchain not found")
    src = tmp_path / "planted.cpp"
    src.write_text("#include <vector>\nint main(int c, char**) { std::vector<int> v(4); return v.data()[3 + c]; }\n")
    exe = str(tmp_path / "planted")
    subprocess.check_call([CLANGXX, "-O0", "-g", *SAN, str(src), "-o", exe])
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=60)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_copy_crew_clean_under_thread_sanitizer(tmp_path):
    """The host copy crew of the serving submissions (csrc/ss_copy.h) driven by six threads at once
    under ThreadSanitizer (tests/sanitize/copy_crew.cpp): no data race is reported and every copy is
    exact.  A race planted in a tiny program built with the same flags is reported (the runtime is
    live)."""
    if not os.path.exists(CLANGXX):
        pytest.skip("ROCm clang toolchain not found")
    tsan = ["-O1", "-g", "-std=c++17", "-fsanitize=thread"]
    exe = str(tmp_path / "copy_crew")
    subprocess.check_call([CLANGXX, *tsan, "-I", os.path.join(ROOT, "paper_1910_09020_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sanitize", "copy_crew.cpp"), "-o", exe, "-lpthread"])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "copy crew: ok" in r.stdout
    src = tmp_path / "race.cpp"
    src.write_text("#include <thread>\nint x = 0;\nint main() { std::thread a([] { x++; }), b([] { x++; });\n"
                   "a.join(); b.join(); return 0; }\n")
    race = str(tmp_path / "race")
    subprocess.check_call([CLANGXX, *tsan, str(src), "-o", race, "-lpthread"])
    r = subprocess.run([race], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=60)
    assert r.returncode != 0 and "data race" in r.stderr
