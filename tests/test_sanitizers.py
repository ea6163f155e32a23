"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

A child process loads an instrumented build of the oracle (gcc
-fsanitize=address,undefined, with the ASan runtime preloaded) and runs the
oracle's pins that exercise its C code most -- energies, sweeps on both
schedules, replays, flips, the flexible bodies -- leaving out the slow
statistical ones whose time goes to numpy.  Any out-of-bounds access, leak-free
use after free or undefined behaviour aborts the child with a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    try:
        path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_pass_under_asan_and_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    env = dict(os.environ, FLIPMC_ORACLE_SANITIZE="1", LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    deselect = ("not flip_and_local and not schedules_agree and not replay_checkerboard_every_attempt "
                "and not replay_random_schedule and not rocrand")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-k", deselect,
           "tests/test_oracle_pins.py", "tests/test_flex_pins.py", "tests/test_fs_pins.py"]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out


def _clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_c_abi_host_code_passes_under_asan_and_ubsan(tmp_path):
    # the library's host code (argument checks, geometry, layouts, batch
    # bookkeeping, error paths) instrumented on the host side only; the C-ABI
    # tests that need no device run against it in a child process
    import shutil
    rt = _clang_asan_runtime()
    if rt is None or shutil.which("hipcc") is None:
        pytest.skip("hipcc or clang's AddressSanitizer runtime is not installed")
    sys.path.insert(0, os.path.join(ROOT, "paper_2506_21290_amd"))
    import build as libbuild
    sys.path.pop(0)
    out = str(tmp_path / "libflipmc_san.so")
    flags = [f for f in libbuild.HIPCC_FLAGS if f != "-O3"]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"]
    cmd = ["hipcc", *flags, "-O1", "-g", *host_san, "-I" + os.path.join(ROOT, "include"), *libbuild.SOURCES,
           "-o", out, *libbuild.LINK_FLAGS]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    child = ("import sys; sys.path.insert(0, %r)\n"
             "from paper_2506_21290_amd import flipmc\n"
             "flipmc.LIB_PATH = %r\n"
             "import pytest\n"
             "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', %r]))\n"
             % (ROOT, out, os.path.join(ROOT, "tests", "test_capi.py")))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([sys.executable, "-c", child], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=600)
    text = res.stdout + res.stderr
    assert res.returncode == 0, text[-4000:]
    assert "runtime error" not in text and "AddressSanitizer" not in text, text[-4000:]
    assert " passed" in text
