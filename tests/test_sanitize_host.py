"""The library's host code (C-ABI layer, planners, launchers) built with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged),
and the ABI tests run against that build in a child process with the clang
ASan runtime preloaded.  Without a GPU this covers argument checking and
the export table.  (Loaded the same way in a GPU process, the build aborts
inside the first handle creation with no sanitizer report -- ASan's
address-space layout and the HIP runtime's reservations do not coexist on
the GPU machine -- so the GPU tier does not run under it.)"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_code_under_asan_ubsan():
    from paper_2303_08989_amd import build
    rt = build.asan_runtime()
    if rt is None:
        pytest.skip("clang ASan runtime not found")
    lib = build.build(sanitize=True)
    env = dict(os.environ)
    env.update({"QCE_LIB": lib, "LD_PRELOAD": rt, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1"})
    probe = subprocess.run([sys.executable, "-c", "from paper_2303_08989_amd import _lib; _lib.load(); "
                            "print(open('/proc/self/maps').read())"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert "libqcemu_asan.so" in probe.stdout and "libclang_rt.asan" in probe.stdout
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
