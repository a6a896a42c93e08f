"""The oracle's C loops (oracle.c) built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, every UB check fatal), and the oracle's
own CPU tests run against that build in a child process: no out-of-bounds
access, use after free or undefined behaviour in the checker."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if shutil.which("gcc") is None or asan is None:
        pytest.skip("gcc with AddressSanitizer runtime not available")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(lib), "-lm"], check=True)
    env = dict(os.environ)
    env.update({"QCE_ORACLE_LIB": str(lib), "LD_PRELOAD": asan,
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1", "UBSAN_OPTIONS": "print_stacktrace=1"})
    # the child processes load this build, with the sanitizer runtime active
    probe = subprocess.run([sys.executable, "-c", "import oracle.core as c; c._clib(); "
                            "print(open('/proc/self/maps').read())"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0, probe.stderr[-2000:]
    assert str(lib) in probe.stdout and "libasan" in probe.stdout
    tests = [os.path.join(ROOT, "tests", f) for f in
             ("test_oracle_cgemm.py", "test_oracle_split.py", "test_oracle_stats.py", "test_oracle_circuit.py")]
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
