"""Build libqcemu.so (all HIP kernels + the C-ABI) for gfx950 with hipcc.

Objects go to ``_build/`` at the repository root; the shared library is
written next to this file so that it travels with the source tree.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libqcemu.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
if not os.path.exists(HIPCC):
    HIPCC = shutil.which("hipcc") or HIPCC

COMMON_FLAGS = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (the compiler would form them from
    # scalar float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]

SOURCES = ["stats.hip", "split.hip", "gemm.hip", "direct.hip", "permute.hip", "reduce.hip", "group.hip",
           "api.cpp"]


# Host-side sanitizers (the device code is built as usual): AddressSanitizer
# and UndefinedBehaviorSanitizer on the C-ABI layer and the launchers, for a
# separate libqcemu_asan.so loaded through QCE_LIB with the clang ASan
# runtime preloaded.
SANITIZE_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
ASAN_LIB = os.path.join(HERE, "libqcemu_asan.so")


# the compiler's per-kernel resource remarks (registers, scratch, LDS,
# occupancy), kept next to the objects for the build checks in tests/
RESOURCE_REMARKS = "-Rpass-analysis=kernel-resource-usage"
RESOURCES = os.path.join(BUILD, "kernel_resources.txt")


def _compile(src, verbose, sanitize=False):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, ("asan_" if sanitize else "") + src + ".o")
    cmd = [HIPCC, "-x", "hip", *COMMON_FLAGS, *(SANITIZE_FLAGS if sanitize else []), RESOURCE_REMARKS,
           "-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    lines = (res.stdout + res.stderr).splitlines()
    remarks = [l for l in lines if "kernel-resource-usage" in l]
    msgs = "\n".join(l for l in lines if "packed-fp32-ops" not in l and "kernel-resource-usage" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    return obj, remarks


def parse_resources(remarks):
    """{kernel symbol: {"VGPRs": .., "AGPRs": .., "ScratchSize": .., ...}} from
    the compiler's resource remarks."""
    out, cur = {}, None
    for l in remarks:
        body = l.split("remark:", 1)[-1].strip()
        body = body.replace("[-Rpass-analysis=kernel-resource-usage]", "").strip()
        if body.startswith("Function Name:"):
            cur = body.split(":", 1)[1].strip()
            out[cur] = {}
        elif cur and ":" in body:
            key, val = body.split(":", 1)
            key = key.split("[")[0].strip()
            try:
                out[cur][key] = int(val.strip().split()[0])
            except ValueError:
                pass
    return out


def build(verbose=False, jobs=None, sanitize=False):
    """Compile every source and link the shared library (always rebuilds).
    sanitize: the host-sanitizer variant libqcemu_asan.so instead."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        done = list(ex.map(lambda s: _compile(s, verbose, sanitize), SOURCES))
    objs = [o for o, _ in done]
    if not sanitize:
        with open(RESOURCES, "w") as f:
            f.write("\n".join(r for _, rem in done for r in rem) + "\n")
    out = ASAN_LIB if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    link_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-shared-libsan"] if sanitize else []
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *link_san, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, out)
    return out


def asan_runtime():
    """Path of the clang ASan runtime to preload for libqcemu_asan.so."""
    res = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = res.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--asan" in sys.argv))
