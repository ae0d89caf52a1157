"""Build libltrk.so (HIP for gfx950) in-tree: paper_1610_05801_amd/libltrk.so.

    python -m paper_1610_05801_amd.build
    python -m paper_1610_05801_amd.build --sanitize-host OUT_DIR

Every HIP source is compiled with -ffp-contract=off (the kernels spell out
their fma() calls, so rounding is fixed by the source) and without packed
FP32 instruction selection. --sanitize-host builds a copy into OUT_DIR whose
host code (argument checks, plans, scratch and graph caches, the engine's
bookkeeping) carries AddressSanitizer and UndefinedBehaviorSanitizer checks;
device code is built as usual. Load it with LTRK_LIBRARY=OUT_DIR/libltrk.so
in a process that preloads the ASan runtime (printed by the build).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libltrk.so")
SOURCES = ["kernels.hip", "kernels_ext.hip", "kernels_wake.hip", "runtime.hip", "tune.hip",
           "engine.hip"]
ARCH = os.environ.get("LTRK_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libltrk)")


def flags() -> list:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-value", "-Wno-unused-result",
            "-I" + os.path.join(HERE, "..", "include")]


# host-only sanitizer flags: every -fsanitize applies to the host pass alone
SANITIZE_HOST = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-omit-frame-pointer -g").split()


def _compile(src: str, obj_dir: str = OBJ, extra: tuple = ()) -> str:
    out = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc()] + flags() + list(extra) + ["-c", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("compiling %s failed:\n%s%s" % (src, res.stdout, res.stderr))
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("linking libltrk.so failed:\n%s%s" % (res.stdout, res.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized(out_dir: str) -> str:
    """The library with host-side ASan and UBSan into out_dir; returns its path."""
    obj = os.path.join(out_dir, "_build")
    os.makedirs(obj, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(lambda s: _compile(s, obj, SANITIZE_HOST), SOURCES))
    lib = os.path.join(out_dir, "libltrk.so")
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-shared-libasan"] + \
        SANITIZE_HOST[:4] + ["-o", lib] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("linking the sanitized libltrk.so failed:\n%s%s" %
                           (res.stdout, res.stderr))
    rt = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    print("built %s\nASan runtime to preload: %s" % (lib, rt))
    return lib


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--sanitize-host":
        build_sanitized(os.path.abspath(sys.argv[2]))
    else:
        build(verbose=True)
    sys.exit(0)
