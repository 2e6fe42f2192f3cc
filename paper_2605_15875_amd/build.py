"""Build libabd.so for gfx950 in-tree.

    python -m paper_2605_15875_amd.build

Each HIP source is compiled to an object under _build/ and linked into
paper_2605_15875_amd/libabd.so.  Packed FP32 instructions are disabled
and FP64 atomics use the hardware instructions.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libabd.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["kernels.hip", "runtime.hip"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"),
         "-Wno-unused-result"]


# host-code sanitizer for libabd_san.so: UndefinedBehaviorSanitizer on the
# host pass only (the GPU code is built as in libabd.so).  The clang
# AddressSanitizer runtime intercepts the HSA memory-pool allocator and
# fails its first device allocation with the ROCm runtime of this image,
# so the host runtime runs under UBSan only
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
             "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
LIB_SAN = os.path.join(HERE, "libabd_san.so")


def _compile(src, san=False):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ("_san.o" if san else ".o"))
    cmd = [HIPCC, *FLAGS, *(SAN_FLAGS if san else []), "-c", os.path.join(CSRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """libabd.so, or (sanitize) libabd_san.so with UndefinedBehaviorSanitizer
    on the host code (run with the clang UBSan runtime preloaded and ABD_LIB
    pointing at it)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize), SOURCES))
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
