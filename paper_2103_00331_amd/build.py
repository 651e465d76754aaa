"""Build libcpmdp.so (HIP for gfx950) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); hipcc's host pass warns
that it does not know the feature, which is harmless.

`build.py --sanitize` builds libcpmdp_san.so instead: the host code (argument
checks, factor classification, layouts, the Tucker -> Tensor-Train rewrite,
the CP-fit host solves, the batch and solver bookkeeping) with AddressSanitizer
and UndefinedBehaviorSanitizer, the device code as usual.  Run the CPU tests
against it with `run_sanitized.sh` beside this file.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libcpmdp.so")
LIB_SAN = os.path.join(PKG, "libcpmdp_san.so")
# host pass only: each sanitizer flag behind -Xarch_host
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-g"]

SOURCES = ["api.cpp", "batch.hip", "stencil.hip", "chain.hip", "chain16.hip", "util.hip", "lists.hip", "tt.hip", "cpfit.hip",
           "mlp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CPMDP_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def _compile(src, san=False):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + (".san.o" if san else ".o"))
    flags = COMMON + (SAN_FLAGS if san else [])
    cmd = [HIPCC] + flags + ["-c", path, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + flags + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose=False, sanitize=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, sanitize), srcs))
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp"
    # a sanitizer build leaves the runtime's symbols undefined: the process
    # that loads it preloads the ASan runtime (which carries UBSan's too)
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv[1:])
    sys.exit(0)
