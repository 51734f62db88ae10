"""Build ``librefl.so`` (the C-ABI reflector library) for gfx950 with hipcc.

Every source under ``csrc/`` is compiled in parallel into ``_build/`` at the
repository root and linked in-tree as ``paper_2605_24840_amd/librefl.so``.
With ``debug=True`` the same sources are compiled with ``-DREFL_DEBUG`` (the
kernels' launch-extent guards, see csrc/dbg.h) into ``_build/debug/`` and
linked as ``paper_2605_24840_amd/librefl_debug.so``.
"""
import concurrent.futures as cf
import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "librefl.so")
DEBUG_OUT = os.path.join(PKG, "librefl_debug.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions stay disabled (they are generated from ordinary
# float code otherwise); the host pass warns that it does not know the
# feature, which is harmless.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-pass-failed",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def _compile(src: str, debug: bool = False) -> str:
    obj = os.path.join(BUILD, "debug" if debug else "", os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + (["-DREFL_DEBUG"] if debug else []) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8, debug: bool = False) -> str:
    out = DEBUG_OUT if debug else OUT
    os.makedirs(os.path.join(BUILD, "debug") if debug else BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda src: _compile(src, debug), srcs))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} from {len(srcs)} sources", flush=True)
    return out


if __name__ == "__main__":
    import sys
    build(verbose=True, debug="--debug" in sys.argv[1:])
