"""Build libftcg.so for gfx950 in-tree with hipcc.

Every HIP source is compiled with -O3 for gfx950 and with packed-FP32
instructions disabled (-Xclang -target-feature -Xclang -packed-fp32-ops),
then linked into paper_1706_08575_amd/libftcg.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libftcg.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC, *lang, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # keep warnings visible but not the harmless host-pass note about the feature flag
    noise = "packed-fp32-ops"
    warn = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l)
    if warn.strip():
        print(warn, file=sys.stderr)
    return obj


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()


def build_abi_check(verbose: bool = False) -> str:
    """Executable of tests/abi_check.cpp against the library's objects, with the
    host code of the entry-point files (the .cpp sources: argument checks,
    status plumbing, plan lifecycle) and the test program built with
    AddressSanitizer and UndefinedBehaviorSanitizer. Device code is built
    as usual (the sanitizers apply to the host side only); the .hip objects
    come from the regular build. Returns the executable's path."""
    build(verbose=False)
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    host_flags = ["-O1", "-g", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    objs = []
    srcs = [s for s in sources() if s.endswith(".cpp")] + [os.path.join(ROOT, "tests", "abi_check.cpp")]

    def comp(src):
        obj = os.path.join(san, os.path.basename(src) + ".o")
        flags = [f for f in COMMON if f != "-O3"]
        cmd = [HIPCC, "-x", "hip", *flags, *host_flags, "-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    objs += [os.path.join(BUILD, os.path.basename(s) + ".o") for s in sources() if s.endswith(".hip")]
    exe = os.path.join(san, "abi_check")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-fsanitize=address,undefined", "-fno-gpu-sanitize", "-o", exe, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {exe}")
    return exe
