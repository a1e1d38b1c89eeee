"""Build libevs.so (HIP for gfx950) in-tree with hipcc.

Each source is compiled to an object in parallel, then linked into
paper_2508_18071_amd/libevs.so.  Every HIP compile disables packed-FP32
instruction selection.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libevs.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


# Per-source extra flags.  evs_tnet.hip keeps its register rings as 16-dword
# vectors whose 4-dword slices feed the MFMAs in place; LLVM's splitting of
# large vector phis into 32-bit pieces would turn those slices into copies.
EXTRA = {"evs_tnet.hip": ["-mllvm", "-amdgpu-codegenprepare-break-large-phis=false"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA.get(os.path.basename(src), []), "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{msg}")
    return obj, msg


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, srcs))
    if verbose:
        for _, msg in results:
            if msg.strip():
                print(msg)
    objs = [o for o, _ in results]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stdout + r.stderr)
    os.replace(tmp, OUT)
    return OUT


# Host-side sanitizers: the C++ files of the boundary (argument validation,
# workspace sizing, tile cache, entry points) built with AddressSanitizer and
# UndefinedBehaviorSanitizer on their host compilation only, linked with the
# kernel objects of the normal build into _build/libevs_sanitized.so.  Load it
# with EVS_LIB_PATH and the ASan runtime preloaded (see
# tests/test_abi_host_sanitized.py).
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
SAN_OUT = os.path.join(BUILD, "libevs_sanitized.so")


def asan_runtime() -> str:
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        for root in ("/opt/rocm/llvm/lib/clang",):
            for dirpath, _, files in os.walk(root):
                if "libclang_rt.asan-x86_64.so" in files:
                    return os.path.join(dirpath, "libclang_rt.asan-x86_64.so")
        raise RuntimeError("ASan runtime not found")
    return path


def build_sanitized() -> str:
    if not os.path.exists(OUT):
        build()
    os.makedirs(os.path.join(BUILD, "san"), exist_ok=True)
    objs = []
    for src in sources():
        if src.endswith(".cpp"):
            obj = os.path.join(BUILD, "san", os.path.basename(src) + ".o")
            cmd = [HIPCC, *COMMON, *SAN_HOST, "-x", "hip", "-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {src}\n{r.stdout}{r.stderr}")
        else:
            obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        objs.append(obj)
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_HOST, "-shared-libsan", "-o", SAN_OUT, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed\n" + r.stdout + r.stderr)
    return SAN_OUT


if __name__ == "__main__":
    if "--sanitized" in sys.argv:
        print(build_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
