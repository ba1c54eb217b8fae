"""Build libdfx.so for gfx950 from csrc/ (HIP kernels + C-ABI host code).

    python paper_1707_03771_amd/build.py [--force] [-j N]

Objects go to <repo>/_build/, the library to paper_1707_03771_amd/libdfx.so.
Sources are recompiled when they, or any header in csrc/ or include/, are newer
than their object (``--force`` recompiles everything).
"""
import argparse
import concurrent.futures as cf
import glob
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdfx.so")
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Wno-unused-variable", "-Wno-unknown-pragmas",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]
LIBS = ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _includes(path, seen):
    """Local headers reached from path through #include "..." (recursive)."""
    import re
    for inc in re.findall(r'^\s*#\s*include\s+"([^"]+)"', open(path).read(), re.M):
        for base in (os.path.dirname(path), CSRC, os.path.join(ROOT, "include")):
            q = os.path.normpath(os.path.join(base, inc))
            if os.path.exists(q):
                if q not in seen:
                    seen.add(q)
                    _includes(q, seen)
                break
    return seen


def deps_mtime(src):
    return max([os.path.getmtime(src)] + [os.path.getmtime(h) for h in _includes(src, set())])


def obj_of(src):
    return os.path.join(BUILD, os.path.basename(src) + ".o")


def compile_one(src, verbose):
    out = obj_of(src)
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", out + ".tmp"]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", src, "-o", out + ".tmp"]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"compile failed: {os.path.basename(src)}\n{msg}")
    os.replace(out + ".tmp", out)
    if verbose:
        print(f"  {os.path.basename(src)}: {time.time() - t:.1f} s", flush=True)
    return out


def build(force=False, jobs=None, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if force or not os.path.exists(obj_of(s))
            or os.path.getmtime(obj_of(s)) < deps_mtime(s)]
    jobs = jobs or min(16, os.cpu_count() or 4)
    # the heaviest translation units first
    todo.sort(key=lambda s: -os.path.getsize(s) - (10 ** 6 if "eri3_l3" in s or "eri3_l2" in s else 0))
    if todo:
        if verbose:
            print(f"compiling {len(todo)} of {len(srcs)} sources with {jobs} jobs", flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda s: compile_one(s, verbose), todo))
    objs = [obj_of(s) for s in srcs]
    if todo or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(o) for o in objs):
        cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", LIB + ".tmp"] + objs + LIBS
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
        if verbose:
            print("linked", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    try:
        build(force=a.force, jobs=a.j)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
