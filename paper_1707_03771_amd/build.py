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


# Sources compiled once per combination of defines: the derivative integral
# classes (one orbital class (LA, LB) >= and one moved centre and axis per
# object, so that the heavy instantiations build in parallel) and the metric
# derivatives (one axis per object).
VARIANTS = {
    "grad3_class.hip": [dict(GRAD_LA=la, GRAD_LB=lb, GRAD_W=w, GRAD_AX=ax)
                        for la in range(4) for lb in range(la + 1) for w in range(2) for ax in range(3)],
    "grad2_class.hip": [dict(GRAD_AX=ax) for ax in range(3)],
}


class Unit:
    """One object file: a source and the defines it is compiled with."""

    def __init__(self, src, defs=None):
        self.src, self.defs = src, defs or {}
        tag = "".join(f"_{k.split('_')[-1].lower()}{v}" for k, v in self.defs.items())
        self.obj = os.path.join(BUILD, os.path.basename(src) + tag + ".o")

    def cost(self):
        # the heaviest translation units first
        big = ("eri3_l3" in self.src or "eri3_l2" in self.src or
               (self.defs.get("GRAD_LA", 0) >= 2 and "grad3" in self.src))
        return -os.path.getsize(self.src) - (10 ** 6 if big else 0) - 1000 * self.defs.get("GRAD_LA", 0) \
            - 100 * self.defs.get("GRAD_LB", 0)


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def units():
    out = []
    for s in sources():
        name = os.path.basename(s)
        if name in VARIANTS:
            out += [Unit(s, d) for d in VARIANTS[name]]
        else:
            out.append(Unit(s))
    return out


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


def compile_one(u, verbose):
    src, out = u.src, u.obj
    defs = [f"-D{k}={v}" for k, v in u.defs.items()]
    cmd = [HIPCC] + FLAGS + defs + ["-c", src, "-o", out + ".tmp"]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + FLAGS + defs + ["-x", "hip", "-c", src, "-o", out + ".tmp"]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        msg = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"compile failed: {os.path.basename(src)}\n{msg}")
    os.replace(out + ".tmp", out)
    if verbose:
        print(f"  {os.path.basename(out)}: {time.time() - t:.1f} s", flush=True)
    return out


def build(force=False, jobs=None, verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    us = units()
    todo = [u for u in us if force or not os.path.exists(u.obj) or os.path.getmtime(u.obj) < deps_mtime(u.src)]
    jobs = jobs or min(16, os.cpu_count() or 4)
    todo.sort(key=lambda u: u.cost())
    if todo:
        if verbose:
            print(f"compiling {len(todo)} of {len(us)} objects with {jobs} jobs", flush=True)
        with cf.ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda u: compile_one(u, verbose), todo))
    objs = [u.obj for u in us]
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
