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
LIBS = ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"]


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
        """Sort key, heaviest first: the integral classes' compile time grows
        like the square of their Cartesian block (measured: f f ERIs ~280 s,
        their derivatives ~400 s per centre and axis)."""
        import re
        nc = lambda l: (l + 1) * (l + 2) // 2  # noqa: E731
        m = re.search(r"eri3_l(\d)(\d)\.hip$", self.src)
        if m:
            return -2.8 * (nc(int(m.group(1))) * nc(int(m.group(2)))) ** 2 / 100.0
        if "grad3" in self.src:
            la, lb = self.defs["GRAD_LA"], self.defs["GRAD_LB"]
            return -4.0 * (nc(la) * nc(lb)) ** 2 / 100.0
        return -os.path.getsize(self.src) / 1000.0


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


ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(BUILD, "libdfx_asan.so")
# host code only: -Xarch_host before each sanitizer flag keeps device code as it is
ASAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_asan(jobs=None, verbose=True):
    """A second library for the sanitizer test: the host C++ sources (*.cpp:
    the C-ABI, argument checks, plans, arenas, the gradient driver, the guess's
    geometry code) built with AddressSanitizer, linked with the regular objects
    of the HIP sources into _build/libdfx_asan.so.  The package never loads
    it; a process that does must preload the compiler's ASan runtime, which
    resolves the instrumentation's symbols."""
    build(jobs=jobs, verbose=verbose)
    os.makedirs(ASAN_DIR, exist_ok=True)
    objs = []
    for u in units():
        if not u.src.endswith(".cpp"):
            objs.append(u.obj)
            continue
        out = os.path.join(ASAN_DIR, os.path.basename(u.obj))
        if not os.path.exists(out) or os.path.getmtime(out) < deps_mtime(u.src):
            cmd = [HIPCC] + FLAGS + ASAN_FLAGS + ["-x", "hip", "-c", u.src, "-o", out + ".tmp"]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {os.path.basename(u.src)} (asan)\n{r.stderr}")
            os.replace(out + ".tmp", out)
            if verbose:
                print(f"  asan/{os.path.basename(out)}", flush=True)
        objs.append(out)
    if not os.path.exists(ASAN_LIB) or os.path.getmtime(ASAN_LIB) < max(os.path.getmtime(o) for o in objs):
        subprocess.check_call([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", ASAN_LIB + ".tmp"] + objs + LIBS)
        os.replace(ASAN_LIB + ".tmp", ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("--host-asan", action="store_true", help="also build _build/libdfx_asan.so")
    a = ap.parse_args()
    try:
        build(force=a.force, jobs=a.j)
        if a.host_asan:
            build_host_asan(jobs=a.j)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)
