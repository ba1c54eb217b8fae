"""The oracle's C integral engine under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU).

md_ints.c is rebuilt with -fsanitize=address,undefined into a temporary
directory, and a child Python process loads that build (DFX_ORACLE_LIB) with
the sanitizer runtime preloaded.  The child runs every entry point of the C
engine on a small molecule with orbital l <= 3 and auxiliary l <= 4 shells and
contracted shells: the packed three-index integrals, the metric, the Schwarz
factors, the one-electron integrals, the four-index block, and the
derivative integrals of the gradient.  Any out-of-bounds access, use after
free or undefined behaviour aborts the child with the sanitizer's report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, ROOT); sys.path.insert(0, ROOT + "/tests")
import oracle as O
from oracle import grad as G
import systems
xyz, Z, sh, ax = systems.mixed_molecule(seed=2, natom=2, lorb=3, laux=4)
bas, aux = O.Basis(sh), O.Basis(ax)
Qab, QC = O.schwarz(bas, aux)
scr = O.screen(bas, aux, Qab, QC, 1e-12)
raw = O.eri3_packed(bas, aux, scr)
J2 = O.eri2(aux)
S, T, V = O.int1e(bas, xyz, Z)
blk = O.eri4_block(bas, 1, 0, 2, 1)
d3 = G.eri3_deriv_block(bas, 3, 1, aux, 4)
d2 = G.eri2_deriv_block(aux, 2, 5)
rng = np.random.default_rng(0)
C = np.linalg.qr(rng.normal(size=(bas.nbf, 3)))[0]
eps = -np.arange(1.0, 4.0)
g, parts = G.df_rhf_gradient(Z, xyz, sh, ax, C, eps)
assert np.isfinite(raw).all() and np.isfinite(g).all()
print("sanitized oracle ok", raw.shape, J2.shape, float(np.abs(g).max()))
"""


def _runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True, check=True)
    except (OSError, subprocess.CalledProcessError):
        return None
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    rt = _runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build(out=str(tmp_path / "liboracle_asan.so"), sanitize=True)
    env = dict(os.environ, LD_PRELOAD=rt, DFX_ORACLE_LIB=lib, OMP_NUM_THREADS="1",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", f"ROOT = {ROOT!r}\n" + CHILD], env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, report
    assert "sanitized oracle ok" in r.stdout


def _clang_asan():
    import glob
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.slow
def test_host_library_under_address_sanitizer(tmp_path):
    """The library's host C++ (the C-ABI's argument checks, shell setup, plans,
    arena sizing, run log) built with AddressSanitizer: the CPU boundary tests
    run against that build in a child process (a copy of the binding next to
    the sanitized library), and must pass with no sanitizer report."""
    import shutil
    rt = _clang_asan()
    if rt is None:
        pytest.skip("the compiler's AddressSanitizer runtime is not installed")
    sys.path.insert(0, ROOT)
    try:
        from paper_1707_03771_amd import build as pb
    except ImportError:
        import importlib.util
        spec = importlib.util.spec_from_file_location("dfx_build", os.path.join(ROOT, "paper_1707_03771_amd", "build.py"))
        pb = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(pb)
    lib = pb.build_host_asan(verbose=False)
    pkg = tmp_path / "paper_1707_03771_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_1707_03771_amd", "__init__.py"), pkg / "__init__.py")
    shutil.copy(lib, pkg / "libdfx.so")
    env = dict(os.environ, LD_PRELOAD=rt, PYTHONPATH=f"{tmp_path}{os.pathsep}{ROOT}",
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0:abort_on_error=1")
    probe = ("import paper_1707_03771_amd as m, os; "
             "assert os.path.dirname(m.LIB_PATH) == os.path.join(os.environ['PYTHONPATH'].split(os.pathsep)[0], "
             "'paper_1707_03771_amd'), m.LIB_PATH; print('sanitized library', m.LIB_PATH)")
    r = subprocess.run([sys.executable, "-c", probe], env=env, capture_output=True, text=True, timeout=300,
                       cwd=str(tmp_path))
    assert r.returncode == 0 and "sanitized library" in r.stdout, r.stderr[-4000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_runlog.py")],
                       env=env, capture_output=True, text=True, timeout=900, cwd=str(tmp_path))
    out = r.stdout[-3000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr, out
    assert " passed" in r.stdout and "failed" not in r.stdout, out
