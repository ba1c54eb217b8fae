"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
include/dfx.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "dfx.h")
LIB = os.path.join(ROOT, "paper_1707_03771_amd", "libdfx.so")


def declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(dfx_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("dfx_eri3", "dfx_jk", "dfx_scf", "dfx_int1e", "dfx_last_error", "dfx_B_free"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")
def test_argument_errors_are_status_codes():
    import paper_1707_03771_amd as dfx
    lib = dfx._lib
    out = ctypes.c_void_p()
    # empty basis
    assert lib.dfx_eri3(None, 0, None, 0, None, None, 0, None, ctypes.byref(out)) == dfx.EINVAL
    assert "empty" in dfx.last_error()
    # NULL output handle
    assert lib.dfx_eri3(None, 1, None, 1, None, None, 0, None, None) == dfx.EINVAL
    # l beyond the compiled classes is reported before any device work
    e = np.array([1.0]); c = np.array([1.0])
    sh = (dfx.Shell * 1)()
    sh[0].l, sh[0].nprim, sh[0].exps, sh[0].coefs = 4, 1, e.ctypes.data, c.ctypes.data
    ax = (dfx.Shell * 1)()
    ax[0].l, ax[0].nprim, ax[0].exps, ax[0].coefs = 0, 1, e.ctypes.data, c.ctypes.data
    assert lib.dfx_eri3(sh, 1, ax, 1, None, None, 0, None, ctypes.byref(out)) == dfx.EUNSUPPORTED
    sh[0].l = 1
    ax[0].l = 5
    assert lib.dfx_eri3(sh, 1, ax, 1, None, None, 0, None, ctypes.byref(out)) == dfx.EUNSUPPORTED
    # malformed shells
    sh[0].nprim = 0
    ax[0].l = 0
    assert lib.dfx_eri3(sh, 1, ax, 1, None, None, 0, None, ctypes.byref(out)) == dfx.EINVAL
    sh[0].nprim = 1
    neg = np.array([-1.0])
    sh[0].exps = neg.ctypes.data
    assert lib.dfx_eri3(sh, 1, ax, 1, None, None, 0, None, ctypes.byref(out)) == dfx.EINVAL
    # jk / B calls on a NULL handle
    assert lib.dfx_jk(None, None, 1, 1, 0, None, None, None) == dfx.EINVAL
    assert lib.dfx_B_info_get(None, None) == dfx.EINVAL
    # eigen-decomposition: NULL matrix, NULL eigenvalues, empty size
    assert lib.dfx_eigh(None, 4, None, None, None) == dfx.EINVAL
    assert lib.dfx_eigh(ctypes.c_void_p(16), 0, ctypes.c_void_p(16), None, None) == dfx.EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")
def test_eri3_plan_sizes_host_only():
    """dfx_eri3_plan touches no GPU: counts and byte sizes from the shells."""
    import paper_1707_03771_amd as dfx
    import workloads as W
    _, _, sh, ax = W.workload("h4")
    z = dfx.eri3_plan(sh, ax)
    assert (z["nbf"], z["naux"], z["ncols_tiled"]) == (24, 100, 1024)
    assert z["bytes_B"] == 2 * 100 * 1024 * 4
    # every pair a >= b of 16 shells (4 x (3s 1p) on H): raw columns (24^2 + 4 (3 + 9)) / 2
    assert 0 <= z["bytes_raw"] - 100 * ((24 * 24 + 4 * 12) // 2) * 8 < 256
    assert 0 <= z["bytes_metric"] - 2 * 100 * 100 * 8 < 2 * 256  # J_PQ and L, each 256-byte aligned
    assert z["bytes_workspace"] >= z["bytes_persistent"] + z["bytes_jk"]
    assert z["bytes_persistent"] >= z["bytes_B"] + 100 * 100 * 8
    zk = dfx.eri3_plan(sh, ax, flags=dfx.KEEP_RAW | dfx.KEEP_METRIC)
    assert zk["bytes_persistent"] >= z["bytes_persistent"] + z["bytes_raw"] + 100 * 100 * 8
    _, _, sh, ax = W.workload("water4")
    z = dfx.eri3_plan(sh, ax)
    nt = 1536 // 32
    assert (z["nbf"], z["naux"], z["ncols_tiled"]) == (1536, 6784, nt * (nt + 1) // 2 * 1024)
    # B (65 GB) + raw bound (64 GB) + metric, well inside one GPU's 288 GB
    assert 1.2e11 < z["bytes_workspace"] < 1.6e11
    with pytest.raises(dfx.DfxError) as e:
        dfx.eri3_plan([], ax)
    assert e.value.code == dfx.EINVAL
    bad = [dict(sh[0], l=4)]
    with pytest.raises(dfx.DfxError) as e:
        dfx.eri3_plan(bad, ax)
    assert e.value.code == dfx.EUNSUPPORTED


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")
def test_open_shell_and_mp2_argument_errors_before_device_work():
    """dfx_uhf / dfx_rohf / dfx_scf / dfx_mp2 validate their arguments before any
    HIP call: NULL pointers, a multiplicity whose parity does not match the
    electron count or that exceeds it, a negative level shift, a level shift
    given to RHF, options the open-shell drivers do not support."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import systems
    import paper_1707_03771_amd as dfx
    lib = dfx._lib
    E = ctypes.c_double()
    assert lib.dfx_uhf(None, None, 0, None, 0, None, 1, ctypes.byref(E), None, None, None) == dfx.EINVAL
    assert lib.dfx_rohf(None, None, 0, None, 0, None, 1, ctypes.byref(E), None, None, None) == dfx.EINVAL
    assert lib.dfx_mp2(None, None, 1, None, 1, 0, ctypes.byref(E), None) == dfx.EINVAL
    xyz, Z, sh, ax, _ = systems.h4()                   # 4 electrons
    for fn in (dfx.uhf, dfx.rohf):
        for kw in (dict(multiplicity=2), dict(multiplicity=6), dict(multiplicity=0),
                   dict(multiplicity=1, level_shift=-0.5), dict(multiplicity=1, schedule=dfx.SCHED_MIXED),
                   dict(multiplicity=1, guess=dfx.GUESS_DENSITY)):
            with pytest.raises(dfx.DfxError) as e:
                fn(xyz, Z, sh, ax, want_c=False, **kw)
            assert e.value.code == dfx.EINVAL, kw
    with pytest.raises(dfx.DfxError) as e:
        dfx.scf(xyz, Z, sh, ax, want_c=False, level_shift=0.3)
    assert e.value.code == dfx.EINVAL and "level_shift" in dfx.last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdfx.so not built")
def test_undersized_workspace_is_enomem_before_device_work():
    """A caller's workspace smaller than the plan is refused with DFX_ENOMEM
    before anything touches the device (the pointer here is not device memory
    and is never dereferenced); a NULL workspace is DFX_EINVAL."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import systems
    import paper_1707_03771_amd as dfx
    lib = dfx._lib
    xyz, Z, sh, ax, _ = systems.h4()
    s, a = dfx._ShellArray(sh), dfx._ShellArray(ax)
    need = dfx.eri3_plan(sh, ax)["bytes_workspace"]
    fake = ctypes.c_void_p(0x100000)
    out = ctypes.c_void_p()
    for short in (0, 1, need // 2, need - 1):
        assert lib.dfx_eri3(s.arr, s.n, a.arr, a.n, None, fake, short, None, ctypes.byref(out)) == dfx.ENOMEM
        assert "workspace" in dfx.last_error() and str(need) in dfx.last_error()
        assert not out.value
    assert lib.dfx_eri3(s.arr, s.n, a.arr, a.n, None, None, need, None, ctypes.byref(out)) == dfx.EINVAL
    # kept raw integrals need more
    keep = dfx.Eri3Opts(1e-12, dfx.KEEP_RAW)
    assert lib.dfx_eri3(s.arr, s.n, a.arr, a.n, ctypes.byref(keep), fake, need, None, ctypes.byref(out)) == dfx.ENOMEM
    # the SCF drivers check opts.workspace the same way
    sneed = dfx.scf_plan(sh, ax, len(Z))
    assert sneed > need
    g = dfx._GeomC(xyz, Z)
    E = ctypes.c_double()
    o = dfx.scf_default_opts()
    o.workspace, o.ws_bytes = 0x100000, sneed - 1
    assert lib.dfx_scf(ctypes.byref(g.g), s.arr, s.n, a.arr, a.n, ctypes.byref(o), None, ctypes.byref(E),
                       None, None, None) == dfx.ENOMEM
    assert "dfx_scf_plan" in dfx.last_error()
    for fn in (lib.dfx_uhf, lib.dfx_rohf):
        assert fn(ctypes.byref(g.g), s.arr, s.n, a.arr, a.n, ctypes.byref(o), 1, ctypes.byref(E), None, None,
                  None) == dfx.ENOMEM


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets of
    the C struct it mirrors, as a C compiler lays the header out."""
    import shutil
    import subprocess
    import paper_1707_03771_amd as dfx
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [(dfx.Shell, "dfx_shell"), (dfx.Geom, "dfx_geom"), (dfx.Eri3Opts, "dfx_eri3_opts"),
             (dfx.BInfo, "dfx_B_info"), (dfx.Eri3Sizes, "dfx_eri3_sizes"), (dfx.ScfOpts, "dfx_scf_opts"),
             (dfx.ScfInfo, "dfx_scf_info"), (dfx.GradInfo, "dfx_grad_info"), (dfx.GuessSpec, "dfx_guess_spec")]
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "dfx.h"', "int main(void) {"]
    want = []
    for cls, cname in pairs:
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        want.append(ctypes.sizeof(cls))
        for f in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {f[0]}));')
            want.append(getattr(cls, f[0]).offset)
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert got == want
