"""dfx: density-fitted restricted Hartree-Fock hot path for AMD MI355X (gfx950).

Thin Python binding over the C-ABI of ``libdfx.so`` (include/dfx.h).  Every
step of the computation runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch supplies device memory and the current stream.
Importing fails loudly if the library has not been built
(``python paper_1707_03771_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import json
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdfx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1707_03771_amd/build.py`")

# torch first: its HIP runtime is then the one libdfx.so binds to (same soname).
# Loaded the other way round, the process holds two HIP/HSA runtimes and torch's
# finds no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EHIP, ENOTPOSDEF, ENOCONV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, BF16 = 0, 1, 2
DENSITY, COCC = 0, 1
KEEP_RAW, KEEP_METRIC = 1, 2
EXPORT_B, EXPORT_BHI, EXPORT_RAW = 0, 1, 2
GUESS_CORE, GUESS_CINIT, GUESS_DENSITY, GUESS_LEARNED = 0, 1, 2, 3
SCHED_FP64, SCHED_MIXED = 0, 1
MAXHIST = 256


class DfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dfx error {code}: {msg}")
        self.code = code


class Shell(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_double * 3), ("l", ctypes.c_int32), ("nprim", ctypes.c_int32),
                ("exps", ctypes.c_void_p), ("coefs", ctypes.c_void_p)]


class Geom(ctypes.Structure):
    _fields_ = [("natom", ctypes.c_int32), ("xyz", ctypes.c_void_p), ("Z", ctypes.c_void_p),
                ("charge", ctypes.c_int32)]


class Eri3Opts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("flags", ctypes.c_int32)]


class BInfo(ctypes.Structure):
    _fields_ = [("nbf", ctypes.c_int32), ("naux", ctypes.c_int32), ("nsh", ctypes.c_int32),
                ("nauxsh", ctypes.c_int32), ("npairs", ctypes.c_int32), ("ncols", ctypes.c_int64),
                ("ncols_tiled", ctypes.c_int64), ("ntriplets", ctypes.c_int64),
                ("nintegrals", ctypes.c_int64), ("eri_seconds", ctypes.c_double),
                ("metric_seconds", ctypes.c_double), ("trsm_seconds", ctypes.c_double),
                ("kappa_lb", ctypes.c_double), ("trsm_update_seconds", ctypes.c_double),
                ("trsm_update_flops", ctypes.c_double), ("trsm_update_launches", ctypes.c_int32)]


class ScfOpts(ctypes.Structure):
    _fields_ = [("tau", ctypes.c_double), ("conv_dE", ctypes.c_double), ("conv_err", ctypes.c_double),
                ("ortho_thresh", ctypes.c_double), ("switch_err", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("diis_size", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("mixed_prec", ctypes.c_int32), ("guess", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("switch_auto", ctypes.c_int32), ("purify", ctypes.c_int32),
                ("level_shift", ctypes.c_double), ("workspace", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class ScfInfo(ctypes.Structure):
    _fields_ = [("niter", ctypes.c_int32), ("converged", ctypes.c_int32), ("n_mixed", ctypes.c_int32),
                ("ndropped", ctypes.c_int32), ("nbf", ctypes.c_int32), ("naux", ctypes.c_int32),
                ("nocc", ctypes.c_int32), ("E_nuc", ctypes.c_double), ("err_max", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_scf", ctypes.c_double), ("t_total", ctypes.c_double),
                ("t_eri", ctypes.c_double), ("t_metric", ctypes.c_double), ("t_trsm", ctypes.c_double),
                ("t_j", ctypes.c_double), ("t_kx", ctypes.c_double), ("t_ksyrk", ctypes.c_double),
                ("t_eig", ctypes.c_double), ("n_jk", ctypes.c_int32), ("n_kx_launch", ctypes.c_int32),
                ("t_kx_p", ctypes.c_double * 3), ("t_ksyrk_p", ctypes.c_double * 3),
                ("n_jk_p", ctypes.c_int32 * 3), ("n_kx_launch_p", ctypes.c_int32 * 3),
                ("nintegrals", ctypes.c_int64), ("ncols", ctypes.c_int64),
                ("E_hist", ctypes.c_double * MAXHIST), ("err_hist", ctypes.c_double * MAXHIST),
                ("prec_hist", ctypes.c_int8 * MAXHIST), ("t_guess", ctypes.c_double),
                ("floor_est", ctypes.c_double * 3), ("guess_fallback", ctypes.c_int32),
                ("n_purified", ctypes.c_int32), ("n_eigh", ctypes.c_int32), ("purify_steps", ctypes.c_int32),
                ("t_trsm_update", ctypes.c_double), ("trsm_update_flops", ctypes.c_double),
                ("n_trsm_update", ctypes.c_int32), ("t_purify", ctypes.c_double)]


class Eri3Sizes(ctypes.Structure):
    _fields_ = [("nbf", ctypes.c_int32), ("naux", ctypes.c_int32), ("ncols_tiled", ctypes.c_int64),
                ("bytes_B", ctypes.c_int64), ("bytes_raw", ctypes.c_int64), ("bytes_metric", ctypes.c_int64),
                ("bytes_persistent", ctypes.c_int64), ("bytes_jk", ctypes.c_int64),
                ("bytes_workspace", ctypes.c_int64)]


class GradInfo(ctypes.Structure):
    _fields_ = [("natom", ctypes.c_int32), ("t_setup", ctypes.c_double), ("t_weights", ctypes.c_double),
                ("t_deriv3", ctypes.c_double), ("t_deriv2", ctypes.c_double), ("t_onee", ctypes.c_double),
                ("t_total", ctypes.c_double)]


class GuessSpec(ctypes.Structure):
    _fields_ = [("nelem", ctypes.c_int32), ("Z", ctypes.c_void_p), ("nshell", ctypes.c_void_p),
                ("shell_l", ctypes.c_void_p), ("rc", ctypes.c_double), ("rc_env", ctypes.c_double),
                ("hidden", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("seed", ctypes.c_uint64)]


_vp, _i, _d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_SIGS = {
    "dfx_eri3": [_vp, _i, _vp, _i, _vp, _vp, ctypes.c_size_t, _vp, _vp],
    "dfx_B_info_get": [_vp, _vp],
    "dfx_B_lists": [_vp, _vp, _vp, _vp, _vp, _vp],
    "dfx_B_export": [_vp, _i, _i, _i, _vp, _vp],
    "dfx_B_metric": [_vp, _i, _vp, _vp],
    "dfx_B_free": [_vp],
    "dfx_jk": [_vp, _vp, _i, _i, _i, _vp, _vp, _vp],
    "dfx_jk_noalloc": [_vp, _vp, _i, _i, _vp, _vp, _vp],
    "dfx_mp2": [_vp, _vp, _i, _vp, _i, _i, _vp, _vp],
    "dfx_int1e": [_vp, _i, _vp, _vp, _vp, _vp, _vp],
    "dfx_scf": [_vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp, _vp, _vp],
    "dfx_uhf": [_vp, _vp, _i, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp],
    "dfx_rohf": [_vp, _vp, _i, _vp, _i, _vp, _i, _vp, _vp, _vp, _vp],
    "dfx_scf_default_opts": [_vp],
    "dfx_metric": [_vp, _i, _vp, _vp],
    "dfx_cholesky": [_vp, _i, _vp, _vp],
    "dfx_eigh": [_vp, _i, _vp, _vp, _vp],
    "dfx_guess_create": [_vp, _vp],
    "dfx_guess_free": [_vp],
    "dfx_guess_add": [_vp, _vp, _vp],
    "dfx_guess_train": [_vp, _i, _i, _d, _vp],
    "dfx_guess_predict": [_vp, _vp, _vp],
    "dfx_guess_info": [_vp, _vp, _vp],
    "dfx_guess_export": [_vp, _i, _vp, _vp, _vp, _vp, _vp],
    "dfx_eri3_plan": [_vp, _i, _vp, _i, _vp, _vp],
    "dfx_scf_plan": [_vp, _i, _vp, _i, _i, _vp, _vp],
    "dfx_grad_plan": [_vp, _i, _vp, _i, _i, _i, _vp],
    "dfx_rhf_grad": [_vp, _vp, _i, _vp, _i, _vp, _vp, _vp, _i, _vp, _vp],
    "dfx_B_unpack": [_vp, _i, _i, _vp, _vp],
    "dfx_lowdin": [_vp, _vp, _i, _vp, _vp, _vp],
    "dfx_guess_samples": [_vp, _i, _vp, _vp],
    "dfx_guess_import": [_vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp],
    "dfx_guess_features": [_vp, _vp, _i, _i, _vp, _vp, _vp],
    "dfx_sh_rotation": [_i, _vp, _vp],
    "dfx_guess_save": [_vp, ctypes.c_char_p],
    "dfx_guess_load": [ctypes.c_char_p, _vp],
    "dfx_mlp_forward": [_vp, _i, _vp, _vp, _i, _vp, _vp],
    "dfx_mlp_loss_grad": [_vp, _i, _vp, _vp, _vp, _i, _vp, _vp, _vp],
    "dfx_mlp_adam": [_vp, _vp, _vp, _vp, ctypes.c_int64, _i, ctypes.c_float, _vp],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name, None)
    if _f is not None:
        _f.argtypes = _args
        _f.restype = None if _name == "dfx_scf_default_opts" else ctypes.c_int
_lib.dfx_last_error.restype = ctypes.c_char_p
_lib.dfx_last_error.argtypes = []


def last_error():
    return _lib.dfx_last_error().decode()


def _check(code):
    if code != OK:
        raise DfxError(code, last_error())
    return code


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class _ShellArray:
    """dfx_shell[] over shell dicts (center, l, exps, coefs); keeps the arrays alive."""

    def __init__(self, shells):
        self.keep = []
        self.arr = (Shell * max(1, len(shells)))()
        for i, s in enumerate(shells):
            e = np.ascontiguousarray(s["exps"], dtype=np.float64)
            c = np.ascontiguousarray(s["coefs"], dtype=np.float64)
            self.keep += [e, c]
            sh = self.arr[i]
            for k in range(3):
                sh.xyz[k] = float(s["center"][k])
            sh.l, sh.nprim = int(s["l"]), len(e)
            sh.exps, sh.coefs = e.ctypes.data, c.ctypes.data
        self.n = len(shells)


class _GeomC:
    def __init__(self, xyz, Z, charge=0):
        self.xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        self.Z = np.ascontiguousarray(np.asarray(Z, dtype=np.int32))
        self.g = Geom(len(self.Z), self.xyz.ctypes.data, self.Z.ctypes.data, int(charge))


class DFTensor:
    """Owns a dfx_B handle (the fitted three-index tensor resident in HBM) and
    the torch tensor that is its workspace: B and dfx_jk's work live in that
    memory, which is released only after the handle is freed."""

    def __init__(self, handle, workspace=None):
        self.h = handle
        self.ws = workspace
        inf = BInfo()
        _check(_lib.dfx_B_info_get(self.h, ctypes.byref(inf)))
        self.info = {k: getattr(inf, k) for k, _ in BInfo._fields_}
        self.nbf, self.naux = inf.nbf, inf.naux

    def lists(self, keep=False):
        """Integer screening lists and Schwarz factors (host copies)."""
        inf = self.info
        pairs = np.zeros((inf["npairs"], 2), np.int32)
        off = np.zeros(inf["npairs"] + 1, np.int64)
        kp = np.zeros((inf["npairs"], inf["nauxsh"]), np.uint8) if keep else None
        Qab = np.zeros((inf["nsh"], inf["nsh"]))
        QC = np.zeros(inf["nauxsh"])
        _check(_lib.dfx_B_lists(self.h, pairs.ctypes.data, off.ctypes.data,
                                kp.ctypes.data if keep else None, Qab.ctypes.data, QC.ctypes.data))
        return pairs, off, kp, Qab, QC

    def export(self, what=EXPORT_B, q0=0, q1=None, stream=None):
        import torch
        q1 = self.naux if q1 is None else q1
        out = torch.empty((q1 - q0, self.info["ncols"]), dtype=torch.float64, device="cuda")
        _check(_lib.dfx_B_export(self.h, what, q0, q1, _ptr(out), _stream(stream)))
        return out

    def metric(self, what=0, stream=None):
        import torch
        out = torch.empty((self.naux, self.naux), dtype=torch.float64, device="cuda")
        _check(_lib.dfx_B_metric(self.h, what, _ptr(out), _stream(stream)))
        return out

    def unpack(self, q0=0, q1=None, stream=None):
        """Rows q0..q1-1 of B as dense (q1 - q0, nbf, nbf) float64 cuda tensors."""
        import torch
        q1 = self.naux if q1 is None else q1
        out = torch.empty((q1 - q0, self.nbf, self.nbf), dtype=torch.float64, device="cuda")
        _check(_lib.dfx_B_unpack(self.h, q0, q1, _ptr(out), _stream(stream)))
        return out

    def free(self):
        if self.h:
            _check(_lib.dfx_B_free(self.h))
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def eri3_plan(shells, aux, flags=0):
    """dfx_eri3_plan: the workspace dfx_eri3 needs, in bytes (host only)."""
    s, a = _ShellArray(shells), _ShellArray(aux)
    z = Eri3Sizes()
    _check(_lib.dfx_eri3_plan(s.arr, s.n, a.arr, a.n, ctypes.byref(Eri3Opts(1e-12, flags)), ctypes.byref(z)))
    return {k: getattr(z, k) for k, _ in Eri3Sizes._fields_}


def eri3(shells, aux, tau=1e-12, flags=0, stream=None, workspace=None):
    """dfx_eri3: Rys (mu nu|P), metric, Cholesky and B = L^-1 (mu nu|P) in HBM,
    inside a workspace torch allocates (dfx_eri3_plan's size) unless one is
    given (a uint8 cuda tensor)."""
    import torch
    s, a = _ShellArray(shells), _ShellArray(aux)
    if workspace is None:
        need = eri3_plan(shells, aux, flags)["bytes_workspace"]
        workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    _check(_lib.dfx_eri3(s.arr, s.n, a.arr, a.n, ctypes.byref(Eri3Opts(tau, flags)), _ptr(workspace),
                         workspace.numel() * workspace.element_size(), _stream(stream), ctypes.byref(h)))
    return DFTensor(h, workspace)


def jk(B, x, kind=COCC, nocc=None, precision=FP64, want_j=True, want_k=True, stream=None):
    """dfx_jk: J (Eqs. 3a, 3b) and K (Eqs. 1a, 2a) as (nbf, nbf) float64 cuda tensors."""
    import torch
    x = x.contiguous()
    if x.dtype != torch.float64 or not x.is_cuda:
        raise ValueError("jk: input must be a float64 cuda tensor")
    n = B.nbf
    if nocc is None:
        nocc = x.shape[1] if kind == COCC else 0
    J = torch.empty((n, n), dtype=torch.float64, device=x.device) if want_j else None
    K = torch.empty((n, n), dtype=torch.float64, device=x.device) if want_k else None
    _check(_lib.dfx_jk(B.h, _ptr(x), kind, nocc, precision, _ptr(J) if want_j else None,
                       _ptr(K) if want_k else None, _stream(stream)))
    return J, K


def jk_noalloc(B, C, precision=FP64, want_j=True, want_k=True, J=None, K=None, stream=None):
    """dfx_jk_noalloc: J and K from C_occ with the library's fixed device scratch
    (no device allocation in the library).  J, K: (nbf, nbf) float64 cuda
    outputs, allocated here unless given."""
    import torch
    if C.dtype != torch.float64 or not C.is_cuda or not C.is_contiguous():
        raise ValueError("jk_noalloc: C must be a contiguous float64 cuda tensor")
    n = B.nbf
    if want_j and J is None:
        J = torch.empty((n, n), dtype=torch.float64, device=C.device)
    if want_k and K is None:
        K = torch.empty((n, n), dtype=torch.float64, device=C.device)
    _check(_lib.dfx_jk_noalloc(B.h, _ptr(C), C.shape[1], precision, _ptr(J) if want_j else None,
                               _ptr(K) if want_k else None, _stream(stream)))
    return (J if want_j else None), (K if want_k else None)


def mp2(B, C, eps, nocc, nfrozen=0, stream=None):
    """dfx_mp2: DF-MP2 correlation energy from B and canonical orbitals C (an
    (nbf, nmo) float64 cuda tensor or array, columns = orbitals) with energies eps."""
    import torch
    C = torch.as_tensor(C, dtype=torch.float64, device="cuda").contiguous()
    e = np.ascontiguousarray(eps, dtype=np.float64)
    nmo = C.shape[1]
    if e.shape[0] < nmo:
        raise ValueError("mp2: eps shorter than the number of orbitals")
    E2 = ctypes.c_double()
    _check(_lib.dfx_mp2(B.h, _ptr(C), nmo, e.ctypes.data, nocc, nfrozen, ctypes.byref(E2), _stream(stream)))
    return E2.value


def int1e(shells, xyz, Z, stream=None):
    """dfx_int1e: overlap, kinetic and nuclear-attraction matrices (cuda tensors)."""
    import torch
    s = _ShellArray(shells)
    g = _GeomC(xyz, Z)
    n = sum(2 * int(q["l"]) + 1 for q in shells)
    S, T, V = (torch.empty((n, n), dtype=torch.float64, device="cuda") for _ in range(3))
    _check(_lib.dfx_int1e(s.arr, s.n, ctypes.byref(g.g), _ptr(S), _ptr(T), _ptr(V), _stream(stream)))
    return S, T, V


def metric(aux, stream=None):
    """dfx_metric: the Coulomb metric (P|Q) as an (naux, naux) cuda tensor."""
    import torch
    a = _ShellArray(aux)
    n = sum(2 * int(q["l"]) + 1 for q in aux)
    J = torch.empty((n, n), dtype=torch.float64, device="cuda")
    _check(_lib.dfx_metric(a.arr, a.n, _ptr(J), _stream(stream)))
    return J


def cholesky(A, stream=None):
    """dfx_cholesky: returns (L, L^-1) of a symmetric positive definite cuda tensor."""
    import torch
    L = A.detach().clone().contiguous()
    Linv = torch.empty_like(L)
    _check(_lib.dfx_cholesky(_ptr(L), L.shape[0], _ptr(Linv), _stream(stream)))
    return L, Linv


def eigh(A, stream=None):
    """dfx_eigh: (w, V, sweeps) of a symmetric cuda tensor, w ascending and the
    columns of V the eigenvectors (V[:, k] belongs to w[k])."""
    import torch
    W = A.detach().to(torch.float64).clone().contiguous()
    w = torch.empty(W.shape[0], dtype=torch.float64, device=W.device)
    sw = ctypes.c_int(0)
    _check(_lib.dfx_eigh(_ptr(W), W.shape[0], _ptr(w), ctypes.byref(sw), _stream(stream)))
    return w, W.T, sw.value


# ---- run log -------------------------------------------------------------------
# With a path set (set_run_log, or the DFX_RUN_LOG environment variable), every
# dfx_scf / dfx_uhf / dfx_rohf / dfx_rhf_grad call appends one JSON line: the
# entry point, the system's size, the status, the energy and the info record
# (per-iteration energies, error norms and precisions, phase times).
_RUN_LOG = os.environ.get("DFX_RUN_LOG") or None


def set_run_log(path):
    """Append a JSON line per SCF / gradient call to `path` (None: stop)."""
    global _RUN_LOG
    _RUN_LOG = os.fspath(path) if path is not None else None


def _plain(v):
    if isinstance(v, (list, tuple)):
        return [_plain(x) for x in v]
    if isinstance(v, (np.integer,)):
        return int(v)
    if isinstance(v, (np.floating,)):
        return float(v)
    if isinstance(v, np.ndarray):
        return v.tolist()
    return v


def _log_run(entry, natom, nbf, record):
    if not _RUN_LOG:
        return
    line = {"entry": entry, "unix_time": round(time.time(), 3), "natom": int(natom), "nbf": int(nbf)}
    line.update({k: _plain(v) for k, v in record.items()})
    with open(_RUN_LOG, "a") as f:
        f.write(json.dumps(line) + "\n")


def scf_default_opts():
    o = ScfOpts()
    _lib.dfx_scf_default_opts(ctypes.byref(o))
    return o


def scf_plan(shells, aux, natom, diis_size=8):
    """dfx_scf_plan: bytes of the SCF workspace for these shells (host only)."""
    s, a = _ShellArray(shells), _ShellArray(aux)
    o = scf_default_opts()
    o.diis_size = diis_size
    b = ctypes.c_int64()
    _check(_lib.dfx_scf_plan(s.arr, s.n, a.arr, a.n, int(natom), ctypes.byref(o), ctypes.byref(b)))
    return b.value


# One SCF workspace per device, reused by every dfx_scf / dfx_uhf / dfx_rohf
# call from this module (the calls are synchronous, so one buffer serves them
# in turn) and grown when a larger system needs more.
_SCF_WS = {}


def _scf_workspace(o, shells, aux, natom, need=None):
    import torch
    if not torch.cuda.is_available():
        return None  # the library then reports the missing device itself
    if need is None:
        need = scf_plan(shells, aux, natom, o.diis_size)
    dev = torch.cuda.current_device()
    ws = _SCF_WS.get(dev)
    if ws is None or ws.numel() < need:
        _SCF_WS.pop(dev, None)
        ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{dev}")
        _SCF_WS[dev] = ws
    o.workspace = ws.data_ptr()
    o.ws_bytes = ws.numel()
    return ws


def release_scf_workspace():
    """Drop the cached SCF workspaces (their memory returns to torch's allocator)."""
    _SCF_WS.clear()


def scf(xyz, Z, shells, aux, charge=0, init=None, want_c=True, model=None, **opts):
    """dfx_scf: DF-RHF.  Returns (E, C, eps, info dict); C and eps are numpy arrays
    (None with want_c=False).  With a GuessModel, the start is its predicted density (guess = GUESS_LEARNED)."""
    o = scf_default_opts()
    for k, v in opts.items():
        if not hasattr(o, k) or k == "model":
            raise TypeError(f"unknown SCF option {k!r}")
        setattr(o, k, v)
    if model is not None:
        o.model = model.h.value
        o.guess = GUESS_LEARNED
    s, a = _ShellArray(shells), _ShellArray(aux)
    g = _GeomC(xyz, Z, charge)
    ws = _scf_workspace(o, shells, aux, len(g.Z)) if not o.workspace else None  # noqa: F841 (kept alive)
    n = sum(2 * int(q["l"]) + 1 for q in shells)
    E = ctypes.c_double()
    C = np.zeros((n, n)) if want_c else None
    eps = np.zeros(n) if want_c else None
    inf = ScfInfo()
    ini = None
    if init is not None:
        ini = np.ascontiguousarray(init, dtype=np.float64)
        assert ini.shape == (n, n)
    code = _lib.dfx_scf(ctypes.byref(g.g), s.arr, s.n, a.arr, a.n, ctypes.byref(o),
                        ini.ctypes.data if ini is not None else None, ctypes.byref(E),
                        C.ctypes.data if want_c else None, eps.ctypes.data if want_c else None, ctypes.byref(inf))
    if code not in (OK, ENOCONV):
        _check(code)
    info = {k: getattr(inf, k) for k, _ in ScfInfo._fields_ if not k.endswith("_hist")}
    for k in ("t_kx_p", "t_ksyrk_p", "n_jk_p", "n_kx_launch_p", "floor_est"):
        info[k] = list(getattr(inf, k))
    info["E_hist"] = list(inf.E_hist)[: inf.niter]
    info["err_hist"] = list(inf.err_hist)[: inf.niter]
    info["prec_hist"] = list(inf.prec_hist)[: inf.niter]
    info["status"] = code
    _log_run("dfx_scf", len(g.Z), n, dict(E=E.value, **info))
    return E.value, C, eps, info


def grad_plan(shells, aux, natom, nocc):
    """dfx_grad_plan: bytes of the gradient's workspace (host only)."""
    s, a = _ShellArray(shells), _ShellArray(aux)
    b = ctypes.c_int64()
    _check(_lib.dfx_grad_plan(s.arr, s.n, a.arr, a.n, int(natom), int(nocc), ctypes.byref(b)))
    return b.value


def rhf_grad(xyz, Z, shells, aux, C_occ, eps_occ, tau=1e-12, charge=0):
    """dfx_rhf_grad: the DF-RHF nuclear gradient [natom][3] (Eh/bohr) at the
    converged occupied orbitals C_occ (nbf x nocc) with levels eps_occ, and the
    timing info.  The workspace is the module's cached SCF workspace, grown to
    the gradient's size when needed."""
    C = np.ascontiguousarray(C_occ, dtype=np.float64)
    e = np.ascontiguousarray(eps_occ, dtype=np.float64)
    nocc = C.shape[1]
    if e.shape[0] != nocc:
        raise ValueError("rhf_grad: eps_occ must have one level per column of C_occ")
    o = scf_default_opts()
    o.tau = tau
    s, a = _ShellArray(shells), _ShellArray(aux)
    g = _GeomC(xyz, Z, charge)
    ws = _scf_workspace(o, shells, aux, len(g.Z), need=grad_plan(shells, aux, len(g.Z), nocc))  # noqa: F841
    out = np.zeros((len(g.Z), 3))
    inf = GradInfo()
    _check(_lib.dfx_rhf_grad(ctypes.byref(g.g), s.arr, s.n, a.arr, a.n, ctypes.byref(o), C.ctypes.data,
                             e.ctypes.data, nocc, out.ctypes.data, ctypes.byref(inf)))
    info = {k: getattr(inf, k) for k, _ in GradInfo._fields_}
    _log_run("dfx_rhf_grad", len(g.Z), C.shape[0], dict(nocc=nocc, max_abs_grad=float(np.abs(out).max()), **info))
    return out, info


def _open_shell(fn, nset, xyz, Z, shells, aux, charge, multiplicity, want_c, opts):
    o = scf_default_opts()
    for k, v in opts.items():
        if not hasattr(o, k) or k == "model":
            raise TypeError(f"unknown SCF option {k!r}")
        setattr(o, k, v)
    s, a = _ShellArray(shells), _ShellArray(aux)
    g = _GeomC(xyz, Z, charge)
    ws = _scf_workspace(o, shells, aux, len(g.Z)) if not o.workspace else None  # noqa: F841 (kept alive)
    n = sum(2 * int(q["l"]) + 1 for q in shells)
    E = ctypes.c_double()
    C = np.zeros((nset, n, n)) if want_c else None
    eps = np.zeros((nset, n)) if want_c else None
    inf = ScfInfo()
    code = fn(ctypes.byref(g.g), s.arr, s.n, a.arr, a.n, ctypes.byref(o), int(multiplicity), ctypes.byref(E),
              C.ctypes.data if want_c else None, eps.ctypes.data if want_c else None, ctypes.byref(inf))
    if code not in (OK, ENOCONV):
        _check(code)
    info = {k: getattr(inf, k) for k, _ in ScfInfo._fields_ if not k.endswith("_hist")}
    info["E_hist"] = list(inf.E_hist)[: inf.niter]
    info["err_hist"] = list(inf.err_hist)[: inf.niter]
    info["status"] = code
    _log_run("dfx_uhf" if nset == 2 else "dfx_rohf", len(g.Z), n, dict(E=E.value, multiplicity=int(multiplicity),
                                                                       **info))
    if want_c and nset == 1:
        C, eps = C[0], eps[0]
    return E.value, C, eps, info


def uhf(xyz, Z, shells, aux, charge=0, multiplicity=1, want_c=True, **opts):
    """dfx_uhf: DF-UHF (FP64, core guess).  Returns (E, C, eps, info dict) with
    C [2][nbf][nbf] (alpha, beta) and eps [2][nbf] (None with want_c=False)."""
    return _open_shell(_lib.dfx_uhf, 2, xyz, Z, shells, aux, charge, multiplicity, want_c, opts)


def rohf(xyz, Z, shells, aux, charge=0, multiplicity=1, want_c=True, **opts):
    """dfx_rohf: DF-ROHF (FP64, core guess).  Returns (E, C, eps, info dict) with
    C [nbf][nbf] (core, open, virtual) and eps [nbf] (None with want_c=False)."""
    return _open_shell(_lib.dfx_rohf, 1, xyz, Z, shells, aux, charge, multiplicity, want_c, opts)


# ---- learned starting guess ------------------------------------------------------

class GuessModel:
    """Owns a dfx_guess handle: per-pair-type MLPs predicting blocks of the
    Loewdin-basis density P = S^1/2 D S^1/2 (see lowdin()).

    basis: {Z: [l of each shell of that element, in basis order]}."""

    def __init__(self, basis=None, rc=8.0, rc_env=6.0, hidden=256, depth=3, seed=0, _handle=None):
        self.h = ctypes.c_void_p()
        if _handle is not None:
            self.h = _handle
            return
        Zs = sorted(basis)
        Za = np.array(Zs, np.int32)
        ns = np.array([len(basis[z]) for z in Zs], np.int32)
        ls = np.array([l for z in Zs for l in basis[z]], np.int32)
        spec = GuessSpec(len(Zs), Za.ctypes.data, ns.ctypes.data, ls.ctypes.data, rc, rc_env, hidden, depth, seed)
        _check(_lib.dfx_guess_create(ctypes.byref(spec), ctypes.byref(self.h)))

    @classmethod
    def load(cls, path):
        h = ctypes.c_void_p()
        _check(_lib.dfx_guess_load(os.fsencode(path), ctypes.byref(h)))
        return cls(_handle=h)

    def save(self, path):
        _check(_lib.dfx_guess_save(self.h, os.fsencode(path)))

    def add(self, xyz, Z, P):
        """Samples of one geometry from its Loewdin-basis density P."""
        g = _GeomC(xyz, Z)
        P = np.ascontiguousarray(P, dtype=np.float64)
        _check(_lib.dfx_guess_add(self.h, ctypes.byref(g.g), P.ctypes.data))

    def samples(self, t):
        ty = self.types()[t]
        X = np.zeros((ty["samples"], ty["d_in"]))
        T = np.zeros((ty["samples"], ty["d_out"]))
        _check(_lib.dfx_guess_samples(self.h, t, X.ctypes.data, T.ctypes.data))
        return X, T

    def train(self, epochs, batch=256, lr=1e-3):
        loss = np.zeros(max(1, epochs))
        _check(_lib.dfx_guess_train(self.h, epochs, batch, lr, loss.ctypes.data))
        return loss[:epochs]

    def predict(self, xyz, Z, nbf):
        g = _GeomC(xyz, Z)
        D = np.zeros((nbf, nbf))
        _check(_lib.dfx_guess_predict(self.h, ctypes.byref(g.g), D.ctypes.data))
        return D

    def types(self):
        n = ctypes.c_int()
        _check(_lib.dfx_guess_info(self.h, ctypes.byref(n), None))
        desc = np.zeros((max(1, n.value), 6), np.int32)
        _check(_lib.dfx_guess_info(self.h, ctypes.byref(n), desc.ctypes.data))
        return [dict(atom=bool(d[0]), Za=int(d[1]), Zb=int(d[2]), d_in=int(d[3]), d_out=int(d[4]),
                     samples=int(d[5])) for d in desc[: n.value]]

    def export(self, t, widths):
        ty = self.types()[t]
        npar = sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))
        th = np.zeros(npar, np.float32)
        fm, fs = np.zeros(ty["d_in"]), np.zeros(ty["d_in"])
        tm, ts = np.zeros(ty["d_out"]), np.zeros(ty["d_out"])
        _check(_lib.dfx_guess_export(self.h, t, th.ctypes.data, fm.ctypes.data, fs.ctypes.data,
                                     tm.ctypes.data, ts.ctypes.data))
        return th, fm, fs, tm, ts

    def import_type(self, is_atom, za, zb, theta, fmean, fstd, tmean, tstd):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        arrs = [np.ascontiguousarray(x, dtype=np.float64) for x in (fmean, fstd, tmean, tstd)]
        _check(_lib.dfx_guess_import(self.h, int(is_atom), int(za), int(zb), th.ctypes.data,
                                     *[x.ctypes.data for x in arrs]))

    def features(self, xyz, Z, a, b):
        g = _GeomC(xyz, Z)
        nf = ctypes.c_int()
        _check(_lib.dfx_guess_features(self.h, ctypes.byref(g.g), a, b, None, None, ctypes.byref(nf)))
        f, F = np.zeros(nf.value), np.zeros((3, 3))
        _check(_lib.dfx_guess_features(self.h, ctypes.byref(g.g), a, b, f.ctypes.data, F.ctypes.data, None))
        return f, F

    def free(self):
        if self.h:
            _check(_lib.dfx_guess_free(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lowdin(xyz, Z, shells, D, stream=None):
    """dfx_lowdin: P = S^1/2 D S^1/2 (host numpy arrays in and out)."""
    s = _ShellArray(shells)
    g = _GeomC(xyz, Z)
    D = np.ascontiguousarray(D, dtype=np.float64)
    P = np.zeros_like(D)
    _check(_lib.dfx_lowdin(ctypes.byref(g.g), s.arr, s.n, D.ctypes.data, P.ctypes.data, _stream(stream)))
    return P


def sh_rotation(l, F):
    """dfx_sh_rotation: U with Y_m(F^T u) = sum_m' U[m, m'] Y_m'(u)."""
    F = np.ascontiguousarray(F, dtype=np.float64)
    U = np.zeros((2 * l + 1, 2 * l + 1))
    _check(_lib.dfx_sh_rotation(l, F.ctypes.data, U.ctypes.data))
    return U


def _widths(widths):
    return np.ascontiguousarray(widths, dtype=np.int32)


def mlp_forward(widths, theta, X, stream=None):
    """dfx_mlp_forward on float32 cuda tensors; returns Y (batch, widths[-1])."""
    import torch
    w = _widths(widths)
    Y = torch.empty((X.shape[0], int(w[-1])), dtype=torch.float32, device=X.device)
    _check(_lib.dfx_mlp_forward(w.ctypes.data, len(w) - 1, _ptr(theta), _ptr(X.contiguous()), X.shape[0],
                                _ptr(Y), _stream(stream)))
    return Y


def mlp_loss_grad(widths, theta, X, T, stream=None):
    """dfx_mlp_loss_grad: (mean squared error, gradient in theta as a float32 cuda tensor)."""
    import torch
    w = _widths(widths)
    g = torch.empty_like(theta)
    loss = ctypes.c_double()
    _check(_lib.dfx_mlp_loss_grad(w.ctypes.data, len(w) - 1, _ptr(theta), _ptr(X.contiguous()),
                                  _ptr(T.contiguous()), X.shape[0], _ptr(g), ctypes.byref(loss), _stream(stream)))
    return loss.value, g


def mlp_adam(theta, grad, m, v, step, lr=1e-3, stream=None):
    """dfx_mlp_adam: one in-place Adam step of theta (m, v updated in place)."""
    _check(_lib.dfx_mlp_adam(_ptr(theta), _ptr(grad), _ptr(m), _ptr(v), theta.numel(), step, lr,
                             _stream(stream)))
