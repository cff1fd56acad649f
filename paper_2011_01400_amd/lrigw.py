"""ctypes binding of liblrigw.so (the HIP library declared in include/lrigw.h).

Argument marshalling only: every call forwards device pointers of torch
tensors to the C entry point of the same name.  There is no host compute path;
if the library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrigw.so")

LRIGW_OK = 0
LRIGW_ERR_ARG = -1
LRIGW_ERR_OOM = -2
LRIGW_ERR_HIP = -3
LRIGW_ERR_NOT_HPD = -4
LRIGW_ERR_NOCONV = -5
LRIGW_WARN_QP_NOCONV = 1
LRIGW_WARN_PADE_TRUNC = 2
LRIGW_WARN_CD_RANGE = 3
FIT_SCRATCH_BYTES = 64 << 20   # LRIGW_FIT_SCRATCH_BYTES: workspace limit of lrigw_lri_fit_noalloc

FP64, FP32, SPLIT_BF16, SPLIT3_BF16, SPLIT_MIXED, SPLIT_F16 = 0, 1, 2, 3, 4, 5
PRECISIONS = {"fp64": FP64, "fp32": FP32, "split_bf16": SPLIT_BF16, "split3_bf16": SPLIT3_BF16,
              "split_mixed": SPLIT_MIXED, "split_f16": SPLIT_F16}

# every symbol include/lrigw.h declares
EXPORTS = ["lrigw_create", "lrigw_destroy", "lrigw_strerror", "lrigw_get_sizes", "lrigw_grids", "lrigw_lri_ft",
           "lrigw_build_M", "lrigw_chi0", "lrigw_gamma_prepare", "lrigw_screen", "lrigw_sigma_c", "lrigw_sigma_x",
           "lrigw_sigma_x_pass", "lrigw_lri_fit", "lrigw_lri_fit_noalloc", "lrigw_qp",
           "lrigw_set_real_grid", "lrigw_chi0_real", "lrigw_screen_real", "lrigw_sigma_cd", "lrigw_sigma_cd_pass",
           "lrigw_g0w0_cd", "lrigw_qp_cd", "lrigw_set_gamma_directions", "lrigw_pade_eval", "lrigw_g0w0", "lrigw_set_timing", "lrigw_stage_ms", "lrigw_reset_timing",
           "lrigw_surrogate_create", "lrigw_surrogate_destroy", "lrigw_surrogate_info", "lrigw_surrogate_rule",
           "lrigw_surrogate_params", "lrigw_surrogate_basis", "lrigw_surrogate_add", "lrigw_surrogate_rows",
           "lrigw_surrogate_forward", "lrigw_surrogate_grad", "lrigw_surrogate_train", "lrigw_chi0_surrogate",
           "lrigw_set_surrogate", "lrigw_surrogate_stats", "lrigw_surrogate_reset_stats",
           "lrigw_batch_create", "lrigw_batch_run", "lrigw_batch_status", "lrigw_batch_tuning",
           "lrigw_batch_graph_nodes", "lrigw_batch_destroy", "lrigw_tune", "lrigw_set_tiles", "lrigw_get_tiles"]


class LrigwSystem(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int), ("basis_off", ctypes.POINTER(ctypes.c_int)),
                ("aux_off", ctypes.POINTER(ctypes.c_int)), ("nk", ctypes.c_int * 3), ("n_bands", ctypes.c_int),
                ("n_occ", ctypes.c_int), ("n_freq", ctypes.c_int), ("x0", ctypes.c_double), ("mu", ctypes.c_double),
                ("qp_lo", ctypes.c_int), ("n_qp", ctypes.c_int)]


class LrigwSizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_longlong) for n in ("n_k", "n_b", "n_aux", "n_bands", "n_freq", "nb_max", "h_elems",
                                                  "m_chi_elems", "m_sig_elems", "w_elems", "sigma_elems",
                                                  "m_x_elems")]


class LrigwBatchCell(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("H", ctypes.c_void_p), ("evec", ctypes.c_void_p), ("eig", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("Vcut", ctypes.c_void_p), ("p", ctypes.c_void_p), ("omega_cell", ctypes.c_double),
                ("e_static", ctypes.c_void_p), ("n_par", ctypes.c_int), ("sigma", ctypes.c_void_p),
                ("e_qp", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class LrigwError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_lib = None


def load(path: Optional[str] = None):
    """Load liblrigw.so; raises OSError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    # torch brings its own HIP runtime; it must be the one the library binds to
    # (a second runtime in the process does not see the device)
    import torch  # noqa: F401
    if not os.path.exists(p):
        raise OSError(f"{p} not found: build it with `python -m paper_2011_01400_amd.build`")
    lib = ctypes.CDLL(p)
    vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    ip = ctypes.POINTER(ctypes.c_int)
    ll = ctypes.c_longlong
    llp = ctypes.POINTER(ctypes.c_longlong)
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "lrigw_create": (i, [ctypes.POINTER(vp), ctypes.POINTER(LrigwSystem), i, vp]),
        "lrigw_destroy": (i, [vp]),
        "lrigw_strerror": (ctypes.c_char_p, [i]),
        "lrigw_get_sizes": (i, [vp, ctypes.POINTER(LrigwSizes)]),
        "lrigw_grids": (i, [vp, vp, vp, vp, vp]),
        "lrigw_lri_ft": (i, [vp, vp, ip, i, vp, vp]),
        "lrigw_build_M": (i, [vp, i, i, vp, vp, vp]),
        "lrigw_chi0": (i, [vp, i, vp, vp, i, vp]),
        "lrigw_gamma_prepare": (i, [vp, vp, vp, d]),
        "lrigw_screen": (i, [vp, i, vp, vp, vp, vp, ip]),
        "lrigw_sigma_c": (i, [vp, i, vp, vp, vp, vp]),
        "lrigw_sigma_x": (i, [vp, i, vp, vp, vp]),
        "lrigw_sigma_x_pass": (i, [vp, vp, vp, vp, vp]),
        "lrigw_lri_fit": (i, [vp, i, i, i, i, vp, vp, d, vp, ip]),
        "lrigw_lri_fit_noalloc": (i, [vp, i, i, i, i, vp, vp, d, vp, ip]),
        "lrigw_qp": (i, [vp, vp, vp, vp, i, vp, vp, ip]),
        "lrigw_set_real_grid": (i, [vp, i, d, d]),
        "lrigw_set_gamma_directions": (i, [vp, i, vp, dp]),
        "lrigw_pade_eval": (i, [vp, vp, i, i, vp, vp]),
        "lrigw_chi0_real": (i, [vp, i, vp, vp, i, vp]),
        "lrigw_screen_real": (i, [vp, i, vp, vp, vp, vp, ip]),
        "lrigw_sigma_cd": (i, [vp, i, vp, vp, vp, vp, i, vp, vp]),
        "lrigw_sigma_cd_pass": (i, [vp, vp, vp, vp, vp, vp, vp, d, i, vp, vp, ip]),
        "lrigw_g0w0_cd": (i, [vp, vp, vp, vp, vp, vp, vp, d, vp, d, vp, vp, vp, ip]),
        "lrigw_qp_cd": (i, [vp, vp, vp, vp, vp, vp, vp, d, vp, d, i, i, vp, vp, vp, ip]),
        "lrigw_g0w0": (i, [vp, vp, vp, vp, vp, vp, vp, d, vp, i, i, i, vp, vp, vp, ip]),
        "lrigw_set_timing": (i, [vp, i]),
        "lrigw_stage_ms": (d, [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_longlong)]),
        "lrigw_reset_timing": (None, [vp]),
        "lrigw_surrogate_create": (i, [vp, i, i, i, d, d, ll, vp, vp, ctypes.POINTER(vp)]),
        "lrigw_surrogate_destroy": (i, [vp]),
        "lrigw_surrogate_info": (i, [vp, ip, llp]),
        "lrigw_surrogate_rule": (i, [vp, vp]),
        "lrigw_surrogate_params": (i, [vp, vp, vp]),
        "lrigw_surrogate_basis": (i, [vp, vp, vp, vp]),
        "lrigw_surrogate_add": (i, [vp, vp, vp]),
        "lrigw_surrogate_rows": (i, [vp, llp, vp, vp, ll, ll]),
        "lrigw_surrogate_forward": (i, [vp, vp, i, vp]),
        "lrigw_surrogate_grad": (i, [vp, vp, vp, i, vp, vp]),
        "lrigw_surrogate_train": (i, [vp, i, i, d, vp, ll, vp]),
        "lrigw_chi0_surrogate": (i, [vp, vp, i, vp, vp, i, d, vp]),
        "lrigw_set_surrogate": (i, [vp, vp, d]),
        "lrigw_surrogate_stats": (i, [vp, llp, ip, dp, i]),
        "lrigw_surrogate_reset_stats": (i, [vp]),
        "lrigw_batch_create": (i, [ctypes.POINTER(vp), i, ctypes.POINTER(LrigwBatchCell), i, vp]),
        "lrigw_batch_run": (i, [vp]),
        "lrigw_batch_status": (i, [vp, ip]),
        "lrigw_batch_tuning": (i, [vp, i, ip, ip, dp]),
        "lrigw_batch_graph_nodes": (i, [vp, llp]),
        "lrigw_batch_destroy": (i, [vp]),
        "lrigw_tune": (i, [vp, vp, vp, vp, ip, ip, ip, dp]),
        "lrigw_set_tiles": (i, [vp, i, i, i, i]),
        "lrigw_get_tiles": (i, [vp, ip, ip, ip, ip, ip]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return load().lrigw_strerror(code).decode()
    except OSError:
        return str(code)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


class Context:
    """One lrigw context: a cell's dimensions, grids, workspaces and stream."""

    def __init__(self, *, n_atoms, basis_off, aux_off, nk, n_bands, n_occ, n_freq, x0, mu, qp_lo, n_qp,
                 precision="fp64", stream=None):
        import torch
        self.lib = load()
        self._bo = (ctypes.c_int * (n_atoms + 1))(*[int(v) for v in basis_off])
        self._ao = (ctypes.c_int * (n_atoms + 1))(*[int(v) for v in aux_off])
        s = LrigwSystem()
        s.n_atoms = n_atoms
        s.basis_off = ctypes.cast(self._bo, ctypes.POINTER(ctypes.c_int))
        s.aux_off = ctypes.cast(self._ao, ctypes.POINTER(ctypes.c_int))
        s.nk = (ctypes.c_int * 3)(*[int(v) for v in nk])
        s.n_bands, s.n_occ, s.n_freq = int(n_bands), int(n_occ), int(n_freq)
        s.x0, s.mu = float(x0), float(mu)
        s.qp_lo, s.n_qp = int(qp_lo), int(n_qp)
        self.sys = s
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        rc = self.lib.lrigw_create(ctypes.byref(h), ctypes.byref(s), self.precision, ctypes.c_void_p(stream.cuda_stream))
        if rc != LRIGW_OK:
            raise LrigwError(rc, "lrigw_create")
        self.h = h
        sz = LrigwSizes()
        self._check(self.lib.lrigw_get_sizes(self.h, ctypes.byref(sz)), "lrigw_get_sizes")
        self.sizes = sz
        self.cdtype = torch.complex128 if self.precision == FP64 else torch.complex64

    @classmethod
    def from_system(cls, sysm, precision="fp64", stream=None):
        sp = sysm.spec
        return cls(n_atoms=sp.n_atoms, basis_off=sysm.basis_off, aux_off=sysm.aux_off, nk=sp.nk, n_bands=sp.n_bands,
                   n_occ=sp.n_occ, n_freq=sp.n_freq, x0=sp.x0, mu=sysm.mu, qp_lo=sp.qp_lo, n_qp=sp.n_qp,
                   precision=precision, stream=stream)

    def _check(self, rc, where, allow_warn=False):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise LrigwError(rc, where)
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrigw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- buffers ------------------------------------------------------
    def empty(self, kind):
        import torch
        z = self.sizes
        n = {"H": z.h_elems, "M": z.m_chi_elems, "x": z.m_sig_elems, "xo": z.m_x_elems, "W": z.w_elems}[kind]
        return torch.empty(int(n), dtype=self.cdtype, device="cuda")

    # ---- entry points (same names as the C interface) ------------------
    def grids(self):
        import torch
        n = int(self.sizes.n_freq)
        nk = int(self.sizes.n_k)
        om = torch.empty(n, dtype=torch.float64, device="cuda")
        wt = torch.empty(n, dtype=torch.float64, device="cuda")
        kpq = torch.empty(nk * nk, dtype=torch.int32, device="cuda")
        kmq = torch.empty(nk * nk, dtype=torch.int32, device="cuda")
        self._check(self.lib.lrigw_grids(self.h, _ptr(om), _ptr(wt), _ptr(kpq), _ptr(kmq)), "lrigw_grids")
        return om, wt, kpq.view(nk, nk), kmq.view(nk, nk)

    def lri_ft(self, lri_R, R_list, evec, H_out):
        R = np.ascontiguousarray(R_list, dtype=np.int32)
        rp = R.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        self._check(self.lib.lrigw_lri_ft(self.h, _ptr(lri_R), rp, int(R.shape[0]), _ptr(evec), _ptr(H_out)), "lrigw_lri_ft")
        return H_out

    def build_M(self, iq, slice_, H, evec, M_out):
        self._check(self.lib.lrigw_build_M(self.h, int(iq), int(slice_), _ptr(H), _ptr(evec), _ptr(M_out)), "lrigw_build_M")
        return M_out

    def chi0(self, iq, M, eig, chi_out, apply_gamma=False):
        self._check(self.lib.lrigw_chi0(self.h, int(iq), _ptr(M), _ptr(eig), int(bool(apply_gamma)), _ptr(chi_out)),
                    "lrigw_chi0")
        return chi_out

    def gamma_prepare(self, Vcut0, p, omega_cell):
        self._check(self.lib.lrigw_gamma_prepare(self.h, _ptr(Vcut0), _ptr(p), float(omega_cell)), "lrigw_gamma_prepare")

    def screen(self, iq, chi, V, Wc_out, Vcut=None):
        info = ctypes.c_int(0)
        rc = self.lib.lrigw_screen(self.h, int(iq), _ptr(chi), _ptr(V), _ptr(Vcut), _ptr(Wc_out), ctypes.byref(info))
        if rc < 0:
            e = LrigwError(rc, "lrigw_screen")
            e.info = info.value
            raise e
        return Wc_out

    def sigma_c(self, iq, x, Wc, eig, sigma_acc):
        self._check(self.lib.lrigw_sigma_c(self.h, int(iq), _ptr(x), _ptr(Wc), _ptr(eig), _ptr(sigma_acc)),
                    "lrigw_sigma_c")
        return sigma_acc

    def sigma_x(self, iq, xo, V, sigma_x):
        self._check(self.lib.lrigw_sigma_x(self.h, int(iq), _ptr(xo), _ptr(V), _ptr(sigma_x)), "lrigw_sigma_x")
        return sigma_x

    def sigma_x_pass(self, H, evec, V, sigma_x):
        self._check(self.lib.lrigw_sigma_x_pass(self.h, _ptr(H), _ptr(evec), _ptr(V), _ptr(sigma_x)),
                    "lrigw_sigma_x_pass")
        return sigma_x

    def lri_fit(self, V, T, n_keep, C, scale=1.0):
        """V: FP64 [batch][n][n], T: FP64 [batch][n][nrhs], C: FP64 [batch][n_keep][nrhs] (device)."""
        batch, n, _ = V.shape
        nrhs = T.shape[2]
        info = ctypes.c_int(0)
        rc = self.lib.lrigw_lri_fit(self.h, int(batch), int(n), int(n_keep), int(nrhs), _ptr(V), _ptr(T), float(scale),
                                    _ptr(C), ctypes.byref(info))
        self._check(rc, "lrigw_lri_fit")
        return C

    def lri_fit_noalloc(self, V, T, n_keep, C, scale=1.0):
        """lri_fit with the library's fixed device workspace (no allocation);
        returns (rc, info) without raising, so callers can see ERR_ARG for a
        shape beyond the workspace."""
        batch, n, _ = V.shape
        nrhs = T.shape[2]
        info = ctypes.c_int(0)
        rc = self.lib.lrigw_lri_fit_noalloc(self.h, int(batch), int(n), int(n_keep), int(nrhs), _ptr(V), _ptr(T),
                                            float(scale), _ptr(C), ctypes.byref(info))
        return rc, info.value

    def qp(self, sigma, eps_qp, e_static, n_par, e_qp, z):
        info = ctypes.c_int(0)
        rc = self.lib.lrigw_qp(self.h, _ptr(sigma), _ptr(eps_qp), _ptr(e_static), int(n_par), _ptr(e_qp), _ptr(z),
                               ctypes.byref(info))
        self._check(rc, "lrigw_qp", allow_warn=True)
        return rc, info.value

    def set_gamma_directions(self, p_dirs, weights):
        """p_dirs: complex128 [n_dir][N_k][n_occ][n_unocc] on the device (kept
        alive here), weights: n_dir floats; p_dirs None: one direction."""
        if p_dirs is None:
            self._check(self.lib.lrigw_set_gamma_directions(self.h, 0, None, None), "lrigw_set_gamma_directions")
            self._gdirs = None
            return
        w = np.ascontiguousarray(weights, dtype=np.float64)
        self._check(self.lib.lrigw_set_gamma_directions(self.h, int(w.shape[0]), _ptr(p_dirs),
                                                        w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "lrigw_set_gamma_directions")
        self._gdirs = p_dirs

    # ---- contour deformation (real energies) ---------------------------
    def set_real_grid(self, n_r, omega_max, eta=0.0):
        self._check(self.lib.lrigw_set_real_grid(self.h, int(n_r), float(omega_max), float(eta)), "lrigw_set_real_grid")
        self.n_real = int(n_r)

    def empty_real(self):
        """[n_r][N_aux][N_aux] buffer of the compute type (real-axis response or W^c)."""
        import torch
        n = int(self.sizes.n_aux)
        return torch.empty(self.n_real * n * n, dtype=self.cdtype, device="cuda")

    def chi0_real(self, iq, M, eig, chi_out, apply_gamma=False):
        self._check(self.lib.lrigw_chi0_real(self.h, int(iq), _ptr(M), _ptr(eig), int(bool(apply_gamma)),
                                             _ptr(chi_out)), "lrigw_chi0_real")
        return chi_out

    def screen_real(self, iq, chi, V, Wc_out, Vcut=None):
        info = ctypes.c_int(0)
        rc = self.lib.lrigw_screen_real(self.h, int(iq), _ptr(chi), _ptr(V), _ptr(Vcut), _ptr(Wc_out),
                                        ctypes.byref(info))
        if rc < 0:
            e = LrigwError(rc, "lrigw_screen_real")
            e.info = info.value
            raise e
        return Wc_out

    def sigma_cd(self, iq, x, Wc, Wr, eig, E, sigma_e):
        """E, sigma_e: FP64 [n_e][N_k][n_qp] (device); sigma_e accumulated."""
        self._check(self.lib.lrigw_sigma_cd(self.h, int(iq), _ptr(x), _ptr(Wc), _ptr(Wr), _ptr(eig), int(E.shape[0]),
                                            _ptr(E), _ptr(sigma_e)), "lrigw_sigma_cd")
        return sigma_e

    def sigma_cd_pass(self, H, evec, eig, V, p, omega_cell, E, sigma_e, Vcut=None):
        bad = ctypes.c_int(0)
        rc = self.lib.lrigw_sigma_cd_pass(self.h, _ptr(H), _ptr(evec), _ptr(eig), _ptr(V), _ptr(Vcut), _ptr(p),
                                          float(omega_cell), int(E.shape[0]), _ptr(E), _ptr(sigma_e), ctypes.byref(bad))
        self._check(rc, "lrigw_sigma_cd_pass", allow_warn=True)
        return rc, bad.value

    def g0w0_cd(self, H, evec, eig, V, p, omega_cell, e_static, delta, e_qp, z, sigma3=None, Vcut=None):
        bad = ctypes.c_int(0)
        rc = self.lib.lrigw_g0w0_cd(self.h, _ptr(H), _ptr(evec), _ptr(eig), _ptr(V), _ptr(Vcut), _ptr(p),
                                    float(omega_cell), _ptr(e_static), float(delta), _ptr(sigma3), _ptr(e_qp), _ptr(z),
                                    ctypes.byref(bad))
        self._check(rc, "lrigw_g0w0_cd", allow_warn=True)
        return rc, bad.value

    def qp_cd(self, H, evec, eig, V, p, omega_cell, e_static, delta, n_iter, e_qp, z, sigma3=None, Vcut=None,
              warm=False):
        """warm: continue from the energies e_qp holds (else start at e_n)."""
        bad = ctypes.c_int(0)
        rc = self.lib.lrigw_qp_cd(self.h, _ptr(H), _ptr(evec), _ptr(eig), _ptr(V), _ptr(Vcut), _ptr(p),
                                  float(omega_cell), _ptr(e_static), float(delta), int(n_iter), int(bool(warm)),
                                  _ptr(sigma3), _ptr(e_qp), _ptr(z), ctypes.byref(bad))
        self._check(rc, "lrigw_qp_cd", allow_warn=True)
        return rc, bad.value

    def pade_eval(self, sigma, n_par, E, out):
        """E: FP64 [n_e][N_k][n_qp], out: complex128 [n_e][N_k][n_qp] (device)."""
        self._check(self.lib.lrigw_pade_eval(self.h, _ptr(sigma), int(n_par), int(E.shape[0]), _ptr(E), _ptr(out)),
                    "lrigw_pade_eval")
        return out

    def g0w0(self, H, evec, eig, V, p, omega_cell, e_static, n_par, sigma, e_qp, z, q_first=0, q_last=None, Vcut=None):
        info = ctypes.c_int(0)
        q_last = int(self.sizes.n_k) if q_last is None else q_last
        rc = self.lib.lrigw_g0w0(self.h, _ptr(H), _ptr(evec), _ptr(eig), _ptr(V), _ptr(Vcut), _ptr(p), float(omega_cell),
                                 _ptr(e_static), int(n_par), int(q_first), int(q_last), _ptr(sigma), _ptr(e_qp), _ptr(z),
                                 ctypes.byref(info))
        self._check(rc, "lrigw_g0w0", allow_warn=True)
        return rc, info.value

    def tune(self, H, evec, eig):
        nw, sp, sv, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        self._check(self.lib.lrigw_tune(self.h, _ptr(H), _ptr(evec), _ptr(eig), ctypes.byref(nw), ctypes.byref(sp),
                                        ctypes.byref(sv), ctypes.byref(ms)), "lrigw_tune")
        return nw.value, sp.value, sv.value, ms.value

    def set_tiles(self, nw, splits, pad, sigma_variant):
        self._check(self.lib.lrigw_set_tiles(self.h, int(nw), int(splits), int(pad), int(sigma_variant)), "lrigw_set_tiles")

    def get_tiles(self):
        """(nw, splits, pad, sigma_variant, n_variants) of the context."""
        v = [ctypes.c_int(0) for _ in range(5)]
        self._check(self.lib.lrigw_get_tiles(self.h, *[ctypes.byref(x) for x in v]), "lrigw_get_tiles")
        return tuple(x.value for x in v)

    @property
    def tiles(self):
        return self.get_tiles()[:4]

    def chi0_surrogate(self, sg, iq, M, eig, chi_out, threshold, apply_gamma=False):
        self._check(self.lib.lrigw_chi0_surrogate(self.h, sg.h, int(iq), _ptr(M), _ptr(eig), int(bool(apply_gamma)),
                                                  float(threshold), _ptr(chi_out)), "lrigw_chi0_surrogate")
        return chi_out

    def set_surrogate(self, sg, threshold=0.0):
        self._check(self.lib.lrigw_set_surrogate(self.h, sg.h if sg is not None else None, float(threshold)),
                    "lrigw_set_surrogate")

    def set_timing(self, on=True, kernels_only=False):
        """on: record stage times; kernels_only: only the two MFMA kernel stages."""
        mode = (2 if kernels_only else 1) if on else 0
        self._check(self.lib.lrigw_set_timing(self.h, mode), "lrigw_set_timing")

    def stage_ms(self, stage):
        n = ctypes.c_longlong(0)
        ms = self.lib.lrigw_stage_ms(self.h, stage.encode(), ctypes.byref(n))
        return ms, n.value

    def reset_timing(self):
        self.lib.lrigw_reset_timing(self.h)


class Surrogate:
    """The learned frequency surrogate (lrigw_surrogate_* calls)."""

    def __init__(self, ctx, init_params, start, *, rank, n_anchor=6, hidden=256, d_lo, d_hi, row_capacity=0):
        self.lib = ctx.lib
        self.ctx = ctx
        h = ctypes.c_void_p()
        rc = self.lib.lrigw_surrogate_create(ctx.h, int(rank), int(n_anchor), int(hidden), float(d_lo), float(d_hi),
                                             int(row_capacity), _ptr(init_params), _ptr(start), ctypes.byref(h))
        if rc != LRIGW_OK:
            raise LrigwError(rc, "lrigw_surrogate_create")
        self.h = h
        ints = (ctypes.c_int * 6)()
        n = ctypes.c_longlong(0)
        self._check(self.lib.lrigw_surrogate_info(self.h, ints, ctypes.byref(n)), "lrigw_surrogate_info")
        self.n_anchor, self.n_out, self.holdout, self.t_holdout, self.rank, self.hidden = list(ints)
        self.n_params = n.value

    @staticmethod
    def n_params_of(n_anchor, hidden, n_out):
        return (n_anchor + 1) * hidden + (hidden + 1) * hidden + (hidden + 1) * n_out

    def _check(self, rc, where):
        if rc != LRIGW_OK:
            raise LrigwError(rc, where)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrigw_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rule(self):
        import torch
        C = torch.empty(self.n_anchor * self.n_out, dtype=torch.float64, device="cuda")
        self._check(self.lib.lrigw_surrogate_rule(self.h, _ptr(C)), "lrigw_surrogate_rule")
        return C.view(self.n_anchor, self.n_out)

    def params(self, set_to=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(self.lib.lrigw_surrogate_params(self.h, _ptr(out), _ptr(set_to)), "lrigw_surrogate_params")
        return out

    def basis(self, ctx, chi_a0):
        import torch
        U = torch.empty(int(ctx.sizes.n_aux) * self.rank, dtype=torch.complex128, device="cuda")
        self._check(self.lib.lrigw_surrogate_basis(self.h, ctx.h, _ptr(chi_a0), _ptr(U)), "lrigw_surrogate_basis")
        return U.view(int(ctx.sizes.n_aux), self.rank)

    def add(self, ctx, chi):
        self._check(self.lib.lrigw_surrogate_add(self.h, ctx.h, _ptr(chi)), "lrigw_surrogate_add")

    def rows(self, first=0, count=None):
        import torch
        n = ctypes.c_longlong(0)
        self._check(self.lib.lrigw_surrogate_rows(self.h, ctypes.byref(n), None, None, 0, 0), "lrigw_surrogate_rows")
        count = n.value - first if count is None else count
        x = torch.empty((count, self.n_anchor), dtype=torch.float32, device="cuda")
        y = torch.empty((count, self.n_out), dtype=torch.float32, device="cuda")
        if count > 0:
            self._check(self.lib.lrigw_surrogate_rows(self.h, ctypes.byref(n), _ptr(x), _ptr(y), int(first), int(count)),
                        "lrigw_surrogate_rows")
        return x, y

    def n_rows(self):
        n = ctypes.c_longlong(0)
        self._check(self.lib.lrigw_surrogate_rows(self.h, ctypes.byref(n), None, None, 0, 0), "lrigw_surrogate_rows")
        return n.value

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device="cuda")
        self._check(self.lib.lrigw_surrogate_forward(self.h, _ptr(x), int(x.shape[0]), _ptr(y)), "lrigw_surrogate_forward")
        return y

    def grad(self, x, y):
        import torch
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        self._check(self.lib.lrigw_surrogate_grad(self.h, _ptr(x), _ptr(y), int(x.shape[0]), _ptr(loss), _ptr(g)),
                    "lrigw_surrogate_grad")
        return loss, g

    def train(self, steps, batch, lr, order, loss_hist=None):
        self._check(self.lib.lrigw_surrogate_train(self.h, int(steps), int(batch), float(lr), _ptr(order), int(order.numel()),
                                                   _ptr(loss_hist)), "lrigw_surrogate_train")
        return loss_hist

    def stats(self, max_errors=0):
        n = ctypes.c_longlong(0)
        fb = ctypes.c_int(0)
        errs = (ctypes.c_double * max(1, max_errors))()
        self._check(self.lib.lrigw_surrogate_stats(self.h, ctypes.byref(n), ctypes.byref(fb), errs, int(max_errors)),
                    "lrigw_surrogate_stats")
        return n.value, fb.value, list(errs)[:min(max_errors, n.value)]

    def reset_stats(self):
        self._check(self.lib.lrigw_surrogate_reset_stats(self.h), "lrigw_surrogate_reset_stats")


class Batch:
    """Several cells in one captured hipGraph (lrigw_batch_* calls).
    cells: list of dicts with keys ctx, H, evec, eig, V, p, omega_cell,
    e_static, n_par, sigma, e_qp, z (torch tensors / numbers)."""

    def __init__(self, cells, autotune=True, stream=None):
        import torch
        self.lib = load()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.cells = cells           # keeps the tensors alive
        arr = (LrigwBatchCell * len(cells))()
        for i, c in enumerate(cells):
            arr[i] = LrigwBatchCell(c["ctx"].h.value, _ptr(c["H"]), _ptr(c["evec"]), _ptr(c["eig"]), _ptr(c["V"]),
                                    _ptr(c.get("Vcut")), _ptr(c.get("p")), float(c.get("omega_cell", 0.0)), _ptr(c.get("e_static")),
                                    int(c.get("n_par", 16)), _ptr(c["sigma"]), _ptr(c["e_qp"]), _ptr(c["z"]))
        h = ctypes.c_void_p()
        rc = self.lib.lrigw_batch_create(ctypes.byref(h), len(cells), arr, int(bool(autotune)),
                                         ctypes.c_void_p(self.stream.cuda_stream))
        if rc != LRIGW_OK:
            raise LrigwError(rc, "lrigw_batch_create")
        self.h = h

    def run(self):
        rc = self.lib.lrigw_batch_run(self.h)
        if rc != LRIGW_OK:
            raise LrigwError(rc, "lrigw_batch_run")

    def status(self):
        st = (ctypes.c_int * (3 * len(self.cells)))()
        rc = self.lib.lrigw_batch_status(self.h, st)
        if rc != LRIGW_OK:
            raise LrigwError(rc, "lrigw_batch_status")
        return [tuple(st[3 * i:3 * i + 3]) for i in range(len(self.cells))]

    def tuning(self, i):
        nw, sp, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        self.lib.lrigw_batch_tuning(self.h, int(i), ctypes.byref(nw), ctypes.byref(sp), ctypes.byref(ms))
        return nw.value, sp.value, ms.value

    def graph_nodes(self):
        n = ctypes.c_longlong(0)
        self.lib.lrigw_batch_graph_nodes(self.h, ctypes.byref(n))
        return n.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.lrigw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def device_inputs(sysm, device="cuda", lri_blocks=None, progress=None):
    """Copy the arrays of a synthetic cell to the device (torch tensors).  A
    cell that does not hold its LRI coefficients (lri None) takes them from
    `lri_blocks`, the atoms' blocks in order, each copied into its slice of
    the device array as it comes (the host holds one block at a time);
    progress(A) is called after atom A's block."""
    import torch
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    if sysm.lri is None:
        if lri_blocks is None:
            raise ValueError("the cell holds no LRI coefficients: pass lri_blocks")
        off = np.asarray(sysm.lri_off, dtype=np.int64)
        lri = torch.empty(int(off[-1]), dtype=torch.float64, device=device)
        n = 0
        for A, blk in enumerate(lri_blocks):
            if A >= len(off) - 1 or blk.size != off[A + 1] - off[A]:
                raise ValueError(f"LRI block {A} does not match the cell's offsets")
            lri[int(off[A]):int(off[A + 1])].copy_(torch.from_numpy(np.ascontiguousarray(blk).reshape(-1)))
            n += 1
            if progress is not None:
                progress(A)
        if n != len(off) - 1:
            raise ValueError("fewer LRI blocks than atoms")
    else:
        lri = t(sysm.lri, torch.float64)
    out = dict(
        eig=t(sysm.eig, torch.float64),
        evec=t(sysm.evec, torch.complex128),
        lri=lri,
        V=t(sysm.V, torch.complex128),
        p=t(sysm.p, torch.complex128),
        e_static=t(sysm.e_static, torch.float64),
    )
    if getattr(sysm, "Vcut", None) is not None:
        out["Vcut"] = t(sysm.Vcut, torch.complex128)
    return out
