"""Thin ctypes binding of libefe.so (argument marshalling only).

Every function below forwards to the C entry point of the same name declared
in include/efe.h.  Device memory and streams come from PyTorch; all compute
runs in the library's HIP kernels.  There is no fallback: if the library is
not built or no GPU is present, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libefe.so")

EFE_FP64, EFE_FP32, EFE_BF16 = 0, 1, 2
EFE_FILTER_RESIDUAL, EFE_FILTER_STANDARD = 0, 1
BF16_MAX_AMPLIFICATION = 256.0   # EFE_BF16_MAX_AMPLIFICATION
STATUS = {0: "EFE_OK", -1: "EFE_EINVAL", -2: "EFE_ENOMEM", -3: "EFE_EHIP",
          -4: "EFE_ENOTCONV", -5: "EFE_ENUMERIC", -6: "EFE_ESTATE"}

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)


class MeshDesc(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
                ("ncell", ctypes.c_int32 * 3), ("p", ctypes.c_int32), ("nq", ctypes.c_int32)]


class SystemDesc(ctypes.Structure):
    _fields_ = [("natoms", ctypes.c_int32), ("xyz", c_double_p), ("Z", c_double_p),
                ("loc_rc", ctypes.c_double), ("loc_amp", ctypes.c_double),
                ("loc_rg", ctypes.c_double), ("kb_width", ctypes.c_double),
                ("kb_D", ctypes.c_double), ("kb_rcut", ctypes.c_double),
                ("enr_lmax", ctypes.c_int32), ("enr_alpha", ctypes.c_double),
                ("enr_rcut", ctypes.c_double), ("enr_t", ctypes.c_double),
                ("rho_alpha", ctypes.c_double), ("enr_tab_n", ctypes.c_int32),
                ("enr_tab_dr", ctypes.c_double), ("enr_tab", c_double_p),
                ("enr_tab_rc", ctypes.c_double * 3), ("atom_tab_n", ctypes.c_int32),
                ("atom_tab_dr", ctypes.c_double), ("atom_tab", c_double_p)]


class ChebParams(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("a_min", ctypes.c_double), ("mode", ctypes.c_int32), ("prec", ctypes.c_int32)]


class ScfParams(ctypes.Structure):
    _fields_ = [("passes_first", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("prec", ctypes.c_int32), ("kT", ctypes.c_double),
                ("mix_beta", ctypes.c_double), ("mix_history", ctypes.c_int32),
                ("cg_rtol", ctypes.c_double), ("cg_maxit", ctypes.c_int32),
                ("lanczos_steps", ctypes.c_int32), ("progress", ctypes.c_void_p),
                ("progress_user", ctypes.c_void_p), ("tau", ctypes.c_double),
                ("max_passes", ctypes.c_int32), ("kerker_k0", ctypes.c_double)]


PROGRESS = ctypes.CFUNCTYPE(None, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                            ctypes.c_void_p)


class ScfReport(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("E", "F", "E_band", "E_xc", "E_el", "mu", "n_el", "drho", "dE", "max_occ_res",
                 "b", "t_poisson_ms", "t_filter_ms", "t_rr_ms", "t_density_ms", "t_other_ms",
                 "t_operators_ms", "t_bound_ms", "t_energy_ms")] + \
               [("iter", ctypes.c_int32), ("passes", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("mix_cg_iters", ctypes.c_int32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class RadialParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("h", ctypes.c_double), ("lmax", ctypes.c_int32),
                ("nstates", ctypes.c_int32), ("kT", ctypes.c_double),
                ("mix_beta", ctypes.c_double), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32)]


class RadialReport(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("residual", ctypes.c_double),
                ("mu", ctypes.c_double)]


class EFEError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "efe_setup_mesh": (ctypes.c_int32, [ctypes.POINTER(MeshDesc), ctypes.POINTER(SystemDesc),
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "efe_get_sizes": (ctypes.c_int32, [ctypes.c_void_p, c_int64_p]),
    "efe_radial_atom": (ctypes.c_int32, [ctypes.POINTER(SystemDesc), ctypes.c_int32,
                                         ctypes.POINTER(RadialParams), ctypes.c_void_p]
                        + [ctypes.c_void_p] * 7 + [ctypes.POINTER(RadialReport)]),
    "efe_enrichment_amplification": (ctypes.c_int32, [ctypes.c_void_p, c_double_p]),
    "efe_get_coupling": (ctypes.c_int32, [ctypes.c_void_p, c_int64_p, c_int64_p]),
    "efe_get_tables": (ctypes.c_int32, [ctypes.c_void_p, c_int32_p, c_int32_p, c_int32_p,
                                        c_uint8_p]),
    "efe_get_support": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int64_p, c_int32_p,
                                         c_int32_p]),
    "efe_local_potential": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "efe_set_potential": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "efe_apply_H": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_int64]),
    "efe_apply_H_prec": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]),
    "efe_apply_M": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_int64]),
    "efe_apply_Minv_approx": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_int32, ctypes.c_int64]),
    "efe_spectrum_upper_bound": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int32, c_double_p]),
    "efe_cheb_filter": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int32, ctypes.c_int64,
                                         ctypes.POINTER(ChebParams)]),
    "efe_cheb_filter_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                                 ctypes.POINTER(ChebParams)]),
    "efe_rayleigh_ritz": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "efe_set_density": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "efe_get_density": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "efe_get_quadrature": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "efe_mlp_num_params": (ctypes.c_int64, []),
    "efe_descriptors": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "efe_mlp_forward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]),
    "efe_mlp_loss_grad": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "efe_mlp_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "efe_mlp_adam": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int64]),
    "efe_density_guess": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.POINTER(ctypes.c_float), c_int32_p,
                                           ctypes.POINTER(ctypes.c_double)]),
    "efe_scf_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.POINTER(ScfParams), ctypes.POINTER(ScfReport)]),
    "efe_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "efe_timing_get": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, c_int64_p, c_double_p]),
    "efe_probe_mfma": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "efe_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "efe_destroy": (None, [ctypes.c_void_p]),
}


def lib():
    """Load libefe.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """A library context for one mesh and system (efe_setup_mesh)."""

    def __init__(self, w, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the EFE library needs a GPU")
        L = lib()
        self.w = w
        md = MeshDesc()
        md.lo[:] = [float(v) for v in w["lo"]]
        md.hi[:] = [float(v) for v in w["hi"]]
        md.ncell[:] = [int(v) for v in w["ncell"]]
        md.p = int(w["p"])
        md.nq = int(w["nq"])
        self._xyz = np.ascontiguousarray(np.asarray(w["xyz"], np.float64).reshape(-1, 3))
        self._Z = np.ascontiguousarray(np.asarray(w.get("Zs", np.full(len(self._xyz), w.get("Z", 0.0))),
                                                  np.float64))
        sd = SystemDesc()
        sd.natoms = self._xyz.shape[0]
        sd.xyz = self._xyz.ctypes.data_as(c_double_p)
        sd.Z = self._Z.ctypes.data_as(c_double_p)
        for k in ("loc_rc", "loc_amp", "loc_rg", "kb_width", "kb_D", "kb_rcut", "enr_alpha",
                  "enr_rcut", "enr_t", "rho_alpha"):
            setattr(sd, k, float(w.get(k, 0.0)))
        sd.enr_lmax = int(w.get("enr_lmax", -1))
        tab = w.get("enr_table")
        if tab is not None and sd.enr_lmax >= 0:
            # rows 2l, 2l+1: f_l and f_l' (l <= enr_lmax)
            L_ = sd.enr_lmax + 1
            self._tab = np.ascontiguousarray(np.stack(
                [np.asarray(tab[k][l], np.float64) for l in range(L_) for k in ("f", "df")]))
            sd.enr_tab_n = self._tab.shape[1]
            sd.enr_tab_dr = float(tab["dr"])
            sd.enr_tab = self._tab.ctypes.data_as(c_double_p)
            for l in range(L_):
                sd.enr_tab_rc[l] = float(tab["rc"][l])
        atab = w.get("atom_table")
        if atab is not None:
            # rows rho, rho', phi, phi'
            self._atab = np.ascontiguousarray(np.stack(
                [np.asarray(atab[k][i], np.float64) for k in ("rho", "phi") for i in (0, 1)]))
            sd.atom_tab_n = self._atab.shape[1]
            sd.atom_tab_dr = float(atab["dr"])
            sd.atom_tab = self._atab.ctypes.data_as(c_double_p)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        st = L.efe_setup_mesh(ctypes.byref(md), ctypes.byref(sd), ctypes.c_void_p(stream),
                              ctypes.byref(h))
        if st != 0:
            raise EFEError(st, L.efe_last_error(None).decode())
        self.h = h
        sz = (ctypes.c_int64 * 8)()
        self._check(L.efe_get_sizes(self.h, sz))
        (self.rows, self.n_nodes, self.n_dof, self.n_enr, self.n_cells, self.n_qpts,
         self.natoms, self.nloc) = [int(v) for v in sz]

    def coupling(self):
        """(number of (atom, cell) coupling pairs, largest number of enrichment
        functions coupled to one cell)"""
        n, m = ctypes.c_int64(), ctypes.c_int64()
        self._check(lib().efe_get_coupling(self.h, ctypes.byref(n), ctypes.byref(m)))
        return n.value, m.value

    def amplification(self):
        a = ctypes.c_double()
        self._check(lib().efe_enrichment_amplification(self.h, ctypes.byref(a)))
        return a.value

    # -------------------------------------------------------------- util
    def _check(self, st):
        if st != 0:
            raise EFEError(st, lib().efe_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().efe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _block(X):
        import torch
        if not (X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.stride(1) == 1):
            raise ValueError("blocks are 2-D float64 CUDA tensors with unit column stride")
        return X.shape[1], X.stride(0)

    def empty(self, ncols, ld=None):
        """Zeroed block (rows x ncols) with leading dimension ld (default ncols)."""
        import torch
        ld = ncols if ld is None else ld
        return torch.zeros((self.rows, ld), dtype=torch.float64, device="cuda")[:, :ncols]

    # -------------------------------------------------------------- timing
    TIMERS = {"cell": 0, "pre": 1, "post": 2, "recur": 3, "apply": 4, "rr": 5,
              "cell_narrow": 6, "apply_narrow": 7}

    def timing(self, enable):
        self._check(lib().efe_timing(self.h, 1 if enable else 0))

    def timing_get(self, which):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        self._check(lib().efe_timing_get(self.h, self.TIMERS[which], ctypes.byref(n),
                                         ctypes.byref(ms)))
        return n.value, ms.value

    # -------------------------------------------------------------- tables
    def tables(self):
        c2g = np.empty(self.n_cells * self.nloc, np.int32)
        order = np.empty(self.n_cells, np.int32)
        offs = np.empty(9, np.int32)
        bnd = np.empty(self.n_nodes, np.uint8)
        self._check(lib().efe_get_tables(self.h, c2g.ctypes.data_as(c_int32_p),
                                         order.ctypes.data_as(c_int32_p),
                                         offs.ctypes.data_as(c_int32_p),
                                         bnd.ctypes.data_as(c_uint8_p)))
        return dict(cell_to_global=c2g.reshape(self.n_cells, self.nloc), colour_order=order,
                    colour_offsets=offs, boundary=bnd)

    def support(self, which):
        n = ctypes.c_int64()
        self._check(lib().efe_get_support(self.h, which, ctypes.byref(n), None, None))
        ptr = np.empty(self.natoms + 1, np.int32)
        cells = np.empty(max(n.value, 1), np.int32)
        self._check(lib().efe_get_support(self.h, which, ctypes.byref(n),
                                          ptr.ctypes.data_as(c_int32_p),
                                          cells.ctypes.data_as(c_int32_p)))
        return ptr, cells[:n.value]

    # -------------------------------------------------------------- operators
    def local_potential(self):
        import torch
        vq = torch.empty(self.n_qpts, dtype=torch.float64, device="cuda")
        self._check(lib().efe_local_potential(self.h, _ptr(vq)))
        return vq

    def set_potential(self, vq, precisions=0):
        self._check(lib().efe_set_potential(self.h, _ptr(vq), int(precisions)))

    def apply_H(self, X, Y=None):
        n, ld = self._block(X)
        Y = self.empty(n, ld) if Y is None else Y
        self._check(lib().efe_apply_H(self.h, _ptr(X), _ptr(Y), n, ld))
        return Y

    def apply_H_prec(self, X, prec, Y=None):
        n, ld = self._block(X)
        Y = self.empty(n, ld) if Y is None else Y
        self._check(lib().efe_apply_H_prec(self.h, _ptr(X), _ptr(Y), n, ld, int(prec)))
        return Y

    def apply_M(self, X, Y=None):
        n, ld = self._block(X)
        Y = self.empty(n, ld) if Y is None else Y
        self._check(lib().efe_apply_M(self.h, _ptr(X), _ptr(Y), n, ld))
        return Y

    def apply_Minv_approx(self, X, Y=None):
        n, ld = self._block(X)
        Y = self.empty(n, ld) if Y is None else Y
        self._check(lib().efe_apply_Minv_approx(self.h, _ptr(X), _ptr(Y), n, ld))
        return Y

    def spectrum_upper_bound(self, v0, steps=20):
        b = ctypes.c_double()
        self._check(lib().efe_spectrum_upper_bound(self.h, _ptr(v0), int(steps), ctypes.byref(b)))
        return b.value

    def cheb_filter(self, V, lam, degree, a, b, a_min, mode=EFE_FILTER_RESIDUAL, prec=EFE_FP64):
        n, ld = self._block(V)
        p = ChebParams(int(degree), float(a), float(b), float(a_min), int(mode), int(prec))
        lp = _ptr(lam) if lam is not None else None
        self._check(lib().efe_cheb_filter(self.h, _ptr(V), lp, n, ld, ctypes.byref(p)))
        return V

    def cheb_filter_noalloc(self, V, lam, degree, a, b, a_min, mode=EFE_FILTER_RESIDUAL,
                            prec=EFE_FP64):
        n, ld = self._block(V)
        p = ChebParams(int(degree), float(a), float(b), float(a_min), int(mode), int(prec))
        lp = _ptr(lam) if lam is not None else None
        self._check(lib().efe_cheb_filter_noalloc(self.h, _ptr(V), lp, n, ld, ctypes.byref(p)))
        return V

    def rayleigh_ritz(self, V, want_res=True):
        import torch
        n, ld = self._block(V)
        lam = torch.empty(n, dtype=torch.float64, device="cuda")
        res = torch.empty(n, dtype=torch.float64, device="cuda") if want_res else None
        self._check(lib().efe_rayleigh_ritz(self.h, _ptr(V), n, ld, _ptr(lam),
                                            _ptr(res) if res is not None else None))
        return lam, res


    # -------------------------------------------------------------- SCF
    def set_density(self, rho):
        self._check(lib().efe_set_density(self.h, _ptr(rho)))

    def get_density(self, which=0):
        import torch
        out = torch.empty(self.n_qpts, dtype=torch.float64, device="cuda")
        self._check(lib().efe_get_density(self.h, int(which), _ptr(out)))
        return out

    def density_guess(self, params=None, norm=None):
        """Set the next step's input density to the learned guess (SAD when
        params is None); returns (used_fallback, factor)."""
        fb = ctypes.c_int32()
        fac = ctypes.c_double()
        nm = None
        if params is not None:
            arr = np.ascontiguousarray(np.asarray(norm, np.float32).ravel())
            if arr.size != 51:
                raise ValueError("norm holds shift[25], scale[25], target scale")
            nm = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        self._check(lib().efe_density_guess(self.h, _ptr(params) if params is not None else None,
                                            nm, ctypes.byref(fb), ctypes.byref(fac)))
        return bool(fb.value), fac.value

    def quadrature(self):
        """(positions (n_qpts, 3), weights (n_qpts,)) of the Gauss points."""
        import torch
        xq = torch.empty(self.n_qpts, 3, dtype=torch.float64, device="cuda")
        wq = torch.empty(self.n_qpts, dtype=torch.float64, device="cuda")
        self._check(lib().efe_get_quadrature(self.h, _ptr(xq), _ptr(wq)))
        return xq, wq

    def scf_step(self, V, lam, v0, degree, passes_first=4, passes=1, prec=EFE_FP64,
                 kT=500 * 3.166811563e-6, mix_beta=0.3, mix_history=8, cg_rtol=1e-12,
                 cg_maxit=5000, lanczos_steps=20, progress=None, tau=0.0, max_passes=0,
                 kerker_k0=0.0):
        """One SCF step; `progress(pass, filter_ms, rr_ms)` (optional) is called
        after every filter + Rayleigh-Ritz pass."""
        n, ld = self._block(V)
        cb = PROGRESS(lambda i, tf, tr, _u: progress(i, tf, tr)) if progress else None
        p = ScfParams(int(passes_first), int(passes), int(degree), int(prec), float(kT),
                      float(mix_beta), int(mix_history), float(cg_rtol), int(cg_maxit),
                      int(lanczos_steps),
                      ctypes.cast(cb, ctypes.c_void_p) if cb is not None else None, None,
                      float(tau), int(max_passes), float(kerker_k0))
        rep = ScfReport()
        self._check(lib().efe_scf_step(self.h, _ptr(V), n, ld, _ptr(lam), _ptr(v0),
                                       ctypes.byref(p), ctypes.byref(rep)))
        return rep.as_dict()


def scf_run(ctx, V, lam, v0, degree, tol=1e-5, max_iter=50, rho_tol=1e-5, **kw):
    """Drive efe_scf_step until |E_k - E_{k-1}| / N_atoms < tol and the
    density residual ||rho_out - rho_in||_2 per electron is below rho_tol
    (None: energy test only).  The energy alone can stall for a step while
    the density is still far from self-consistent, so both are required.
    `log(step, report)` (optional keyword) is called after every step.
    Returns the list of step reports."""
    hist = []
    log = kw.pop("log", None)
    for it in range(max_iter):
        rep = ctx.scf_step(V, lam, v0, degree, **kw)
        hist.append(rep)
        if log:
            log(it, rep)
        if (it > 0 and abs(rep["dE"]) / max(ctx.natoms, 1) < tol and
                (rho_tol is None or rep["drho"] / max(rep["n_el"], 1e-300) < rho_tol)):
            break
    return hist


# ------------------------------------------------------------------ learned density
def _stream(stream):
    import torch
    return ctypes.c_void_p(stream if stream is not None else
                           torch.cuda.current_stream().cuda_stream)


def _gcheck(st, what):
    if st != 0:
        raise EFEError(st, f"{what}: " + (lib().efe_last_error(None) or b"").decode())


def mlp_num_params():
    return int(lib().efe_mlp_num_params())


def efe_descriptors(pts, xyz, rho_sad, shift=None, scale=None, out=None, stream=None):
    """(npts, 25) FP32 features; pts (npts, 3), xyz (natoms, 3), rho_sad (npts)
    are FP64 device tensors, shift/scale FP32 device tensors or None."""
    import torch
    n = pts.shape[0]
    if out is None:
        out = torch.empty(n, 25, dtype=torch.float32, device=pts.device)
    _gcheck(lib().efe_descriptors(_stream(stream), _ptr(pts), n, _ptr(xyz), xyz.shape[0],
                                  _ptr(rho_sad), _ptr(shift) if shift is not None else None,
                                  _ptr(scale) if scale is not None else None, _ptr(out)),
            "efe_descriptors")
    return out


def efe_mlp_forward(params, feat, acts=None, out=None, stream=None):
    import torch
    n = feat.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=feat.device)
    _gcheck(lib().efe_mlp_forward(_stream(stream), _ptr(params), _ptr(feat), n, _ptr(out),
                                  _ptr(acts) if acts is not None else None), "efe_mlp_forward")
    return out


def efe_mlp_loss_grad(out, target, weight, dout=None, sums=None, stream=None):
    import torch
    n = out.shape[0]
    if dout is None:
        dout = torch.empty_like(out)
    if sums is None:
        sums = torch.empty(2, dtype=torch.float64, device=out.device)
    _gcheck(lib().efe_mlp_loss_grad(_stream(stream), _ptr(out), _ptr(target), _ptr(weight), n,
                                    _ptr(dout), _ptr(sums)), "efe_mlp_loss_grad")
    return dout, sums


def efe_mlp_backward(params, feat, acts, dout, grads=None, work=None, stream=None):
    import torch
    n = feat.shape[0]
    if grads is None:
        grads = torch.empty_like(params)
    if work is None:
        work = torch.empty(2 * n * 128, dtype=torch.float32, device=feat.device)
    _gcheck(lib().efe_mlp_backward(_stream(stream), _ptr(params), _ptr(feat), _ptr(acts),
                                   _ptr(dout), n, _ptr(grads), _ptr(work)), "efe_mlp_backward")
    return grads


def efe_mlp_adam(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _gcheck(lib().efe_mlp_adam(_stream(stream), _ptr(params), _ptr(grads), _ptr(m), _ptr(v),
                               params.numel(), float(lr), float(beta1), float(beta2), float(eps),
                               int(step)), "efe_mlp_adam")


# module-level names of the C entry points
def radial_atom(w, n=2000, h=0.02, lmax=1, nstates=2, kT=500 * 3.166811563e-6, beta=0.5,
                tol=1e-10, maxit=300, atom=0, stream=None):
    """efe_radial_atom for atom `atom` of workload w: the isolated atom's
    levels, radial functions, density, r0 and enrichment table on the GPU;
    returns numpy arrays (and the table in the form Context accepts as
    w["enr_table"])."""
    import torch
    xyz = np.ascontiguousarray(np.asarray(w["xyz"], np.float64).reshape(-1, 3))
    Z = np.ascontiguousarray(np.asarray(w.get("Zs", np.full(len(xyz), w.get("Z", 0.0))),
                                        np.float64))
    sd = SystemDesc()
    sd.natoms = xyz.shape[0]
    sd.xyz = xyz.ctypes.data_as(c_double_p)
    sd.Z = Z.ctypes.data_as(c_double_p)
    for k in ("loc_rc", "loc_amp", "loc_rg", "kb_width", "kb_D", "kb_rcut", "enr_alpha",
              "enr_rcut", "enr_t", "rho_alpha"):
        setattr(sd, k, float(w.get(k, 0.0)))
    sd.enr_lmax = int(w.get("enr_lmax", -1))
    pr = RadialParams(int(n), float(h), int(lmax), int(nstates), float(kT), float(beta),
                      float(tol), int(maxit))
    nl = (lmax + 1) * nstates
    dev = dict(dtype=torch.float64, device="cuda")
    eps, occ = torch.zeros(nl, **dev), torch.zeros(nl, **dev)
    u = torch.zeros(nl, n, **dev)
    rho = torch.zeros(n, **dev)
    r0 = torch.zeros(lmax + 1, **dev)
    tab = torch.zeros(2 * (lmax + 1), n + 1, **dev)
    atab = torch.zeros(4, n + 1, **dev)
    rep = RadialReport()
    st = lib().efe_radial_atom(ctypes.byref(sd), int(atom), ctypes.byref(pr),
                               _stream(stream), _ptr(eps), _ptr(u), _ptr(occ),
                               _ptr(rho), _ptr(r0), _ptr(tab), _ptr(atab), ctypes.byref(rep))
    if st != 0:
        raise EFEError(st, lib().efe_last_error(None).decode())
    torch.cuda.synchronize()
    t = float(w.get("enr_t", 0.33))
    T = tab.cpu().numpy()
    A = atab.cpu().numpy()
    R0 = r0.cpu().numpy()
    return dict(eps=eps.cpu().numpy().reshape(lmax + 1, nstates),
                occ=occ.cpu().numpy().reshape(lmax + 1, nstates),
                u=u.cpu().numpy().reshape(lmax + 1, nstates, n), rho=rho.cpu().numpy(), r0=R0,
                iterations=rep.iterations, residual=rep.residual, mu=rep.mu,
                table=dict(f=T[0::2], df=T[1::2], dr=float(h), r0=R0, rc=R0 * (1.0 + 1.0 / t),
                           t=t),
                atom_table=dict(rho=(A[0], A[1]), phi=(A[2], A[3]), dr=float(h)))


def efe_setup_mesh(workload, stream=None):
    return Context(workload, stream)


def efe_apply_H(ctx, X, Y=None):
    return ctx.apply_H(X, Y)


def efe_cheb_filter(ctx, V, lam, degree, a, b, a_min, mode=EFE_FILTER_RESIDUAL, prec=EFE_FP64):
    return ctx.cheb_filter(V, lam, degree, a, b, a_min, mode, prec)


def efe_rayleigh_ritz(ctx, V):
    return ctx.rayleigh_ritz(V)
