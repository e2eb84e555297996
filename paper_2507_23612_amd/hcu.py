"""Thin ctypes binding of libhcu.so (include/hubbard_chfsi.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  PyTorch supplies the device workspace and the stream.  The binding
raises if the compiled library is missing - there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libhcu.so")

HCU_OK, HCU_INVALID_ARG, HCU_OOM, HCU_NOT_SPD, HCU_NOT_CONVERGED, HCU_NAN, HCU_DEVICE, HCU_NOT_BOUND = range(8)
STATUS_NAMES = ["HCU_OK", "HCU_INVALID_ARG", "HCU_OOM", "HCU_NOT_SPD", "HCU_NOT_CONVERGED", "HCU_NAN",
                "HCU_DEVICE", "HCU_NOT_BOUND"]
HCU_FP64, HCU_MIXED = 0, 1
MAX_KB = 4


class hcu_species(C.Structure):
    _fields_ = [("vloc_depth", C.c_double), ("vloc_width", C.c_double), ("n_kb", C.c_int),
                ("kb_l", C.c_int * MAX_KB), ("kb_gamma", C.c_double * MAX_KB), ("kb_width", C.c_double),
                ("hub_l", C.c_int), ("hub_U", C.c_double), ("hub_power", C.c_int), ("hub_alpha", C.c_double),
                ("threshold", C.c_double)]


class hcu_problem(C.Structure):
    _fields_ = [("L", C.c_double * 3), ("n", C.c_int * 3), ("n0", C.c_int), ("nspin", C.c_int), ("nk", C.c_int),
                ("kpts", C.POINTER(C.c_double)), ("kw", C.POINTER(C.c_double)), ("natom", C.c_int),
                ("atom_species", C.POINTER(C.c_int)), ("pos", C.POINTER(C.c_double)), ("nspecies", C.c_int),
                ("species", C.POINTER(hcu_species)), ("ns", C.c_int), ("nelec", C.c_double), ("kT", C.c_double),
                ("degree", C.c_int), ("precision", C.c_int), ("lowdin", C.c_int), ("hxc", C.c_int)]


class hcu_scf_opts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("first_passes", C.c_int), ("lanczos_steps", C.c_int),
                ("pulay_history", C.c_int), ("pulay_beta", C.c_double), ("tol_d", C.c_double),
                ("tol_f", C.c_double), ("fixed_iterations", C.c_int), ("verbose", C.c_int),
                ("kerker_k0", C.c_double), ("tol_rho", C.c_double)]


class hcu_scf_report(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("F", C.c_double), ("E_U", C.c_double),
                ("e_band", C.c_double), ("residual", C.c_double), ("seconds", C.c_double),
                ("filter_seconds", C.c_double), ("hx_columns", C.c_double), ("residual_rho", C.c_double)]


class hcu_scf_step_info(C.Structure):
    _fields_ = [("iteration", C.c_int), ("converged", C.c_int), ("F", C.c_double), ("E_U", C.c_double),
                ("residual", C.c_double), ("dF", C.c_double), ("residual_rho", C.c_double)]


class hcu_sizes(C.Structure):
    _fields_ = [("nd", C.c_int64), ("nproj", C.c_int), ("nblocks", C.c_int), ("support_points", C.c_int64),
                ("table_nnz", C.c_int64), ("workspace_bytes", C.c_size_t), ("max_brick_functions", C.c_int),
                ("brick_slots", C.c_int64)]


class hcu_energies(C.Structure):
    _fields_ = [("F", C.c_double), ("e_band", C.c_double), ("dc", C.c_double), ("E_U", C.c_double),
                ("ts", C.c_double), ("mu", C.c_double), ("E_H", C.c_double), ("E_x", C.c_double),
                ("e_hxc", C.c_double)]


class hcu_kernel_times(C.Structure):
    _fields_ = [("stencil_ms", C.c_double), ("stencil_launches", C.c_longlong),
                ("project_ms", C.c_double), ("project_launches", C.c_longlong),
                ("gram_ms", C.c_double), ("gram_launches", C.c_longlong),
                ("eig_ms", C.c_double), ("eig_launches", C.c_longlong),
                ("rotate_ms", C.c_double), ("rotate_launches", C.c_longlong),
                ("scatter_ms", C.c_double), ("scatter_launches", C.c_longlong),
                ("fused_ms", C.c_double), ("fused_launches", C.c_longlong),
                ("hxc_ms", C.c_double), ("hxc_launches", C.c_longlong)]


class hcu_tuning(C.Structure):
    _fields_ = [("tile_x", C.c_int), ("tile_yt", C.c_int), ("ry", C.c_int), ("tile_z", C.c_int),
                ("halo_ring", C.c_int), ("stencil_ms", C.c_double)]


_lib = None


def load_library(path=LIB_PATH):
    """Load libhcu.so (raises FileNotFoundError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} not built: run python -m paper_2507_23612_amd.build")
    lib = C.CDLL(path)
    P = C.c_void_p
    sig = {
        "hcu_create": (C.c_int, [C.POINTER(hcu_problem), C.POINTER(P)]),
        "hcu_destroy": (None, [P]),
        "hcu_last_error": (C.c_char_p, [P]),
        "hcu_workspace_size": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "hcu_bind": (C.c_int, [P, P, C.c_size_t, P]),
        "hcu_set_hubbard_occupation": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_num_hubbard_atoms": (C.c_int, [P]),
        "hcu_get_sizes": (C.c_int, [P, C.POINTER(hcu_sizes)]),
        "hcu_set_start": (C.c_int, [P, C.c_int, C.c_int, P, P]),
        "hcu_apply_h": (C.c_int, [P, C.c_int, C.c_int, P, P, C.c_int, C.c_int64]),
        "hcu_cheb_filter": (C.c_int, [P, C.c_int, C.c_int, P, P, C.c_int, C.c_int64, C.c_int, C.c_double,
                                      C.c_double, C.c_double]),
        "hcu_chfsi_pass": (C.c_int, [P, C.c_int, C.c_int]),
        "hcu_lanczos_bounds": (C.c_int, [P, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double),
                                         C.POINTER(C.c_double)]),
        "hcu_gram": (C.c_int, [P, P, P, C.c_int, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "hcu_rotate": (C.c_int, [P, P, C.POINTER(C.c_double), P, C.c_int, C.c_int64]),
        "hcu_scf": (C.c_int, [P, C.POINTER(hcu_scf_opts), C.POINTER(hcu_scf_report)]),
        "hcu_update_occupations": (C.c_int, [P]),
        "hcu_scf_begin": (C.c_int, [P, C.POINTER(hcu_scf_opts)]),
        "hcu_scf_step": (C.c_int, [P, C.POINTER(hcu_scf_step_info)]),
        "hcu_set_profiling": (C.c_int, [P, C.c_int]),
        "hcu_autotune": (C.c_int, [P, C.POINTER(hcu_tuning)]),
        "hcu_set_tuning": (C.c_int, [P, C.POINTER(hcu_tuning)]),
        "hcu_get_kernel_times": (C.c_int, [P, C.POINTER(hcu_kernel_times)]),
        "hcu_get_eigenvalues": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_get_occupations": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_get_hubbard_occupation": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_get_energies": (C.c_int, [P, C.POINTER(hcu_energies)]),
        "hcu_get_orbitals": (C.c_int, [P, C.c_int, C.c_int, P, C.c_int]),
        "hcu_get_density": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_get_potential": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "hcu_batch_create": (C.c_int, [C.POINTER(P), C.c_int, C.POINTER(P)]),
        "hcu_batch_destroy": (None, [P]),
        "hcu_batch_last_error": (C.c_char_p, [P]),
        "hcu_batch_chfsi_pass": (C.c_int, [P]),
        "hcu_batch_scf": (C.c_int, [P, C.POINTER(hcu_scf_opts), C.POINTER(hcu_scf_report)]),
        "hcu_state_size": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "hcu_save_state": (C.c_int, [P, P, C.c_size_t]),
        "hcu_load_state": (C.c_int, [P, P, C.c_size_t]),
        "hcu_descriptor": (C.c_int, [P, P, C.POINTER(C.c_int)]),
        "hcu_shell_density": (C.c_int, [P, C.POINTER(C.c_double)]),
        "hcu_site_targets": (C.c_int, [P, C.POINTER(C.c_float)]),
        "hcu_mlp_create": (C.c_int, [C.POINTER(C.c_int), C.c_int, C.c_int, C.POINTER(P)]),
        "hcu_mlp_destroy": (None, [P]),
        "hcu_mlp_last_error": (C.c_char_p, [P]),
        "hcu_mlp_param_count": (C.c_int, [P, C.POINTER(C.c_int64)]),
        "hcu_mlp_workspace_size": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "hcu_mlp_bind": (C.c_int, [P, P, C.c_size_t, P]),
        "hcu_mlp_set_params": (C.c_int, [P, C.POINTER(C.c_float)]),
        "hcu_mlp_get_params": (C.c_int, [P, C.POINTER(C.c_float)]),
        "hcu_mlp_set_scaling": (C.c_int, [P] + [C.POINTER(C.c_float)] * 4),
        "hcu_mlp_get_scaling": (C.c_int, [P] + [C.POINTER(C.c_float)] * 4),
        "hcu_mlp_fit_scaling": (C.c_int, [P, P, P, C.c_int]),
        "hcu_mlp_forward": (C.c_int, [P, P, C.c_int, P, C.c_int]),
        "hcu_mlp_gradient": (C.c_int, [P, P, P, P, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_double)]),
        "hcu_mlp_train_step": (C.c_int, [P, P, P, P, C.c_int, C.c_float, C.POINTER(C.c_double)]),
        "hcu_mlp_guess": (C.c_int, [P, P, C.c_int, C.POINTER(C.c_float)]),
        "hcu_gram_noalloc": (C.c_int, [P, P, C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_double, P, P, P]),
        "hcu_hubbard_forces": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "hcu_move_atoms": (C.c_int, [P, C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_double)]),
        "hcu_hubbard_stress": (C.c_int, [P, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HcuError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def species_struct(sp):
    s = hcu_species()
    s.vloc_depth = sp["vloc_depth"]
    s.vloc_width = sp["vloc_width"]
    s.n_kb = len(sp["kb_l"])
    for i, (l, g) in enumerate(zip(sp["kb_l"], sp["kb_gamma"])):
        s.kb_l[i] = l
        s.kb_gamma[i] = g
    s.kb_width = sp["kb_width"]
    s.hub_l = sp["hub_l"]
    s.hub_U = sp["hub_U"]
    s.hub_power = sp["hub_power"]
    s.hub_alpha = sp["hub_alpha"]
    s.threshold = sp["threshold"]
    return s


class Problem:
    """hcu_problem built from a workload dict (keeps the host arrays alive)."""

    def __init__(self, cfg, precision=None):
        self.cfg = cfg
        self.kpts = np.ascontiguousarray(np.asarray(cfg["kpts"], np.float64).reshape(-1, 3))
        self.kw = np.ascontiguousarray(np.asarray(cfg["kw"], np.float64))
        self.pos = np.ascontiguousarray(np.asarray(cfg["pos"], np.float64).reshape(-1, 3))
        self.spec = np.ascontiguousarray(np.asarray(cfg["atom_species"], np.int32))
        self.species = (hcu_species * len(cfg["species"]))(*[species_struct(s) for s in cfg["species"]])
        p = hcu_problem()
        for a in range(3):
            p.L[a] = float(cfg["L"][a])
            p.n[a] = int(cfg["n"][a])
        p.n0 = int(cfg["n0"])
        p.nspin = int(cfg["nspin"])
        p.nk = len(self.kw)
        p.kpts = _dptr(self.kpts)
        p.kw = _dptr(self.kw)
        p.natom = len(self.spec)
        p.atom_species = self.spec.ctypes.data_as(C.POINTER(C.c_int))
        p.pos = _dptr(self.pos)
        p.nspecies = len(cfg["species"])
        p.species = C.cast(self.species, C.POINTER(hcu_species))
        p.ns = int(cfg["ns"])
        p.nelec = float(cfg["nelec"])
        p.kT = float(cfg["kT"])
        p.degree = int(cfg["degree"])
        prec = precision or cfg.get("precision", "fp64")
        p.precision = HCU_MIXED if prec == "mixed" else HCU_FP64
        p.lowdin = 1 if cfg.get("lowdin", True) else 0
        p.hxc = 1 if cfg.get("hxc", False) else 0
        self.p = p


class HcuContext:
    """One library context bound to a torch-allocated device workspace."""

    def __init__(self, cfg, precision=None, device="cuda:0", workspace_margin=0.0):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.prob = Problem(cfg, precision)
        self.cfg = cfg
        self.h = C.c_void_p()
        st = self.lib.hcu_create(C.byref(self.prob.p), C.byref(self.h))
        if st != HCU_OK:
            msg = self.lib.hcu_last_error(self.h).decode() if self.h else "create failed"
            self.lib.hcu_destroy(self.h)
            self.h = None
            raise HcuError(st, msg)
        nb = C.c_size_t()
        self._check(self.lib.hcu_workspace_size(self.h, C.byref(nb)))
        self.workspace_bytes = nb.value
        self.device = torch.device(device)
        # a margin lets moved atoms (hcu_move_atoms) grow their supports in place
        self.bound_bytes = int(self.workspace_bytes * (1.0 + workspace_margin)) // 256 * 256 + 256
        self.ws = torch.empty(self.bound_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hcu_bind(self.h, C.c_void_p(self.ws_ptr), C.c_size_t(self.bound_bytes),
                                      C.c_void_p(self.stream.cuda_stream)))
        self.nspin = int(cfg["nspin"])
        self.nk = len(self.prob.kw)
        self.ns = int(cfg["ns"])
        self.nd = int(np.prod(cfg["n"]))
        self.nhub = self.lib.hcu_num_hubbard_atoms(self.h)
        self.mixed = self.prob.p.precision == HCU_MIXED
        self.complex = bool(np.any(self.prob.kpts != 0))
        base_t = torch.float32 if self.mixed else torch.float64
        self.dtype = {torch.float32: torch.complex64, torch.float64: torch.complex128}[base_t] \
            if self.complex else base_t

    # -------------------------------------------------------------- helpers
    def _check(self, st):
        if st != HCU_OK:
            raise HcuError(st, self.lib.hcu_last_error(self.h).decode())

    def _block(self, X, ncol, ld, name):
        """Device pointer of a block argument after checking that the kernels
        will stay inside it: a contiguous tensor on the context's device, of
        the context's element type, holding ncol states of ld >= nd values."""
        t = self.torch
        if not isinstance(X, t.Tensor):
            raise HcuError(HCU_INVALID_ARG, f"{name}: expected a torch tensor")
        if X.device.type != "cuda" or (X.device.index or 0) != (self.device.index or 0):
            raise HcuError(HCU_INVALID_ARG, f"{name}: tensor on {X.device}, context on {self.device}")
        if X.dtype != self.dtype:
            raise HcuError(HCU_INVALID_ARG, f"{name}: dtype {X.dtype}, context uses {self.dtype}")
        if not X.is_contiguous():
            raise HcuError(HCU_INVALID_ARG, f"{name}: tensor must be contiguous")
        if ncol < 1 or ld < self.nd or (ncol - 1) * ld + self.nd > X.numel():
            raise HcuError(HCU_INVALID_ARG, f"{name}: {ncol} states of leading dimension {ld} do not fit "
                                            f"a tensor of shape {tuple(X.shape)} (nd = {self.nd})")
        return C.c_void_p(X.data_ptr())

    def close(self):
        if self.h:
            self.lib.hcu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- C ABI calls
    def set_hubbard_occupation(self, D):
        D = np.ascontiguousarray(np.asarray(D, np.float64).reshape(-1))
        self._check(self.lib.hcu_set_hubbard_occupation(self.h, _dptr(D)))

    def set_start(self, spin, ik, X0, v0):
        x = self._block(X0, self.ns, self.nd, "X0")
        v = self._block(v0, 1, self.nd, "v0")
        self._check(self.lib.hcu_set_start(self.h, spin, ik, x, v))
        self.stream.synchronize()

    def apply_h(self, X, Y, ncol=None, ld=None, spin=0, ik=0):
        """Y = H X; X, Y torch tensors of shape (ncol, ld) (state-major rows)."""
        ncol = ncol or X.shape[0]
        ld = ld or X.shape[1]
        x, y = self._block(X, ncol, ld, "X"), self._block(Y, ncol, ld, "Y")
        self._check(self.lib.hcu_apply_h(self.h, spin, ik, x, y, ncol, ld))

    def cheb_filter(self, X, Y, m, a, b, aL, ncol=None, ld=None, spin=0, ik=0):
        ncol = ncol or X.shape[0]
        ld = ld or X.shape[1]
        x, y = self._block(X, ncol, ld, "X"), self._block(Y, ncol, ld, "Y")
        self._check(self.lib.hcu_cheb_filter(self.h, spin, ik, x, y, ncol, ld, m, a, b, aL))

    def gram(self, Y, HY, ncol=None, ld=None):
        """(S, Hs) = (Y^H Y dV, Y^H HY dV) as numpy arrays."""
        ncol = ncol or Y.shape[0]
        ld = ld or Y.shape[1]
        y, hy = self._block(Y, ncol, ld, "Y"), self._block(HY, ncol, ld, "HY")
        dt = np.complex128 if self.complex else np.float64
        S = np.zeros((ncol, ncol), dt)
        Hs = np.zeros((ncol, ncol), dt)
        self._check(self.lib.hcu_gram(self.h, y, hy, ncol, ld, S.ctypes.data_as(C.POINTER(C.c_double)),
                                      Hs.ctypes.data_as(C.POINTER(C.c_double))))
        # column-major on the device side: transpose
        return S.T.copy(), Hs.T.copy()

    def rotate(self, Y, Cm, X, ncol=None, ld=None):
        """X = Y C (C numpy ncol x ncol)."""
        ncol = ncol or Y.shape[0]
        ld = ld or Y.shape[1]
        y, x = self._block(Y, ncol, ld, "Y"), self._block(X, ncol, ld, "X")
        dt = np.complex128 if self.complex else np.float64
        Cf = np.asfortranarray(np.asarray(Cm, dt))
        if Cf.shape != (ncol, ncol):
            raise HcuError(HCU_INVALID_ARG, f"C has shape {Cf.shape}, expected ({ncol}, {ncol})")
        self._check(self.lib.hcu_rotate(self.h, y, Cf.ctypes.data_as(C.POINTER(C.c_double)), x, ncol, ld))

    def lanczos_bounds(self, spin=0, ik=0, steps=10):
        tmin, up = C.c_double(), C.c_double()
        self._check(self.lib.hcu_lanczos_bounds(self.h, spin, ik, steps, C.byref(tmin), C.byref(up)))
        return tmin.value, up.value

    def chfsi_pass(self, spin=0, ik=0):
        self._check(self.lib.hcu_chfsi_pass(self.h, spin, ik))

    def update_occupations(self):
        self._check(self.lib.hcu_update_occupations(self.h))

    def scf(self, max_iter=100, first_passes=4, lanczos_steps=10, pulay_history=7, pulay_beta=0.3, tol_d=1e-7,
            tol_f=1e-7, fixed_iterations=0, verbose=False, raise_on_nonconv=True, kerker_k0=0.8, tol_rho=1e-6):
        o = hcu_scf_opts(max_iter, first_passes, lanczos_steps, pulay_history, pulay_beta, tol_d, tol_f,
                         fixed_iterations, 1 if verbose else 0, kerker_k0, tol_rho)
        r = hcu_scf_report()
        st = self.lib.hcu_scf(self.h, C.byref(o), C.byref(r))
        if st != HCU_OK and not (st == HCU_NOT_CONVERGED and not raise_on_nonconv):
            self._check(st)
        out = {k: getattr(r, k) for k, _ in hcu_scf_report._fields_}
        out["status"] = st
        return out

    def move_atoms(self, pos, extrapolate=True):
        """Move the atoms (positions [natom][3] bohr); returns the
        extrapolation coefficients (a, b, order)."""
        p = np.ascontiguousarray(np.asarray(pos, np.float64).reshape(-1))
        if p.size != 3 * len(self.prob.spec):
            raise HcuError(HCU_INVALID_ARG, "positions must be [natom][3]")
        out = np.zeros(3)
        self._check(self.lib.hcu_move_atoms(self.h, _dptr(p), 1 if extrapolate else 0, _dptr(out)))
        return float(out[0]), float(out[1]), int(out[2])

    def _occ_arg(self, occ):
        if occ is None:
            return None, None
        o = np.ascontiguousarray(np.asarray(occ, np.float64))
        if o.size != self.nspin * self.nk * self.ns:
            raise HcuError(HCU_INVALID_ARG, f"occ has {o.size} values, expected [nspin][nk][ns]")
        return o, _dptr(o)

    def hubbard_forces(self, occ=None):
        """Hubbard forces (natom, 3) in Ha/bohr of the current orbitals with
        occupations occ [nspin][nk][ns] (None: the context's)."""
        o, p = self._occ_arg(occ)
        out = np.zeros((len(self.prob.spec), 3))
        self._check(self.lib.hcu_hubbard_forces(self.h, p, _dptr(out)))
        return out

    def hubbard_stress(self, occ=None):
        """Hubbard stress tensor (3, 3) in Ha/bohr^3."""
        o, p = self._occ_arg(occ)
        out = np.zeros((3, 3))
        self._check(self.lib.hcu_hubbard_stress(self.h, p, _dptr(out)))
        return out

    def get_sizes(self):
        z = hcu_sizes()
        self._check(self.lib.hcu_get_sizes(self.h, C.byref(z)))
        return {k: getattr(z, k) for k, _ in hcu_sizes._fields_}

    def autotune(self):
        t = hcu_tuning()
        self._check(self.lib.hcu_autotune(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in hcu_tuning._fields_}

    def set_tuning(self, tile_x, tile_yt=1, ry=4, tile_z=1, halo_ring=0):
        t = hcu_tuning(tile_x, tile_yt, ry, tile_z, halo_ring, 0.0)
        self._check(self.lib.hcu_set_tuning(self.h, C.byref(t)))

    def set_profiling(self, on=True):
        self._check(self.lib.hcu_set_profiling(self.h, 1 if on else 0))

    def get_kernel_times(self):
        t = hcu_kernel_times()
        self._check(self.lib.hcu_get_kernel_times(self.h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in hcu_kernel_times._fields_}

    def scf_begin(self, max_iter=100, first_passes=4, lanczos_steps=10, pulay_history=7, pulay_beta=0.3,
                  tol_d=1e-7, tol_f=1e-7, verbose=False, kerker_k0=0.8, tol_rho=1e-6):
        self._scf_opts = hcu_scf_opts(max_iter, first_passes, lanczos_steps, pulay_history, pulay_beta, tol_d,
                                      tol_f, 0, 1 if verbose else 0, kerker_k0, tol_rho)
        self._check(self.lib.hcu_scf_begin(self.h, C.byref(self._scf_opts)))

    def scf_step(self):
        i = hcu_scf_step_info()
        self._check(self.lib.hcu_scf_step(self.h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in hcu_scf_step_info._fields_}

    def get_eigenvalues(self):
        out = np.zeros((self.nspin, self.nk, self.ns))
        self._check(self.lib.hcu_get_eigenvalues(self.h, _dptr(out)))
        return out

    def get_occupations(self):
        out = np.zeros((self.nspin, self.nk, self.ns))
        self._check(self.lib.hcu_get_occupations(self.h, _dptr(out)))
        return out

    def get_hubbard_occupation(self):
        out = np.zeros((self.nspin, max(self.nhub, 0), 5, 5))
        self._check(self.lib.hcu_get_hubbard_occupation(self.h, _dptr(out)))
        return out

    def get_energies(self):
        e = hcu_energies()
        self._check(self.lib.hcu_get_energies(self.h, C.byref(e)))
        return {k: getattr(e, k) for k, _ in hcu_energies._fields_}

    def get_potential(self):
        """(V, rho_in): the local potential of the next H application and,
        with the density-dependent Hamiltonian, the input density (else None)."""
        V = np.zeros(self.nd)
        rho = np.zeros(self.nd) if self.prob.p.hxc else None
        self._check(self.lib.hcu_get_potential(self.h, _dptr(V), _dptr(rho) if rho is not None else None))
        return V, rho

    def get_orbitals(self, spin=0, ik=0):
        X = self.torch.empty((self.ns, self.nd), dtype=self.dtype, device=self.device)
        self._check(self.lib.hcu_get_orbitals(self.h, spin, ik, C.c_void_p(X.data_ptr()), 1))
        return X

    def save_state(self):
        """The SCF state as a host byte array."""
        n = C.c_size_t()
        self._check(self.lib.hcu_state_size(self.h, C.byref(n)))
        buf = np.zeros(n.value, np.uint8)
        self._check(self.lib.hcu_save_state(self.h, C.c_void_p(buf.ctypes.data), n))
        return buf

    def load_state(self, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        self._check(self.lib.hcu_load_state(self.h, C.c_void_p(buf.ctypes.data), C.c_size_t(buf.size)))

    def descriptor(self):
        """Site descriptors (device float32 tensor [nhub][32 nspecies]) and
        frame flags (numpy int32 [nhub])."""
        nsp = len(self.cfg["species"])
        d = self.torch.empty((max(self.nhub, 1), 32 * nsp), dtype=self.torch.float32, device=self.device)
        fl = np.zeros(max(self.nhub, 1), np.int32)
        self._check(self.lib.hcu_descriptor(self.h, C.c_void_p(d.data_ptr()),
                                            fl.ctypes.data_as(C.POINTER(C.c_int))))
        return d[:self.nhub], fl[:self.nhub]

    def site_targets(self):
        out = np.zeros((max(self.nhub, 1), 30), np.float32)
        self._check(self.lib.hcu_site_targets(self.h, out.ctypes.data_as(C.POINTER(C.c_float))))
        return out[:self.nhub]

    def shell_density(self):
        out = np.zeros((max(self.nhub, 1), 15))
        self._check(self.lib.hcu_shell_density(self.h, _dptr(out)))
        return out[:self.nhub]

    def get_density(self):
        out = np.zeros((self.nspin, self.nd))
        self._check(self.lib.hcu_get_density(self.h, _dptr(out)))
        return out


class HcuBatch:
    """Several bound contexts advanced together (one persistent stencil
    launch per Chebyshev step over all their blocks).  Holds references to
    the contexts; does not own them."""

    def __init__(self, ctxs):
        self.lib = load_library()
        self.ctxs = list(ctxs)
        arr = (C.c_void_p * len(self.ctxs))(*[c.h for c in self.ctxs])
        self.h = C.c_void_p()
        st = self.lib.hcu_batch_create(arr, len(self.ctxs), C.byref(self.h))
        if st != HCU_OK:
            msg = self.lib.hcu_batch_last_error(self.h).decode() if self.h else "batch create failed"
            self.lib.hcu_batch_destroy(self.h)
            self.h = None
            raise HcuError(st, msg)

    def _check(self, st):
        if st != HCU_OK:
            raise HcuError(st, self.lib.hcu_batch_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.lib.hcu_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def chfsi_pass(self):
        self._check(self.lib.hcu_batch_chfsi_pass(self.h))

    def scf(self, max_iter=100, first_passes=4, lanczos_steps=10, pulay_history=7, pulay_beta=0.3, tol_d=1e-7,
            tol_f=1e-7, fixed_iterations=0, verbose=False, raise_on_nonconv=True, kerker_k0=0.8, tol_rho=1e-6):
        o = hcu_scf_opts(max_iter, first_passes, lanczos_steps, pulay_history, pulay_beta, tol_d, tol_f,
                         fixed_iterations, 1 if verbose else 0, kerker_k0, tol_rho)
        reps = (hcu_scf_report * len(self.ctxs))()
        st = self.lib.hcu_batch_scf(self.h, C.byref(o), reps)
        if st != HCU_OK and not (st == HCU_NOT_CONVERGED and not raise_on_nonconv):
            self._check(st)
        return [{k: getattr(r, k) for k, _ in hcu_scf_report._fields_} for r in reps]


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class HcuMlp:
    """The site MLP of the learned occupation guess, bound to a torch
    workspace on the current stream."""

    def __init__(self, dims, max_batch, device="cuda:0"):
        import torch
        self.lib = load_library()
        self.torch = torch
        self.dims = list(dims)
        d = (C.c_int * len(self.dims))(*self.dims)
        self.h = C.c_void_p()
        st = self.lib.hcu_mlp_create(d, len(self.dims) - 1, int(max_batch), C.byref(self.h))
        if st != HCU_OK:
            msg = self.lib.hcu_mlp_last_error(self.h).decode() if self.h else "create failed"
            self.lib.hcu_mlp_destroy(self.h)
            self.h = None
            raise HcuError(st, msg)
        n = C.c_int64()
        self._check(self.lib.hcu_mlp_param_count(self.h, C.byref(n)))
        self.nparam = n.value
        nb = C.c_size_t()
        self._check(self.lib.hcu_mlp_workspace_size(self.h, C.byref(nb)))
        self.device = torch.device(device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self._check(self.lib.hcu_mlp_bind(self.h, C.c_void_p(ptr), C.c_size_t(nb.value),
                                          C.c_void_p(self.stream.cuda_stream)))

    def _check(self, st):
        if st != HCU_OK:
            raise HcuError(st, self.lib.hcu_mlp_last_error(self.h).decode())

    def close(self):
        if self.h:
            self.lib.hcu_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        p = np.ascontiguousarray(np.asarray(theta, np.float32))
        assert p.size == self.nparam
        self._check(self.lib.hcu_mlp_set_params(self.h, _fptr(p)))

    def get_params(self):
        p = np.zeros(self.nparam, np.float32)
        self._check(self.lib.hcu_mlp_get_params(self.h, _fptr(p)))
        return p

    def set_scaling(self, in_mean, in_sd, out_mean, out_sd):
        a = [np.ascontiguousarray(np.asarray(v, np.float32)) for v in (in_mean, in_sd, out_mean, out_sd)]
        self._check(self.lib.hcu_mlp_set_scaling(self.h, *[_fptr(v) for v in a]))

    def get_scaling(self):
        a = [np.zeros(self.dims[0], np.float32), np.zeros(self.dims[0], np.float32),
             np.zeros(self.dims[-1], np.float32), np.zeros(self.dims[-1], np.float32)]
        self._check(self.lib.hcu_mlp_get_scaling(self.h, *[_fptr(v) for v in a]))
        return a

    def _mat(self, A, rows, width, name):
        """Device pointer of a row-major FP32 matrix argument holding at least
        `rows` rows of `width` values on the object's device."""
        t = self.torch
        if not isinstance(A, t.Tensor) or A.device.type != "cuda" or \
                (A.device.index or 0) != (self.device.index or 0):
            raise HcuError(HCU_INVALID_ARG, f"{name}: expected a tensor on {self.device}")
        if A.dtype != t.float32 or not A.is_contiguous() or A.dim() != 2:
            raise HcuError(HCU_INVALID_ARG, f"{name}: expected a contiguous 2-D float32 tensor")
        if A.shape[1] != width or A.shape[0] < rows:
            raise HcuError(HCU_INVALID_ARG, f"{name}: shape {tuple(A.shape)}, need >= {rows} rows of {width}")
        return C.c_void_p(A.data_ptr())

    def _rows(self, X, T, idx, batch):
        """Pointers of a training batch: X, T and the optional row index
        (int32, every entry a row of X and T)."""
        nrow = int(X.shape[0]) if hasattr(X, "shape") else 0
        x = self._mat(X, 1 if idx is not None else batch, self.dims[0], "X")
        tt = self._mat(T, nrow, self.dims[-1], "T")
        if idx is None:
            return x, tt, C.c_void_p(0)
        t = self.torch
        if not isinstance(idx, t.Tensor) or idx.dtype != t.int32 or idx.dim() != 1 or not idx.is_contiguous() \
                or idx.device != X.device or idx.shape[0] < batch:
            raise HcuError(HCU_INVALID_ARG, "idx: expected a contiguous 1-D int32 tensor on the device")
        if batch > 0:
            lo, hi = int(idx[:batch].min()), int(idx[:batch].max())
            if lo < 0 or hi >= nrow:
                raise HcuError(HCU_INVALID_ARG, f"idx: rows {lo}..{hi} outside 0..{nrow - 1}")
        return x, tt, C.c_void_p(idx.data_ptr())

    def fit_scaling(self, X, T):
        rows = int(X.shape[0])
        x, tt = self._mat(X, rows, self.dims[0], "X"), self._mat(T, rows, self.dims[-1], "T")
        self._check(self.lib.hcu_mlp_fit_scaling(self.h, x, tt, rows))

    def forward(self, X, bf16=False):
        X = X.contiguous()
        x = self._mat(X, int(X.shape[0]), self.dims[0], "X")
        Y = self.torch.empty((X.shape[0], self.dims[-1]), dtype=self.torch.float32, device=self.device)
        self._check(self.lib.hcu_mlp_forward(self.h, x, int(X.shape[0]), C.c_void_p(Y.data_ptr()),
                                             1 if bf16 else 0))
        return Y

    def gradient(self, X, T, idx=None, batch=None):
        batch = int(idx.shape[0]) if idx is not None else int(X.shape[0]) if batch is None else batch
        x, tt, ip = self._rows(X, T, idx, batch)
        g = np.zeros(self.nparam, np.float32)
        loss = C.c_double()
        self._check(self.lib.hcu_mlp_gradient(self.h, x, tt, ip, batch, _fptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, X, T, idx=None, lr=1e-3, want_loss=True):
        batch = int(idx.shape[0]) if idx is not None else int(X.shape[0])
        x, tt, ip = self._rows(X, T, idx, batch)
        loss = C.c_double()
        self._check(self.lib.hcu_mlp_train_step(self.h, x, tt, ip, batch, C.c_float(lr),
                                                C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def guess(self, ctx, bf16=True):
        """Set ctx's occupation matrices from the network; returns the raw
        outputs [nhub][dims[-1]]."""
        out = np.zeros((max(ctx.nhub, 1), self.dims[-1]), np.float32)
        st = self.lib.hcu_mlp_guess(ctx.h, self.h, 1 if bf16 else 0, _fptr(out))
        if st != HCU_OK:
            msg = self.lib.hcu_mlp_last_error(self.h).decode() or self.lib.hcu_last_error(ctx.h).decode()
            raise HcuError(st, msg)
        return out[:ctx.nhub]


def gram_noalloc(Y, HY, ncol, nd, ld, precision, is_complex, dv, S, Hs, stream=None):
    """hcu_gram_noalloc on device tensors (S, Hs: ncol x ncol device buffers
    written column-major); returns the status code."""
    lib = load_library()
    st = stream.cuda_stream if stream is not None else 0
    return lib.hcu_gram_noalloc(C.c_void_p(Y.data_ptr()), C.c_void_p(HY.data_ptr()), int(ncol), int(nd), int(ld),
                                HCU_MIXED if precision == "mixed" else HCU_FP64, 1 if is_complex else 0,
                                float(dv), C.c_void_p(S.data_ptr()), C.c_void_p(Hs.data_ptr()), C.c_void_p(st))


def start_inputs(ctx, cfg, spin=0, ik=0):
    """Seeded start block and Lanczos vector of (spin, ik) as device tensors
    in the context precision."""
    import torch
    import workloads
    cplx = ctx.complex
    X0 = workloads.random_block(ctx.nd, ctx.ns, workloads.start_seed(cfg, spin, ik), cplx)
    v0 = workloads.random_vector(ctx.nd, workloads.lanczos_seed(cfg, spin, ik), cplx)
    X0 = torch.from_numpy(X0).to(ctx.device).to(ctx.dtype)
    v0 = torch.from_numpy(v0).to(ctx.device).to(ctx.dtype)
    return X0, v0


def initial_occupation(ctx, cfg):
    """Diagonal initial D (isolated-atom average occupation), [nspin][nhub][5][5]."""
    import workloads
    D = np.zeros((ctx.nspin, ctx.nhub, 5, 5))
    for s in range(ctx.nspin):
        for h, g in enumerate(workloads.initial_occupation_diag(cfg, s)):
            D[s, h] = g * np.eye(5)
    return D
