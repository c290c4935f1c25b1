"""Python binding of liblam (argument marshalling only).

Every numerical step runs in the HIP kernels of ``liblam.so``; this module
checks shapes and dtypes, passes device pointers of torch tensors and the
current torch stream, and converts error codes into exceptions.  If the
library is not built, every entry point raises: there is no CPU fallback.

The names follow the C ABI in ``include/lam.h`` (``lam_create`` ...).  The
class :class:`Propagator` wraps one context, and :class:`LeastActionPropagate`
is the ``torch.autograd.Function`` that propagates a wavefunction over many
steps and differentiates a real loss of the final state with respect to the
initial state, the potential V0 and the Fourier pulse amplitudes (adjoint
solve of every step, recomputing the forward solve from step-boundary
checkpoints).
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblam.so")

LAM_OK, LAM_EINVAL, LAM_ENOMEM, LAM_EHIP, LAM_ENOCONV, LAM_EDIVERGED, LAM_ESTATE = 0, -1, -2, -3, -4, -5, -6
LAM_ETOOBIG = -7
LAM_MAX_NT = 8
LAM_MAX_BLOCK = 64
LAM_MAX_INNER = 32
LAM_MAX_SPLIT = 8
PULSE = {"none": 0, "sin2": 1, "fourier": 2, "sin2+fourier": 3}
PRECISION = {"fp64": 0, "mixed": 1}
INTERP = {"linear": 0, "constant": 1}
COARSE_OP = {"rediscretised": 0, "galerkin": 1}
TIME_FACTOR = {"shared": 0, "stored": 1}


class LamError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class NotConverged(LamError):
    pass


class LamGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("h", ctypes.c_double),
                ("periodic", ctypes.c_int), ("block", ctypes.c_int * 3), ("levels", ctypes.c_int),
                ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("nu_coarse", ctypes.c_int),
                ("interp", ctypes.c_int), ("coarse_op", ctypes.c_int)]


class LamTime(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int), ("dt", ctypes.c_double)]


class LamHam(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("v0", ctypes.c_void_p), ("field_axis", ctypes.c_int),
                ("pulse_kind", ctypes.c_int), ("e0", ctypes.c_double), ("omega", ctypes.c_double),
                ("t_total", ctypes.c_double), ("n_coef", ctypes.c_int),
                ("coef", ctypes.POINTER(ctypes.c_double))]


class LamSolver(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("tol", ctypes.c_double), ("max_cycles", ctypes.c_int),
                ("n_inner", ctypes.c_int), ("time_factor", ctypes.c_int), ("coarse_reduction", ctypes.c_double),
                ("max_split", ctypes.c_int), ("inner_tol", ctypes.c_double)]


class LamPWRegime(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int), ("n_t", ctypes.c_int), ("mode", ctypes.c_int), ("kappa", ctypes.c_double),
                ("nu", ctypes.c_double)]


PW_MODE = {"one": 0, "simultaneous": 1, "intergrid": 2}
LAM_PW_MAX_UNKNOWNS = 72


class LamStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("sweeps_fine", ctypes.c_int), ("resid0", ctypes.c_double),
                ("resid", ctypes.c_double), ("t_factor_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("resid0_last", ctypes.c_double), ("resid_last", ctypes.c_double),
                ("coarse_sweeps", ctypes.c_int), ("coarse_unmet", ctypes.c_int), ("substeps", ctypes.c_int),
                ("split_depth", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI = ctypes.POINTER(ctypes.c_int)
SIGNATURES = {
    "lam_create": (_I, [ctypes.POINTER(LamGrid), ctypes.POINTER(LamTime), ctypes.POINTER(LamHam),
                        ctypes.POINTER(LamSolver), _P, ctypes.POINTER(_P)]),
    "lam_destroy": (_I, [_P]),
    "lam_set_pulse": (_I, [_P, _I, _PD]),
    "lam_set_potential": (_I, [_P, _P]),
    "lam_residual_action": (_I, [_P, _D, _P, _P, _P, _P, _P, _PD]),
    "lam_residual_adjoint": (_I, [_P, _D, _P, _P, _P, _P, _P, _PD]),
    "lam_set_state": (_I, [_P, _D, _P, _P, _P]),
    "lam_set_adjoint_state": (_I, [_P, _D, _P, _P, _P]),
    "lam_get_state": (_I, [_P, _P, _P]),
    "lam_relax_sweep": (_I, [_P, _I, _I]),
    "lam_vcycle": (_I, [_P, _PD]),
    "lam_solve_step": (_I, [_P, _D, _P, _P, ctypes.POINTER(LamStats)]),
    "lam_propagate": (_I, [_P, _D, _I, _P, _P, ctypes.POINTER(LamStats)]),
    "lam_adjoint_step": (_I, [_P, _D, _P, _P, _P, _P, _PD, ctypes.POINTER(LamStats)]),
    "lam_adjoint_step_stored": (_I, [_P, _D, _P, _P, _P, _P, _PD, ctypes.POINTER(LamStats)]),
    "lam_restrict": (_I, [_P, _I, _P, _P, _P, _P]),
    "lam_prolong_add": (_I, [_P, _I, _P, _P, _P, _P]),
    "lam_level_shape": (_I, [_P, _I, _PI]),
    "lam_block_factor": (_I, [_P, _I, _I, _PD, _PD]),
    "lam_pass_stats": (_I, [_P, _I, ctypes.POINTER(ctypes.c_longlong)]),
    "lam_set_refinement": (_I, [_P, _P]),
    "lam_block_detail": (_I, [_P, _P, _P]),
    "lam_plane_wave_map": (_I, [ctypes.POINTER(LamPWRegime), _I, _PD, _I, _PD, _P, _P, _P]),
    "lam_residual_action_noalloc": (_I, [ctypes.POINTER(LamGrid), ctypes.POINTER(LamTime), ctypes.POINTER(LamHam),
                                         _D, _P, _P, _P, _P, _P, _P, _P]),
    "lam_profile": (_I, [_P, _I]),
    "lam_profile_read": (_I, [_P, _PI, _PD]),
    "lam_strerror": (ctypes.c_char_p, [_I]),
}

_lib = None


def load_library(path=None):
    """Load liblam.so (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"liblam.so not built ({path}); run `python -m paper_1111_4363_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def strerror(code):
    try:
        return load_library().lam_strerror(code).decode()
    except Exception:
        return "error"


def _check(code, where):
    if code == LAM_ENOCONV:
        raise NotConverged(code, where)
    if code != LAM_OK:
        raise LamError(code, where)


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _pulse_fields(pulse):
    pulse = dict(pulse or {})
    kind = pulse.get("kind", "none")
    coef = [float(a) for a in pulse.get("coef", [])]
    return PULSE[kind], float(pulse.get("e0", 0.0)), float(pulse.get("omega", 0.0)), \
        float(pulse.get("t_total", 0.0)), coef


def _describe(shape, h, v0, n_t, dt, block, levels=1, nu_pre=1, nu_post=1, nu_coarse=2, interp="linear",
              periodic=False, mass=1.0, field_axis=-1, pulse=None, coarse_op="rediscretised"):
    """The lam_grid, lam_time and lam_ham structs (and the host array the last points to)."""
    shape = tuple(int(s) for s in shape)
    block = tuple(int(b) for b in block)
    dim = len(shape)
    if dim not in (1, 2, 3) or len(block) != dim:
        raise ValueError("shape and block must have the same rank 1, 2 or 3")
    npts = 1
    for s in shape:
        npts *= s
    g = LamGrid()
    g.dim = dim
    for a in range(3):
        g.n[a] = shape[a] if a < dim else 1
        g.block[a] = block[a] if a < dim else 1
    g.h, g.periodic, g.levels = float(h), int(bool(periodic)), int(levels)
    g.nu_pre, g.nu_post, g.nu_coarse, g.interp = int(nu_pre), int(nu_post), int(nu_coarse), INTERP[interp]
    g.coarse_op = COARSE_OP[coarse_op]
    t = LamTime(int(n_t), float(dt))
    kind, e0, omega, t_total, coef = _pulse_fields(pulse)
    carr = (ctypes.c_double * max(1, len(coef)))(*coef)
    ham = LamHam()
    ham.mass = float(mass)
    ham.v0 = _ptr(v0, torch.float64, npts, "v0")
    ham.field_axis = int(field_axis) % dim
    ham.pulse_kind, ham.e0, ham.omega, ham.t_total = kind, e0, omega, t_total
    ham.n_coef = len(coef)
    ham.coef = carr
    return g, t, ham, carr, coef, npts


def residual_action_noalloc(shape, h, v0, n_t, dt, t0, psi0, c, lam, rho=None, sigma=None, norm=None,
                            block=None, periodic=False, mass=1.0, field_axis=-1, pulse=None, stream=None):
    """lam_residual_action_noalloc: the action residual without a context or any
    device allocation.  v0, psi0, c, lam: device inputs; rho, sigma: device outputs
    or None; norm: a device float64 tensor of one element or None.  Returns the
    library's code (0 on success); nothing is raised."""
    lib = load_library()
    block = block if block is not None else (1,) * len(shape)
    v0 = v0.contiguous()
    g, t, ham, carr, _, P = _describe(shape, h, v0, n_t, dt, block, periodic=periodic, mass=mass,
                                      field_axis=field_axis, pulse=pulse)
    nt = int(n_t)
    return lib.lam_residual_action_noalloc(
        ctypes.byref(g), ctypes.byref(t), ctypes.byref(ham), float(t0), _ptr(psi0, torch.complex128, P, "psi0"),
        _ptr(c, torch.complex128, P * nt, "c"), _ptr(lam, torch.complex128, P, "lam"),
        _ptr(rho, torch.complex128, P * nt, "rho"), _ptr(sigma, torch.complex128, P, "sigma"),
        _ptr(norm, torch.float64, 1, "norm"), _stream_handle(stream))


def plane_wave_map(n_x, n_t, mode, kappa, nu, k, w, stream=None, device="cuda"):
    """lam_plane_wave_map: residual-norm and action ratios of one relaxation of the
    trial exp(i(k x + w t)) for every (w, k) of the grid; returns two device float64
    tensors of shape (len(w), len(k))."""
    lib = load_library()
    k = [float(v) for v in k]
    w = [float(v) for v in w]
    rg = LamPWRegime(int(n_x), int(n_t), PW_MODE[mode], float(kappa), float(nu))
    rr = torch.empty((len(w), len(k)), dtype=torch.float64, device=device)
    ar = torch.empty_like(rr)
    ka = (ctypes.c_double * len(k))(*k)
    wa = (ctypes.c_double * len(w))(*w)
    _check(lib.lam_plane_wave_map(ctypes.byref(rg), len(k), ka, len(w), wa, _ptr(rr, torch.float64),
                                  _ptr(ar, torch.float64), _stream_handle(stream)), "lam_plane_wave_map")
    return rr, ar


class Propagator:
    """One liblam context: a grid, a time basis, a Hamiltonian and a solver."""

    def __init__(self, shape, h, v0, n_t, dt, block, levels=1, nu_pre=1, nu_post=1, nu_coarse=2,
                 interp="linear", periodic=False, mass=1.0, field_axis=-1, pulse=None,
                 precision="fp64", tol=1e-10, max_cycles=50, n_inner=-1, time_factor="shared", coarse_reduction=0.0,
                 max_split=0, coarse_op="rediscretised", inner_tol=0.0, stream=None):
        lib = load_library()
        v0 = v0.contiguous()
        g, t, ham, self._coef, coef, self.npts = _describe(shape, h, v0, n_t, dt, block, levels, nu_pre, nu_post,
                                                           nu_coarse, interp, periodic, mass, field_axis, pulse,
                                                           coarse_op)
        self.shape = tuple(int(s) for s in shape)
        self.block = tuple(int(b) for b in block)
        self.n_t, self.dt, self.h = int(n_t), float(dt), float(h)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.n_coef = len(coef)
        s = LamSolver(PRECISION[precision], float(tol), int(max_cycles), int(n_inner), TIME_FACTOR[time_factor],
                      float(coarse_reduction), int(max_split), float(inner_tol))
        self.levels = int(levels)
        self.precision = precision
        # what the context holds (the autograd function restores its own inputs)
        self._v0_held = v0.detach().clone()
        self._coef_held = list(coef)
        self.refined = False   # a refinement set by set_refinement
        h_ctx = ctypes.c_void_p()
        _check(lib.lam_create(ctypes.byref(g), ctypes.byref(t), ctypes.byref(ham), ctypes.byref(s),
                              _stream_handle(self.stream), ctypes.byref(h_ctx)), "lam_create")
        self._ctx = h_ctx
        self._lib = lib
        self.device = v0.device

    # -- lifetime ----------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.lam_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n, dtype=torch.complex128):
        return torch.empty(n, dtype=dtype, device=self.device)

    # -- C ABI mirrors -----------------------------------------------------
    def set_pulse(self, coef):
        coef = [float(a) for a in coef]
        arr = (ctypes.c_double * max(1, len(coef)))(*coef)
        _check(self._lib.lam_set_pulse(self._ctx, len(coef), arr), "lam_set_pulse")
        self._coef_held = coef

    def set_potential(self, v0):
        v0 = v0.contiguous()
        _check(self._lib.lam_set_potential(self._ctx, _ptr(v0, torch.float64, self.npts, "v0")),
               "lam_set_potential")
        self._v0_held = v0.detach().clone()

    def hold(self, v0, coef):
        """Make the context hold potential v0 and pulse amplitudes coef, calling
        lam_set_potential / lam_set_pulse only for what differs from what it holds."""
        v0 = v0.detach().contiguous()
        if v0.shape != self._v0_held.shape or not torch.equal(v0, self._v0_held):
            self.set_potential(v0)
        coef = [float(a) for a in coef]
        if self.n_coef and coef != self._coef_held:
            self.set_pulse(coef)

    def residual_action(self, t0, psi0, c, lam, want_fields=True):
        P, nt = self.npts, self.n_t
        rho = self._new(P * nt) if want_fields else None
        sig = self._new(P) if want_fields else None
        N = ctypes.c_double()
        _check(self._lib.lam_residual_action(self._ctx, float(t0), _ptr(psi0, torch.complex128, P, "psi0"),
                                             _ptr(c, torch.complex128, P * nt, "c"),
                                             _ptr(lam, torch.complex128, P, "lam"),
                                             _ptr(rho, torch.complex128), _ptr(sig, torch.complex128),
                                             ctypes.byref(N)), "lam_residual_action")
        return rho, sig, N.value

    def residual_adjoint(self, t0, g, mu_c, mu_lam, want_fields=True):
        P, nt = self.npts, self.n_t
        rho = self._new(P * nt) if want_fields else None
        sig = self._new(P) if want_fields else None
        N = ctypes.c_double()
        _check(self._lib.lam_residual_adjoint(self._ctx, float(t0), _ptr(g, torch.complex128, P, "g"),
                                              _ptr(mu_c, torch.complex128, P * nt, "mu_c"),
                                              _ptr(mu_lam, torch.complex128, P, "mu_lam"),
                                              _ptr(rho, torch.complex128), _ptr(sig, torch.complex128),
                                              ctypes.byref(N)), "lam_residual_adjoint")
        return rho, sig, N.value

    def set_state(self, t0, psi0, c, lam):
        P, nt = self.npts, self.n_t
        _check(self._lib.lam_set_state(self._ctx, float(t0), _ptr(psi0, torch.complex128, P, "psi0"),
                                       _ptr(c, torch.complex128, P * nt, "c"),
                                       _ptr(lam, torch.complex128, P, "lam")), "lam_set_state")

    def set_adjoint_state(self, t0, g, mu_c, mu_lam):
        P, nt = self.npts, self.n_t
        _check(self._lib.lam_set_adjoint_state(self._ctx, float(t0), _ptr(g, torch.complex128, P, "g"),
                                               _ptr(mu_c, torch.complex128, P * nt, "mu_c"),
                                               _ptr(mu_lam, torch.complex128, P, "mu_lam")),
               "lam_set_adjoint_state")

    def get_state(self):
        c, lam = self._new(self.npts * self.n_t), self._new(self.npts)
        _check(self._lib.lam_get_state(self._ctx, _ptr(c, torch.complex128), _ptr(lam, torch.complex128)),
               "lam_get_state")
        return c, lam

    def set_refinement(self, active):
        """lam_set_refinement: refine the finest level only on the subvolumes whose
        flag is set (host array, one per subvolume in C order of subvolume
        coordinates); None clears the refinement."""
        if active is None:
            _check(self._lib.lam_set_refinement(self._ctx, None), "lam_set_refinement")
            self.refined = False
            return
        import numpy as np
        a = np.ascontiguousarray(np.asarray(active, dtype=np.uint8).ravel())
        nblk = 1
        for s_, b_ in zip(self.shape, self.block):
            nblk *= s_ // b_
        if a.size != nblk:
            raise ValueError(f"one flag per finest subvolume expected ({nblk}), got {a.size}")
        _check(self._lib.lam_set_refinement(self._ctx, a.ctypes.data_as(ctypes.c_void_p)), "lam_set_refinement")
        self.refined = True

    def block_detail(self, psi):
        """lam_block_detail: Haar detail energy of psi per finest subvolume (numpy)."""
        import numpy as np
        nblk = 1
        for s_, b_ in zip(self.shape, self.block):
            nblk *= s_ // b_
        out = np.zeros(nblk)
        _check(self._lib.lam_block_detail(self._ctx, _ptr(psi, torch.complex128, self.npts, "psi"),
                                          out.ctypes.data_as(ctypes.c_void_p)), "lam_block_detail")
        return out

    def relax_sweep(self, colour, level=0):
        _check(self._lib.lam_relax_sweep(self._ctx, int(level), int(colour)), "lam_relax_sweep")

    def vcycle(self, norm=True):
        """One V-cycle; returns N afterwards (synchronises), or None with norm=False
        (queued on the stream only)."""
        if not norm:
            _check(self._lib.lam_vcycle(self._ctx, None), "lam_vcycle")
            return None
        N = ctypes.c_double()
        _check(self._lib.lam_vcycle(self._ctx, ctypes.byref(N)), "lam_vcycle")
        return N.value

    def solve_step(self, t0, psi_in, psi_out=None, allow_noconv=False):
        P = self.npts
        if psi_out is None:
            psi_out = self._new(P)
        st = LamStats()
        code = self._lib.lam_solve_step(self._ctx, float(t0), _ptr(psi_in, torch.complex128, P, "psi_in"),
                                        _ptr(psi_out, torch.complex128, P, "psi_out"), ctypes.byref(st))
        if not (allow_noconv and code == LAM_ENOCONV):
            _check(code, "lam_solve_step")
        return psi_out, st.as_dict()

    def adjoint_step(self, t0, psi_in, g_out, dv0, dcoef=None):
        """Returns (g_in, stats); dv0 (device float64) and dcoef (host list) are accumulated."""
        P = self.npts
        g_in = self._new(P)
        st = LamStats()
        nc = self.n_coef
        arr = (ctypes.c_double * max(1, nc))(*(dcoef if dcoef is not None else [0.0] * nc))
        _check(self._lib.lam_adjoint_step(self._ctx, float(t0), _ptr(psi_in, torch.complex128, P, "psi_in"),
                                          _ptr(g_out, torch.complex128, P, "g_out"),
                                          _ptr(g_in, torch.complex128, P, "g_in"),
                                          _ptr(dv0, torch.float64, P, "dv0"),
                                          arr if dcoef is not None else None, ctypes.byref(st)),
               "lam_adjoint_step")
        if dcoef is not None:
            for q in range(nc):
                dcoef[q] = arr[q]
        return g_in, st.as_dict()

    def adjoint_step_stored(self, t0, c_fwd, g_out, dv0, dcoef=None):
        """As adjoint_step, from the step's converged forward coefficients c_fwd
        (get_state after its solve_step) instead of a recomputed forward solve."""
        P, nt = self.npts, self.n_t
        g_in = self._new(P)
        st = LamStats()
        nc = self.n_coef
        arr = (ctypes.c_double * max(1, nc))(*(dcoef if dcoef is not None else [0.0] * nc))
        _check(self._lib.lam_adjoint_step_stored(self._ctx, float(t0), _ptr(c_fwd, torch.complex128, P * nt, "c_fwd"),
                                                 _ptr(g_out, torch.complex128, P, "g_out"),
                                                 _ptr(g_in, torch.complex128, P, "g_in"),
                                                 _ptr(dv0, torch.float64, P, "dv0"),
                                                 arr if dcoef is not None else None, ctypes.byref(st)),
               "lam_adjoint_step_stored")
        if dcoef is not None:
            for q in range(nc):
                dcoef[q] = arr[q]
        return g_in, st.as_dict()

    def level_shape(self, level):
        n = (ctypes.c_int * 3)()
        _check(self._lib.lam_level_shape(self._ctx, int(level), n), "lam_level_shape")
        return tuple(n[a] for a in range(len(self.shape)))

    def level_points(self, level):
        p = 1
        for s in self.level_shape(level):
            p *= s
        return p

    def restrict(self, level, rho_f, sigma_f):
        Pf, Pc, nt = self.level_points(level), self.level_points(level + 1), self.n_t
        rho_c, sig_c = self._new(Pc * nt), self._new(Pc)
        _check(self._lib.lam_restrict(self._ctx, int(level), _ptr(rho_f, torch.complex128, Pf * nt, "rho_f"),
                                      _ptr(sigma_f, torch.complex128, Pf, "sigma_f"),
                                      _ptr(rho_c, torch.complex128), _ptr(sig_c, torch.complex128)),
               "lam_restrict")
        return rho_c, sig_c

    def prolong_add(self, level, c_c, lam_c, c_f, lam_f):
        Pf, Pc, nt = self.level_points(level), self.level_points(level + 1), self.n_t
        _check(self._lib.lam_prolong_add(self._ctx, int(level), _ptr(c_c, torch.complex128, Pc * nt, "c_c"),
                                         _ptr(lam_c, torch.complex128, Pc, "lam_c"),
                                         _ptr(c_f, torch.complex128, Pf * nt, "c_f"),
                                         _ptr(lam_f, torch.complex128, Pf, "lam_f")), "lam_prolong_add")

    def block_factor(self, level, block):
        b = 1
        for x in self.block:
            b *= x
        vecs = (ctypes.c_double * (b * b))()
        vals = (ctypes.c_double * b)()
        _check(self._lib.lam_block_factor(self._ctx, int(level), int(block), vecs, vals), "lam_block_factor")
        import numpy as np
        return np.array(vecs[:]).reshape(b, b), np.array(vals[:])

    def pass_stats(self, level=0):
        """(histogram of inner passes of the last solve of every subvolume on the level,
        number of subvolumes left unsolved): lam_pass_stats."""
        hist = (ctypes.c_longlong * (LAM_MAX_INNER + 2))()
        _check(self._lib.lam_pass_stats(self._ctx, int(level), hist), "lam_pass_stats")
        return [int(hist[k]) for k in range(LAM_MAX_INNER + 1)], int(hist[LAM_MAX_INNER + 1])

    def profile(self, enable):
        _check(self._lib.lam_profile(self._ctx, int(enable)), "lam_profile")

    def profile_read(self):
        n = ctypes.c_int()
        ms = ctypes.c_double()
        _check(self._lib.lam_profile_read(self._ctx, ctypes.byref(n), ctypes.byref(ms)), "lam_profile_read")
        return n.value, ms.value

    # -- conveniences ------------------------------------------------------
    def propagate(self, psi0, n_steps, t_start=0.0, keep=False):
        """n_steps steps from t_start.  keep=False: one lam_propagate call (no
        host round trip between steps); returns (psi, [summed stats]).
        keep=True: step by step, returns ([psi_0, ..., psi_K], [stats per step])."""
        psi = psi0.contiguous()
        if not keep:
            if n_steps == 0:
                return psi.clone(), [LamStats().as_dict()]
            P = self.npts
            out = self._new(P)
            st = LamStats()
            _check(self._lib.lam_propagate(self._ctx, float(t_start), int(n_steps),
                                           _ptr(psi, torch.complex128, P, "psi0"),
                                           _ptr(out, torch.complex128, P, "psi_out"), ctypes.byref(st)),
                   "lam_propagate")
            return out, [st.as_dict()]
        out = [psi]
        stats = []
        for k in range(n_steps):
            psi, st = self.solve_step(t_start + k * self.dt, psi)
            stats.append(st)
            out.append(psi)
        return out, stats


class LeastActionPropagate(torch.autograd.Function):
    """psi_K = F_{K-1}( ... F_0(psi_0)) with one least-action solve per step.

    Inputs: psi0 (complex128, device), v0 (float64, device) and coef
    (float64, host or device; the Fourier amplitudes of the pulse).  With
    store=False only the step-boundary wavefunctions are kept, and backward
    recomputes each step's forward solve from its checkpoint before it solves
    the adjoint step system with the same relaxation and multigrid machinery
    (lam_adjoint_step).  With store=True the forward coefficients of every step
    are kept as well (P n_t complex values per step, in device memory), and
    backward solves only the adjoint systems (lam_adjoint_step_stored); steps
    whose forward solve was split, or solved on the adaptive tree, keep the
    recomputing form.
    """

    @staticmethod
    def forward(ctx, psi0, v0, coef, prop, n_steps, t_start, store=False):
        ctx.v0 = v0.detach().contiguous().clone()
        ctx.coef = [float(a) for a in coef.detach().cpu().tolist()] if prop.n_coef else []
        prop.hold(ctx.v0, ctx.coef)
        n_steps, t_start = int(n_steps), float(t_start)
        stored = [None] * n_steps
        if store:
            psis = [psi0.detach().contiguous()]
            for k in range(n_steps):
                psi, st = prop.solve_step(t_start + k * prop.dt, psis[-1])
                psis.append(psi)
                if st["substeps"] == 1 and not prop.refined:
                    stored[k] = prop.get_state()[0]
        else:
            psis, _ = prop.propagate(psi0.detach().contiguous(), n_steps, t_start, keep=True)
        ctx.prop = prop
        ctx.n_steps = n_steps
        ctx.t_start = t_start
        ctx.checkpoints = psis[:-1]
        ctx.stored = stored
        ctx.coef_device = coef.device
        return psis[-1].clone()

    @staticmethod
    def backward(ctx, grad_out):
        prop = ctx.prop
        # the system this forward solved: another forward on the same Propagator
        # since then may have replaced the potential or the pulse
        prop.hold(ctx.v0, ctx.coef)
        # torch passes 2 dL/dpsi^*; the library works with dL/dpsi^*
        g = (0.5 * grad_out).contiguous()
        dv0 = torch.zeros(prop.npts, dtype=torch.float64, device=prop.device)
        dcoef = [0.0] * prop.n_coef
        for k in reversed(range(ctx.n_steps)):
            t_k = ctx.t_start + k * prop.dt
            if ctx.stored[k] is not None:
                g, _ = prop.adjoint_step_stored(t_k, ctx.stored[k], g, dv0, dcoef)
            else:
                g, _ = prop.adjoint_step(t_k, ctx.checkpoints[k], g, dv0, dcoef)
        grad_psi0 = 2.0 * g
        grad_coef = torch.tensor(dcoef, dtype=torch.float64, device=ctx.coef_device)
        return grad_psi0, dv0, grad_coef, None, None, None, None


def propagate_differentiable(prop, psi0, v0, coef, n_steps, t_start=0.0, store=False):
    """psi_K of n_steps least-action steps, differentiable in psi0, v0 and coef;
    store=True keeps every step's forward coefficients for the backward pass
    (LeastActionPropagate)."""
    return LeastActionPropagate.apply(psi0, v0, coef, prop, n_steps, t_start, store)
