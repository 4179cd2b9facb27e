"""Thin Python binding of the C ABI in ``include/ffmg.h`` (``libffmg.so``).

Argument marshalling only: torch supplies device memory and the stream, every
step of the method runs in the library's HIP kernels.  There is no CPU
fallback -- importing works without a GPU, but any call needs the built
library and a gfx950 device, and fails loudly otherwise.

Names follow the C entry points: ``mg_setup``, ``mg_rhs_plane_wave``,
``mg_vcycle``, ``mg_fmg``, ``mg_solve``, ``farfield_map``, ``mg_apply``, ``mg_smooth``,
``mg_residual_norm``, ``mg_destroy``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffmg.so")

FFMG_OK, FFMG_EINVAL, FFMG_ENOMEM, FFMG_EDEVICE, FFMG_ENOCONV, FFMG_ERANGE, FFMG_ENAN = range(7)
HELMHOLTZ, SCHRODINGER = 0, 1
FP64, FP32_IR = 0, 1
SMOOTH_JACOBI, SMOOTH_LEARNED, SMOOTH_GMRES, SMOOTH_RBGS = 0, 1, 2, 3
FF_FP64, FF_BF16X3, FF_BF16X6 = 0, 1, 2


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("gamma", ctypes.c_double), ("kind", ctypes.c_int),
                ("k0", ctypes.c_double), ("energy", ctypes.c_double), ("coef", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("omega", ctypes.c_double),
                ("coarsest_n", ctypes.c_int), ("max_cycles", ctypes.c_int), ("precision", ctypes.c_int),
                ("smoother", ctypes.c_int), ("smoother_weights", ctypes.c_void_p),
                ("ff_precision", ctypes.c_int), ("tile_config", ctypes.c_int), ("inner_cycles", ctypes.c_int),
                ("nu_coarse", ctypes.c_int), ("learned_levels", ctypes.c_int), ("krylov_m", ctypes.c_int),
                ("fmg_cycles", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("vcycles", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_residual", ctypes.c_double),
                ("conv_factor", ctypes.c_double), ("fell_back", ctypes.c_int), ("t_solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FfmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ffmg status {status}: {msg}")
        self.status = status


_lib = None

EXPORTS = ["ffmg_default_options", "ffmg_strerror", "ffmg_last_error", "mg_setup", "mg_rhs_plane_wave",
           "mg_vcycle", "mg_fmg", "mg_solve", "farfield_map", "mg_apply", "mg_smooth", "mg_residual_norm",
           "mg_num_levels", "mg_level_shape", "mg_destroy", "mg_profile_enable", "mg_profile_read",
           "mg_tune_variants", "mg_tune_get", "mg_tune_set", "mg_tune_farfield", "mg_tune_solve", "mg_solve_batched",
           "farfield_map_batched", "ml_net_create", "ml_net_set_weights", "ml_net_get_weights", "ml_loss_grad",
           "ml_train_step", "ml_net_last_error", "ml_net_destroy", "mg_learned_smooth", "mg_jacobi_factor",
           "mg_gmres_smooth", "mg_solve_begin", "mg_solve_end", "farfield_map_noalloc", "mg_rhs_phase",
           "mg_residual", "mg_profile_durations", "mg_rhs_source", "ion_bound_state", "ion_wavenumbers",
           "ion_test_functions", "ion_amplitudes", "ion_cross_sections"]


def lib():
    """Load libffmg.so (built in-tree by ``build.py``); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950) first")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    L.ffmg_default_options.argtypes = [ctypes.POINTER(Options)]
    L.ffmg_strerror.restype = ctypes.c_char_p
    L.ffmg_strerror.argtypes = [ip]
    L.ffmg_last_error.restype = ctypes.c_char_p
    L.ffmg_last_error.argtypes = [vp]
    L.mg_setup.argtypes = [ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.mg_rhs_plane_wave.argtypes = [vp, vp, vp]
    L.mg_rhs_phase.argtypes = [vp, vp, vp]
    L.mg_residual.argtypes = [vp, vp, vp, vp]
    L.mg_vcycle.argtypes = [vp, vp, vp]
    L.mg_fmg.argtypes = [vp, vp, vp, ip]
    L.mg_solve.argtypes = [vp, vp, vp, dp, ctypes.POINTER(SolveInfo)]
    L.mg_solve_begin.argtypes = [vp, vp, vp, dp]
    L.mg_solve_end.argtypes = [vp, ctypes.POINTER(SolveInfo)]
    L.farfield_map.argtypes = [vp, vp, vp, ip, vp, vp]
    L.farfield_map_noalloc.argtypes = [vp, vp, vp, ip, vp, vp]
    L.mg_apply.argtypes = [vp, vp, vp]
    L.mg_smooth.argtypes = [vp, vp, vp, vp]
    L.mg_residual_norm.argtypes = [vp, vp, vp, ctypes.POINTER(dp)]
    L.mg_num_levels.argtypes = [vp]
    L.mg_num_levels.restype = ip
    L.mg_level_shape.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int64)]
    L.mg_destroy.argtypes = [vp]
    L.mg_destroy.restype = None
    L.mg_profile_enable.argtypes = [vp, ip]
    L.mg_profile_read.argtypes = [vp, ip, ctypes.POINTER(dp), ctypes.POINTER(ctypes.c_int64)]
    L.mg_profile_durations.argtypes = [vp, ip, vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.mg_tune_variants.argtypes = [vp, ip]
    L.mg_tune_get.argtypes = [vp, ip, ctypes.POINTER(ip)]
    L.mg_tune_set.argtypes = [vp, ip, ip]
    L.mg_tune_farfield.argtypes = [vp, vp, vp, ip, vp, ip, ctypes.POINTER(dp), ip, ctypes.POINTER(ip)]
    L.mg_tune_solve.argtypes = [vp, ip, vp, vp, dp, ip, ctypes.POINTER(dp), ip, ctypes.POINTER(ip)]
    L.mg_solve_batched.argtypes = [vp, ip, vp, vp, dp, vp]
    fp = ctypes.POINTER(ctypes.c_float)
    L.ml_net_create.argtypes = [fp, vp, ctypes.POINTER(vp)]
    L.ml_net_set_weights.argtypes = [vp, fp]
    L.ml_net_get_weights.argtypes = [vp, fp]
    L.ml_loss_grad.argtypes = [vp, vp, vp, vp, ip, ip, fp, fp]
    L.ml_train_step.argtypes = [vp, vp, vp, vp, ip, ip, ctypes.c_float, fp]
    L.ml_net_last_error.argtypes = [vp]
    L.ml_net_last_error.restype = ctypes.c_char_p
    L.ml_net_destroy.argtypes = [vp]
    L.ml_net_destroy.restype = None
    L.mg_rhs_source.argtypes = [vp, vp, vp]
    L.ion_bound_state.argtypes = [vp, ip, vp, dp, vp, vp]
    L.ion_wavenumbers.argtypes = [dp, vp, ip, vp, vp, vp, vp]
    L.ion_test_functions.argtypes = [vp, ip, vp, ip, vp, vp]
    L.ion_amplitudes.argtypes = [vp, vp, vp, vp, ip, vp, vp, vp, vp]
    L.ion_cross_sections.argtypes = [ip, vp, ip, vp, vp, vp, vp]
    L.mg_learned_smooth.argtypes = [vp, vp, vp]
    L.mg_learned_smooth.restype = ip
    L.mg_jacobi_factor.argtypes = [vp]
    L.mg_gmres_smooth.argtypes = [vp, vp, vp]
    L.mg_gmres_smooth.restype = ip
    L.mg_jacobi_factor.restype = ctypes.c_double
    L.farfield_map_batched.argtypes = [vp, ip, vp, vp, ip, vp, vp]
    for name in ("mg_setup", "mg_rhs_plane_wave", "mg_vcycle", "mg_fmg", "mg_solve", "farfield_map", "mg_apply",
                 "mg_smooth", "mg_residual_norm", "mg_level_shape", "mg_profile_enable", "mg_profile_read",
                 "mg_tune_variants", "mg_tune_get", "mg_tune_set", "mg_tune_farfield", "mg_tune_solve",
                 "mg_solve_batched", "farfield_map_batched", "ml_net_create", "ml_net_set_weights", "ml_net_get_weights",
                 "ml_loss_grad", "ml_train_step"):
        getattr(L, name).restype = ip
    _lib = L
    return L


def default_options(**kw) -> Options:
    """ffmg_default_options with overrides.  smoother_weights may be a list of
    the three complex weight arrays or a flat float32 array; it is kept alive
    with the options object."""
    o = Options()
    lib().ffmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "smoother_weights" and v is not None and not isinstance(v, int):
            w = net_flatten(v) if isinstance(v, (list, tuple)) else np.ascontiguousarray(v, dtype=np.float32)
            o._weights = w
            v = w.ctypes.data
        setattr(o, k, v)
    return o


def _torch():
    import torch
    return torch


def _dev_ptr(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.complex128:
        raise TypeError(f"{name} must be complex128 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """Owns one ``ffmg_handle``.  Arrays are complex128 device tensors whose
    memory layout is x fastest (numpy/torch shape (ny, nx) or (nz, ny, nx))."""

    def __init__(self, ptr, shape, options=None):
        self._p = ptr
        self.shape = shape
        # the options the handle was set up with (plain values, no pointers)
        self.options = {} if options is None else {
            k: getattr(options, k) for k, _ in Options._fields_ if k not in ("stream", "smoother_weights")}

    def _check(self, st, what):
        if st != FFMG_OK:
            msg = lib().ffmg_last_error(self._p).decode()
            raise FfmgError(st, f"{what}: {msg}")

    @property
    def ptr(self):
        return self._p

    def num_levels(self):
        return lib().mg_num_levels(self._p)

    def level_shape(self, level):
        m = (ctypes.c_int64 * 3)()
        self._check(lib().mg_level_shape(self._p, level, m), "mg_level_shape")
        return tuple(m)

    def destroy(self):
        if self._p:
            lib().mg_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def mg_setup(dim, n, lo, hi, gamma, coef, kind=HELMHOLTZ, k0=1.0, energy=0.0, options: Optional[Options] = None,
             stream=None) -> Handle:
    """Build the hierarchy for a problem; coef is the contrast k^2 - k0^2
    (Helmholtz) or V (Schroedinger) at every interior node."""
    torch = _torch()
    p = Problem()
    p.dim = dim
    nn = list(n) if isinstance(n, (list, tuple)) else [n] * dim
    ll = list(lo) if isinstance(lo, (list, tuple)) else [lo] * dim
    hh = list(hi) if isinstance(hi, (list, tuple)) else [hi] * dim
    for k in range(3):
        p.n[k] = int(nn[k]) if k < dim else 1
        p.lo[k] = float(ll[k]) if k < dim else 0.0
        p.hi[k] = float(hh[k]) if k < dim else 1.0
    p.gamma, p.kind, p.k0, p.energy = float(gamma), int(kind), float(k0), float(energy)
    p.coef = _dev_ptr(coef, "coef")
    o = options if options is not None else default_options()
    if stream is None:
        stream = torch.cuda.current_stream()
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    h = ctypes.c_void_p()
    st = lib().mg_setup(ctypes.byref(p), ctypes.byref(o), ctypes.byref(h))
    if st != FFMG_OK:
        raise FfmgError(st, "mg_setup: " + lib().ffmg_strerror(st).decode())
    shape = tuple(int(v) - 1 for v in nn[:dim][::-1])
    return Handle(h, shape, o)


def _eta3(eta):
    e = (ctypes.c_double * 3)()
    for k, v in enumerate(np.asarray(eta, dtype=np.float64).ravel()[:3]):
        e[k] = v
    return e


def _opt_dev_ptr(t, name):
    return ctypes.c_void_p(None) if t is None else _dev_ptr(t, name)


def mg_rhs_plane_wave(h: Handle, eta, b):
    """b = q exp(i k0 eta.z) (Sec. 2.1); also records eta as the handle's
    plane wave.  b = None records it only: mg_solve(h, None, u) then solves
    for that right-hand side without storing it."""
    h._check(lib().mg_rhs_plane_wave(h.ptr, _eta3(eta), _opt_dev_ptr(b, "b")), "mg_rhs_plane_wave")
    return b


def mg_rhs_phase(h: Handle, eta, b):
    """b = q exp(i k0 cos(gamma) eta.x) (the bounded stress right-hand side)."""
    h._check(lib().mg_rhs_phase(h.ptr, _eta3(eta), _dev_ptr(b, "b")), "mg_rhs_phase")
    return b


def mg_rhs_source(h: Handle, src, b):
    """b = 2 src (Schroedinger form) or src (Helmholtz)."""
    h._check(lib().mg_rhs_source(h.ptr, _dev_ptr(src, "src"), _dev_ptr(b, "b")), "mg_rhs_source")
    return b


def _host_c128(a, n):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.size != n:
        raise ValueError(f"expected {n} complex values")
    return a


def ion_bound_state(h: Handle, axis: int, v, shift: float = -1.0, phi=None):
    """(lambda, phi): eq. boundstate on one axis (v: device potential at the
    axis nodes); phi normalised by sum phi^2 h~ = 1."""
    torch = _torch()
    if phi is None:
        phi = torch.empty(v.numel(), dtype=torch.complex128, device=v.device)
    lam = np.zeros(2)
    h._check(lib().ion_bound_state(h.ptr, int(axis), _dev_ptr(v, "v"), float(shift), lam.ctypes.data_as(ctypes.c_void_p),
                                   _dev_ptr(phi, "phi")), "ion_bound_state")
    return complex(lam[0], lam[1]), phi


def ion_wavenumbers(E: float, lam: complex, M: int):
    """(k_n or None, k1[M], k2[M], w[M]) of the single and double channels."""
    lm = np.array([complex(lam).real, complex(lam).imag])
    kn = ctypes.c_double(0.0)
    k1, k2, w = np.zeros(M), np.zeros(M), np.zeros(M)
    st = lib().ion_wavenumbers(float(E), lm.ctypes.data_as(ctypes.c_void_p), int(M), ctypes.byref(kn), k1.ctypes.data_as(ctypes.c_void_p),
                               k2.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p))
    if st:
        raise FfmgError(st, "ion_wavenumbers: bad argument")
    n = M if E > 0 else 0
    return (kn.value if kn.value > 0 else None), k1[:n], k2[:n], w[:n]


def ion_test_functions(h: Handle, axis: int, v, ks, out=None):
    """eq. testfunction: (M, m) device table of regular solutions with free
    amplitude 1/sqrt(k)."""
    torch = _torch()
    ks = np.ascontiguousarray(ks, dtype=np.float64).ravel()
    if out is None:
        out = torch.empty((ks.size, v.numel()), dtype=torch.complex128, device=v.device)
    h._check(lib().ion_test_functions(h.ptr, int(axis), _dev_ptr(v, "v"), int(ks.size), ks.ctypes.data_as(ctypes.c_void_p),
                                      _dev_ptr(out, "out")), "ion_test_functions")
    return out


def ion_amplitudes(h: Handle, src, v12, u, tx, ty):
    """(amp[M], opt): eq. single-ionization / eq. double-ionization for the
    rows of tx, ty, and the optical-theorem product <phi, u>."""
    M = int(tx.shape[0])
    if int(ty.shape[0]) != M:
        raise ValueError("tx and ty need the same number of rows")
    amp = np.zeros(M, dtype=np.complex128)
    opt = np.zeros(2)
    h._check(lib().ion_amplitudes(h.ptr, _dev_ptr(src, "src"), _dev_ptr(v12, "v12"), _dev_ptr(u, "u"), M,
                                  _dev_ptr(tx, "tx"), _dev_ptr(ty, "ty"), amp.ctypes.data_as(ctypes.c_void_p),
                                  opt.ctypes.data_as(ctypes.c_void_p)), "ion_amplitudes")
    return amp, complex(opt[0], opt[1])


def ion_cross_sections(s0, f, w, opt):
    """(single, double, total) cross sections from the amplitudes."""
    f = _host_c128(f, len(w))
    w = np.ascontiguousarray(w, dtype=np.float64)
    s = np.array([complex(s0).real, complex(s0).imag]) if s0 is not None else np.zeros(2)
    o = np.array([complex(opt).real, complex(opt).imag])
    sig = np.zeros(3)
    st = lib().ion_cross_sections(int(s0 is not None), s.ctypes.data_as(ctypes.c_void_p), int(len(w)), f.ctypes.data_as(ctypes.c_void_p),
                                  w.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p), sig.ctypes.data_as(ctypes.c_void_p))
    if st:
        raise FfmgError(st, "ion_cross_sections: bad argument")
    return float(sig[0]), float(sig[1]), float(sig[2])


def ion_observables(h: Handle, src, v12, u, v1x, v1y, E: float, M: int, lam: complex, phi0):
    """All cross sections at energy E from the solution u: one batch of
    test functions per axis ([k_n] + k1 on x, k2 on y), one contraction of
    M + 1 amplitudes (the bound state phi0 of the y axis pairs with k_n),
    and the cross sections.  Returns a dict."""
    torch = _torch()
    kn, k1, k2, w = ion_wavenumbers(E, lam, M)
    kx = ([kn] if kn else []) + list(k1)
    out = dict(kn=kn, s0=None, f=np.zeros(0, dtype=np.complex128), k1=k1, k2=k2, w=w)
    if kx:
        tx = ion_test_functions(h, 0, v1x, kx)
        rows = []
        if kn:
            rows.append(phi0.reshape(1, -1))
        if len(k2):
            rows.append(ion_test_functions(h, 1, v1y, k2))
        ty = torch.cat(rows, 0) if len(rows) > 1 else rows[0].contiguous()
        amp, opt = ion_amplitudes(h, src, v12, u, tx, ty)
        if kn:
            out["s0"], out["f"] = amp[0], amp[1:]
        else:
            out["f"] = amp
    else:
        z = torch.zeros((1, v1x.numel()), dtype=torch.complex128, device=v1x.device)
        _, opt = ion_amplitudes(h, src, v12, u, z, torch.zeros((1, v1y.numel()), dtype=torch.complex128,
                                                              device=v1y.device))
    out["opt"] = opt
    out["single"], out["double"], out["total"] = ion_cross_sections(out["s0"], out["f"], w, opt)
    return out


def mg_residual(h: Handle, b, u, r):
    """r = b - A u (FP64)."""
    h._check(lib().mg_residual(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u"), _dev_ptr(r, "r")), "mg_residual")
    return r


def mg_vcycle(h: Handle, b, u):
    h._check(lib().mg_vcycle(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u")), "mg_vcycle")
    return u


def mg_fmg(h: Handle, b, u, k):
    """u <- the full multigrid start with k V-cycles per coarse level."""
    h._check(lib().mg_fmg(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u"), int(k)), "mg_fmg")
    return u


def mg_solve(h: Handle, b, u, tol=1e-10, raise_on_noconv=True):
    info = SolveInfo()
    st = lib().mg_solve(h.ptr, _opt_dev_ptr(b, "b"), _dev_ptr(u, "u"), float(tol), ctypes.byref(info))
    if st != FFMG_OK and (st != FFMG_ENOCONV or raise_on_noconv):
        h._check(st, "mg_solve")
    return info


def mg_solve_begin(h: Handle, b, u, tol=1e-10):
    """Queue a solve on the handle's stream and return without waiting;
    b and u must stay untouched until mg_solve_end (b = None: the handle's
    plane wave, as mg_solve)."""
    h._check(lib().mg_solve_begin(h.ptr, _opt_dev_ptr(b, "b"), _dev_ptr(u, "u"), float(tol)), "mg_solve_begin")


def mg_solve_end(h: Handle, raise_on_noconv=True):
    """Finish the solve begun by mg_solve_begin; returns its SolveInfo."""
    info = SolveInfo()
    st = lib().mg_solve_end(h.ptr, ctypes.byref(info))
    if st != FFMG_OK and (st != FFMG_ENOCONV or raise_on_noconv):
        h._check(st, "mg_solve_end")
    return info


def farfield_map(h: Handle, eta, u, dirs, out=None):
    """F for each row of dirs (unit vectors); out: complex128 device tensor
    or None (returns a host numpy array)."""
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64))
    M = d.shape[0]
    up = None if u is None else _dev_ptr(u, "u")
    if out is None:
        F = np.empty(M, dtype=np.complex128)
        fp = ctypes.c_void_p(F.ctypes.data)
    else:
        F = out
        fp = _dev_ptr(out, "F")
    h._check(lib().farfield_map(h.ptr, _eta3(eta), up, M, ctypes.c_void_p(d.ctypes.data), fp), "farfield_map")
    return F


NOALLOC_SCRATCH_BYTES = 64 << 20   # FFMG_NOALLOC_SCRATCH_BYTES
NOALLOC_MAX_DIRS = 8192            # FFMG_NOALLOC_MAX_DIRS


def farfield_map_noalloc(h: Handle, eta, u, dirs, out=None):
    """farfield_map (FP64 contraction) with every work buffer in the
    library's static scratch array: no device allocation.  out: complex128
    device tensor or None (returns a host numpy array)."""
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64))
    M = d.shape[0]
    up = None if u is None else _dev_ptr(u, "u")
    if out is None:
        F = np.empty(M, dtype=np.complex128)
        fp = ctypes.c_void_p(F.ctypes.data)
    else:
        F = out
        fp = _dev_ptr(out, "F")
    h._check(lib().farfield_map_noalloc(h.ptr, _eta3(eta), up, M, ctypes.c_void_p(d.ctypes.data), fp),
             "farfield_map_noalloc")
    return F


TUNE_FF_GEMM = 0
TUNE_TAIL = 1
TUNE_SMOOTH = 2
TUNE_PRE = 3
TUNE_SMOOTH_COARSE = 4
TUNE_SWEEP3D = 5
TUNE_BATCH = 6


def _etas(etas):
    E = np.zeros((len(etas), 3), dtype=np.float64)
    for i, e_ in enumerate(etas):
        v = np.asarray(e_, dtype=np.float64).ravel()[:3]
        E[i, :len(v)] = v
    return E


def mg_solve_batched(hs, etas, us, tol=1e-10, raise_on_noconv=True):
    """Solve the plane-wave problems (hs[i], etas[i]) together; us[i] are
    device tensors of each handle's interior shape (written).  Returns the
    list of SolveInfo."""
    n = len(hs)
    if n == 0 or len(us) != n or len(etas) != n:
        raise ValueError("hs, etas and us must have the same nonzero length")
    H = (ctypes.c_void_p * n)(*[h.ptr for h in hs])
    U = (ctypes.c_void_p * n)(*[_dev_ptr(u, "u").value for u in us])
    E = _etas(etas)
    infos = (SolveInfo * n)()
    st = lib().mg_solve_batched(H, n, ctypes.c_void_p(E.ctypes.data), U, float(tol), infos)
    if st != FFMG_OK and not (st == FFMG_ENOCONV and not raise_on_noconv):
        hs[0]._check(st, "mg_solve_batched")
    return list(infos)


def farfield_map_batched(hs, etas, us, dirs, out=None):
    """Far-field maps of the instances (hs[i], etas[i], us[i]) at the same
    directions: a (len(hs), len(dirs)) complex array (host numpy, or `out`)."""
    n = len(hs)
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64))
    M = d.shape[0]
    H = (ctypes.c_void_p * n)(*[h.ptr for h in hs])
    U = None if us is None else (ctypes.c_void_p * n)(*[_dev_ptr(u, "u").value for u in us])
    E = _etas(etas)
    if out is None:
        F = np.empty((n, M), dtype=np.complex128)
        fp = ctypes.c_void_p(F.ctypes.data)
    else:
        F = out
        fp = _dev_ptr(out, "F")
    hs[0]._check(lib().farfield_map_batched(H, n, ctypes.c_void_p(E.ctypes.data), U, M,
                                            ctypes.c_void_p(d.ctypes.data), fp), "farfield_map_batched")
    return F


def mg_tune_variants(h: Handle, tunable=TUNE_FF_GEMM) -> int:
    return int(lib().mg_tune_variants(h.ptr, int(tunable)))


def mg_tune_get(h: Handle, tunable=TUNE_FF_GEMM) -> int:
    v = ctypes.c_int()
    h._check(lib().mg_tune_get(h.ptr, int(tunable), ctypes.byref(v)), "mg_tune_get")
    return v.value


def mg_tune_set(h: Handle, variant, tunable=TUNE_FF_GEMM):
    h._check(lib().mg_tune_set(h.ptr, int(tunable), int(variant)), "mg_tune_set")


def mg_tune_farfield(h: Handle, eta, u, dirs, reps=5):
    """Time every variant of the far-field contraction on this handle's
    shapes; selects the fastest.  Returns (best, [ms per variant])."""
    d = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64))
    nv = max(mg_tune_variants(h, TUNE_FF_GEMM), 1)
    times = (ctypes.c_double * nv)()
    best = ctypes.c_int()
    up = None if u is None else _dev_ptr(u, "u")
    h._check(lib().mg_tune_farfield(h.ptr, _eta3(eta), up, d.shape[0], ctypes.c_void_p(d.ctypes.data), int(reps),
                                    times, nv, ctypes.byref(best)), "mg_tune_farfield")
    return best.value, list(times)


def mg_tune_solve(h: Handle, b, u, tol=1e-10, reps=3, tunable=TUNE_TAIL):
    """Time `reps` solves per variant of `tunable` (TUNE_TAIL, TUNE_SMOOTH, TUNE_PRE, TUNE_SMOOTH_COARSE;
    u is overwritten); selects the fastest.  Returns (best, [ms per variant])."""
    nv = max(mg_tune_variants(h, tunable), 1)
    times = (ctypes.c_double * nv)()
    best = ctypes.c_int()
    h._check(lib().mg_tune_solve(h.ptr, int(tunable), _dev_ptr(b, "b"), _dev_ptr(u, "u"), float(tol), int(reps),
                                 times, nv, ctypes.byref(best)), "mg_tune_solve")
    return best.value, list(times)


def mg_apply(h: Handle, u, Au):
    h._check(lib().mg_apply(h.ptr, _dev_ptr(u, "u"), _dev_ptr(Au, "Au")), "mg_apply")
    return Au


def mg_learned_smooth(h: Handle, b, u):
    """One learned smoothing step on the finest level, in place on u."""
    h._check(lib().mg_learned_smooth(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u")), "mg_learned_smooth")
    return u


def mg_gmres_smooth(h: Handle, b, u):
    """One GMRES(m) smoothing step on the finest level, in place on u."""
    h._check(lib().mg_gmres_smooth(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u")), "mg_gmres_smooth")
    return u


def mg_jacobi_factor(h: Handle) -> float:
    return float(lib().mg_jacobi_factor(h.ptr))


def mg_smooth(h: Handle, b, u, u_out):
    h._check(lib().mg_smooth(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u"), _dev_ptr(u_out, "u_out")), "mg_smooth")
    return u_out


def mg_residual_norm(h: Handle, b, u):
    r = ctypes.c_double()
    h._check(lib().mg_residual_norm(h.ptr, _dev_ptr(b, "b"), _dev_ptr(u, "u"), ctypes.byref(r)),
             "mg_residual_norm")
    return r.value


def mg_destroy(h: Handle):
    h.destroy()


KERNEL_SWEEP, KERNEL_FARFIELD = 0, 1


PROF_PRE, PROF_FF, PROF_POST, PROF_REFINE, PROF_FFGEMM, PROF_NET, PROF_RR, PROF_SRR, PROF_SRR0 = range(9)


def mg_profile_durations(h: Handle, kernel, cap=1 << 16):
    """Per-launch durations (ms, numpy array) recorded for kernel PROF_*
    since the last read."""
    buf = np.empty(cap, dtype=np.float64)
    n = ctypes.c_int64()
    h._check(lib().mg_profile_durations(h.ptr, int(kernel), ctypes.c_void_p(buf.ctypes.data), int(cap),
                                        ctypes.byref(n)), "mg_profile_durations")
    return buf[: min(n.value, cap)].copy()


def mg_profile_enable(h: Handle, mask=0x1FF):
    """Time kernel k when bit k of mask is set (0 disables)."""
    h._check(lib().mg_profile_enable(h.ptr, int(mask)), "mg_profile_enable")


def mg_profile_read(h: Handle, kernel):
    """(total_ms, launches) recorded for kernel PROF_* since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    h._check(lib().mg_profile_read(h.ptr, int(kernel), ctypes.byref(ms), ctypes.byref(n)), "mg_profile_read")
    return ms.value, n.value


def setup_workload(w, device="cuda", options: Optional[Options] = None):
    """mg_setup for a workload of ``workloads.py``; returns (handle, coef)."""
    torch = _torch()
    coef = torch.from_numpy(np.ascontiguousarray(w.coef)).to(device)
    lo, hi = w.box()
    h = mg_setup(w.dim, [w.n] * w.dim, lo, hi, w.gamma, coef, kind=w.kind, k0=w.k0, energy=w.energy,
                 options=options)
    return h, coef


# ---------------------------------------------------------------------------
# Learned smoother network
NET_WEIGHTS = 2736
NET_SHAPES = ((9, 16, 2), (9, 16, 16), (9, 1, 16))


def net_flatten(Ws) -> np.ndarray:
    """[W1, W2, W3] complex arrays (tap, out, in) -> interleaved float32."""
    z = np.concatenate([np.asarray(W, dtype=np.complex128).ravel() for W in Ws])
    if z.size != NET_WEIGHTS:
        raise ValueError(f"expected {NET_WEIGHTS} complex weights, got {z.size}")
    out = np.empty(2 * NET_WEIGHTS, dtype=np.float32)
    out[0::2], out[1::2] = z.real, z.imag
    return out


def net_unflatten(w) -> list:
    w = np.asarray(w, dtype=np.float32)
    z = w[0::2].astype(np.float64) + 1j * w[1::2].astype(np.float64)
    out, k = [], 0
    for s in NET_SHAPES:
        n = int(np.prod(s))
        out.append(z[k:k + n].reshape(s))
        k += n
    return out


class Net:
    """The learned smoother's network: FP32 master weights, Adam state and
    training buffers on the device (ml_net_*)."""

    def __init__(self, Ws, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        w = net_flatten(Ws)
        p = ctypes.c_void_p()
        st = lib().ml_net_create(w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.c_void_p(stream),
                                 ctypes.byref(p))
        if st != FFMG_OK:
            raise FfmgError(st, "ml_net_create failed")
        self._p = p

    def _check(self, st, what):
        if st != FFMG_OK:
            raise FfmgError(st, f"{what}: {lib().ml_net_last_error(self._p).decode()}")

    @property
    def ptr(self):
        return self._p

    def weights(self) -> list:
        w = np.empty(2 * NET_WEIGHTS, dtype=np.float32)
        self._check(lib().ml_net_get_weights(self._p, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "ml_net_get_weights")
        return net_unflatten(w)

    def set_weights(self, Ws):
        w = net_flatten(Ws)
        self._check(lib().ml_net_set_weights(self._p, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
                    "ml_net_set_weights")

    @staticmethod
    def _patches(t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous complex64 device tensor")
        if t.dim() != 3 or t.shape[1] != 32 or t.shape[2] != 32:
            raise ValueError(f"{name} must have shape (count, 32, 32)")
        return ctypes.c_void_p(t.data_ptr())

    def loss_grad(self, rt, kt, et, border=4):
        loss = ctypes.c_float()
        g = np.empty(2 * NET_WEIGHTS, dtype=np.float32)
        self._check(lib().ml_loss_grad(self._p, self._patches(rt, "rt"), self._patches(kt, "kt"),
                                       self._patches(et, "et"), rt.shape[0], int(border), ctypes.byref(loss),
                                       g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), "ml_loss_grad")
        return loss.value, net_unflatten(g)

    def train_step(self, rt, kt, et, lr, border=4, want_loss=False):
        loss = ctypes.c_float()
        self._check(lib().ml_train_step(self._p, self._patches(rt, "rt"), self._patches(kt, "kt"),
                                        self._patches(et, "et"), rt.shape[0], int(border), ctypes.c_float(lr),
                                        ctypes.byref(loss) if want_loss else None), "ml_train_step")
        return loss.value if want_loss else None

    def destroy(self):
        if self._p:
            lib().ml_net_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
