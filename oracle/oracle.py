"""FP64 CPU oracle for the complex-contour multigrid far-field method
(Cools, Reps & Vanroose, arXiv 1211.4461).

TEST INFRASTRUCTURE ONLY: the reference that the HIP library is checked
against.  Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it.  It shares no code with the GPU library; the
arithmetic lives in ``ffmg_oracle.c`` (plain C, double precision, OpenMP over
the outermost axis), this module only marshals numpy arrays.

Every function states the passage of the paper it follows; see the C source
for the conventions (grid, contour, operator, right-hand side, far field).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ffmg_oracle.c")
_LIB = os.path.join(_HERE, "libffmg_oracle.so")

OK = 0
ENOCONV = 4


def build(force: bool = True, native: bool = False, path: str = None) -> str:
    """Compile the oracle shared library: -O3, OpenMP, IEEE arithmetic with
    no contraction into fused multiply-adds.  The library that the tests load
    is portable; native=True builds one for the host's own instruction set
    (-march=native) at `path`, for timing the oracle on the machine it runs
    on (a native build is not carried to another machine)."""
    out = path or _LIB
    if force or not os.path.exists(out):
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off"]
        if native:
            cmd.append("-march=native")
        cmd += ["-o", out + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


_lib = None
_lib_path = None


def load(path: str):
    """Use the oracle library at `path` (e.g. a native build) from now on."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def num_threads() -> int:
    """Threads of the oracle's OpenMP loops."""
    return int(lib().or_num_threads())


def lib():
    global _lib
    if _lib is None:
        p = _lib_path or _LIB
        if not os.path.exists(p):
            build(path=p)
        L = ctypes.CDLL(p)
        vp, ip, lp, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_long, ctypes.c_double
        L.or_mg_create.restype = vp
        L.or_mg_create.argtypes = [ip, vp, vp, vp, dp, vp, ip, ip, dp, lp]
        L.or_mg_destroy.argtypes = [vp]
        L.or_mg_nlev.argtypes = [vp]
        L.or_mg_nlev.restype = ip
        L.or_mg_coarse_n.argtypes = [vp]
        L.or_mg_coarse_n.restype = lp
        L.or_mg_kappa.argtypes = [vp, ip, vp]
        L.or_mg_vcycle.argtypes = [vp, vp, vp]
        L.or_mg_fmg.argtypes = [vp, vp, vp, ip]
        L.or_mg_set_smoother.argtypes = [vp, ip, ip]
        L.or_gmres.argtypes = [ip, vp, vp, dp, vp, vp, vp, ip]
        L.or_rbgs.argtypes = [ip, vp, vp, dp, vp, vp, vp]
        L.or_mg_solve.argtypes = [vp, vp, vp, dp, ip, vp, vp]
        L.or_mg_solve.restype = ip
        L.or_apply.argtypes = [ip, vp, vp, dp, vp, vp, vp]
        L.or_residual.argtypes = [ip, vp, vp, dp, vp, vp, vp, vp]
        L.or_jacobi.argtypes = [ip, vp, vp, dp, vp, vp, vp, dp, vp]
        L.or_restrict.argtypes = [ip, vp, vp, vp]
        L.or_prolong_add.argtypes = [ip, vp, vp, vp]
        L.or_inject.argtypes = [ip, vp, vp, vp]
        L.or_assemble_dense.argtypes = [ip, vp, vp, dp, vp, vp]
        L.or_lu_factor.argtypes = [lp, vp, vp]
        L.or_lu_factor.restype = ip
        L.or_lu_solve.argtypes = [lp, vp, vp, vp]
        L.or_rhs_plane_wave.argtypes = [ip, vp, vp, vp, dp, dp, vp, vp, vp]
        L.or_rhs_phase.argtypes = [ip, vp, vp, vp, dp, dp, vp, vp, vp]
        L.or_ff_integrand.argtypes = [ip, vp, vp, vp, dp, dp, vp, vp, vp, vp]
        L.or_ff_dense.argtypes = [ip, vp, vp, vp, dp, dp, vp, lp, vp, vp, vp]
        L.or_ff_separable.argtypes = [ip, vp, vp, vp, dp, dp, vp, lp, vp, vp]
        L.or_num_threads.restype = ip
        _lib = L
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def _m3(m):
    out = np.ones(3, dtype=np.int64)
    out[: len(m)] = m
    return out


def _d3(v, fill=0.0):
    out = np.full(3, fill, dtype=np.float64)
    out[: len(v)] = v
    return out


class Grid:
    """Vertex-centred grid: n intervals per axis on [lo, hi], interior nodes
    x_i = lo + i h, i = 1..n-1 (Sec. 4, the n^d mesh on the box)."""

    def __init__(self, dim, n, lo, hi):
        self.dim = int(dim)
        self.n = np.array(n, dtype=np.int64).reshape(-1)
        if self.n.size == 1:
            self.n = np.repeat(self.n, self.dim)
        self.lo = np.array(lo, dtype=np.float64).reshape(-1)
        self.hi = np.array(hi, dtype=np.float64).reshape(-1)
        if self.lo.size == 1:
            self.lo = np.repeat(self.lo, self.dim)
        if self.hi.size == 1:
            self.hi = np.repeat(self.hi, self.dim)
        self.m = self.n - 1
        self.h = (self.hi - self.lo) / self.n
        self.N = int(np.prod(self.m))

    @property
    def shape(self):
        """numpy shape of an x-fastest array: (z, y, x) / (y, x)."""
        return tuple(int(v) for v in self.m[::-1])


# ---------------------------------------------------------------- operators

def apply_A(g: Grid, gamma, kappa):
    """Return a function u -> A u for the contour operator (eq. csg)."""
    kap, kp = _c(kappa.ravel(), np.complex128)
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)

    def f(u):
        uu, up = _c(u.ravel(), np.complex128)
        out = np.empty_like(uu)
        lib().or_apply(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, up, out.ctypes.data)
        return out.reshape(np.shape(u))
    return f


def residual(g: Grid, gamma, kappa, b, u):
    """r = b - A u."""
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)
    kap, kp = _c(kappa.ravel(), np.complex128)
    bb, bp = _c(b.ravel(), np.complex128)
    uu, up = _c(u.ravel(), np.complex128)
    r = np.empty_like(uu)
    lib().or_residual(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, bp, up, r.ctypes.data)
    return r.reshape(np.shape(u))


def jacobi(g: Grid, gamma, kappa, b, u, omega):
    """One omega-Jacobi sweep u' = u + omega (b - A u)/D."""
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)
    kap, kp = _c(kappa.ravel(), np.complex128)
    bb, bp = _c(b.ravel(), np.complex128)
    uu, up = _c(u.ravel(), np.complex128)
    out = np.empty_like(uu)
    lib().or_jacobi(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, bp, up, omega, out.ctypes.data)
    return out.reshape(np.shape(u))


def gmres_step(g: Grid, gamma, kappa, b, u, m):
    """One GMRES(m) smoothing step from u (Sec. 3.3): the least-residual
    update in the Krylov space of the residual (returns a copy)."""
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)
    kap, kp = _c(kappa.ravel(), np.complex128)
    bb, bp = _c(b.ravel(), np.complex128)
    out = np.array(u, dtype=np.complex128, copy=True).ravel()
    lib().or_gmres(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, bp, out.ctypes.data, int(m))
    return out.reshape(np.shape(u))


def rbgs_sweep(g: Grid, gamma, kappa, b, u):
    """One red-black Gauss-Seidel sweep (red: ix + iy + iz even), a copy."""
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)
    kap, kp = _c(kappa.ravel(), np.complex128)
    bb, bp = _c(b.ravel(), np.complex128)
    out = np.array(u, dtype=np.complex128, copy=True).ravel()
    lib().or_rbgs(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, bp, out.ctypes.data)
    return out.reshape(np.shape(u))


def restrict(dim, mf, rf):
    """Full-weighting restriction from a fine grid with interior counts mf."""
    mf = np.asarray(mf, dtype=np.int64).reshape(-1)
    mc = (mf - 1) // 2
    r, rp = _c(rf.ravel(), np.complex128)
    out = np.empty(int(np.prod(mc)), dtype=np.complex128)
    lib().or_restrict(dim, _m3(mf).ctypes.data, rp, out.ctypes.data)
    return out.reshape(tuple(int(v) for v in mc[::-1]))


def prolong_add(dim, mc, ec, uf):
    """uf + P ec with bilinear / trilinear interpolation (returns a copy)."""
    mc = np.asarray(mc, dtype=np.int64).reshape(-1)
    e, ep = _c(ec.ravel(), np.complex128)
    out = np.array(uf, dtype=np.complex128, copy=True).ravel()
    lib().or_prolong_add(dim, _m3(mc).ctypes.data, ep, out.ctypes.data)
    return out.reshape(np.shape(uf))


def assemble_dense(g: Grid, gamma, kappa):
    """Dense matrix of A (small grids only)."""
    m3, h3 = _m3(g.m), _d3(g.h, 1.0)
    kap, kp = _c(kappa.ravel(), np.complex128)
    A = np.empty((g.N, g.N), dtype=np.complex128)
    lib().or_assemble_dense(g.dim, m3.ctypes.data, h3.ctypes.data, gamma, kp, A.ctypes.data)
    return A


def lu_solve_dense(A, b):
    """Solve with the oracle's own LU with partial pivoting."""
    N = A.shape[0]
    LU = np.array(A, dtype=np.complex128, copy=True)
    piv = np.zeros(N, dtype=np.int64)
    rc = lib().or_lu_factor(N, LU.ctypes.data, piv.ctypes.data)
    if rc != 0:
        raise np.linalg.LinAlgError("zero pivot")
    x = np.array(b, dtype=np.complex128, copy=True).ravel()
    lib().or_lu_solve(N, LU.ctypes.data, piv.ctypes.data, x.ctypes.data)
    return x


# ---------------------------------------------------------------- multigrid

class Multigrid:
    """V(nu1, nu2) multigrid with omega-Jacobi (or GMRES(m) / red-black
    Gauss-Seidel, Sec. 3.3) smoothing on the contour grid (Sec. 4), coarsest
    grid with 7^d unknowns solved by dense LU."""

    def __init__(self, g: Grid, gamma, kappa, nu1=2, nu2=2, omega=0.8, coarsest_n=8, smoother="jacobi",
                 krylov_m=3):
        self.g = g
        self.gamma = float(gamma)
        self._kappa = np.ascontiguousarray(kappa.ravel(), dtype=np.complex128)
        n3 = _m3(g.n)
        lo3, hi3 = _d3(g.lo), _d3(g.hi, 1.0)
        self._h = lib().or_mg_create(g.dim, n3.ctypes.data, lo3.ctypes.data, hi3.ctypes.data,
                                     self.gamma, self._kappa.ctypes.data, int(nu1), int(nu2),
                                     float(omega), int(coarsest_n))
        self.nlev = lib().or_mg_nlev(self._h)
        if smoother == "gmres":
            lib().or_mg_set_smoother(self._h, 1, int(krylov_m))
        elif smoother == "rbgs":
            lib().or_mg_set_smoother(self._h, 2, 0)
        elif smoother != "jacobi":
            raise ValueError(f"unknown smoother {smoother}")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.or_mg_destroy(h)
            self._h = None

    def kappa_level(self, l):
        n = self.g.n // (2 ** l)
        N = int(np.prod(n - 1))
        out = np.empty(N, dtype=np.complex128)
        lib().or_mg_kappa(self._h, int(l), out.ctypes.data)
        return out.reshape(tuple(int(v) for v in (n - 1)[::-1]))

    def vcycle(self, b, u):
        bb, bp = _c(b.ravel(), np.complex128)
        uu = np.array(u, dtype=np.complex128, copy=True).ravel()
        lib().or_mg_vcycle(self._h, bp, uu.ctypes.data)
        return uu.reshape(np.shape(u))

    def fmg(self, b, k):
        """Full multigrid initial guess (Sec. 4, Tables 3-4: nested
        iteration; Sec. 5.7: the F(k) cycle): coarse right-hand sides by
        injection, exact coarsest solve, k V-cycles on each level between,
        interpolated to the finest."""
        bb, bp = _c(b.ravel(), np.complex128)
        u = np.empty_like(bb)
        lib().or_mg_fmg(self._h, bp, u.ctypes.data, int(k))
        return u.reshape(np.shape(b))

    def solve(self, b, u0=None, tol=1e-10, max_cycles=200):
        """Returns (u, status, cycles, residual history)."""
        bb, bp = _c(b.ravel(), np.complex128)
        u = np.zeros_like(bb) if u0 is None else np.array(u0, dtype=np.complex128, copy=True).ravel()
        hist = np.zeros(max_cycles + 1, dtype=np.float64)
        cyc = ctypes.c_int(0)
        st = lib().or_mg_solve(self._h, bp, u.ctypes.data, float(tol), int(max_cycles),
                               hist.ctypes.data, ctypes.byref(cyc))
        k = cyc.value
        return u.reshape(np.shape(b)), st, k, hist[: k + 1].copy()


# ---------------------------------------------------------------- RHS / far field

def problem(kind, k0, energy, coef):
    """(kappa, q, k0) of a workload: Helmholtz coef = k0^2 chi(z) gives
    kappa = k0^2 + coef, q = coef (Sec. 2.1); Schroedinger coef = V(z) gives
    kappa = 2(E - V), k0 = sqrt(2E), q = kappa - k0^2 = -2V (Sec. 5)."""
    coef = np.asarray(coef, dtype=np.complex128)
    if kind == 0:
        return k0 * k0 + coef, coef, float(k0)
    return 2.0 * (energy - coef), -2.0 * coef, float(np.sqrt(2.0 * energy))


def rhs_plane_wave(g: Grid, gamma, k0, q, eta):
    """b_j = q_j exp(i k0 eta.z_j) on the contour, q = k^2 - k0^2."""
    m3, h3, lo3 = _m3(g.m), _d3(g.h, 1.0), _d3(g.lo)
    kap, kp = _c(q.ravel(), np.complex128)
    e3 = _d3(eta)
    b = np.empty(g.N, dtype=np.complex128)
    lib().or_rhs_plane_wave(g.dim, m3.ctypes.data, lo3.ctypes.data, h3.ctypes.data,
                            float(gamma), float(k0), kp, e3.ctypes.data, b.ctypes.data)
    return b.reshape(g.shape)


def rhs_phase(g: Grid, gamma, k0, q, eta):
    """b_j = q_j exp(i k0 cos(gamma) eta.x_j): the bounded stress
    right-hand side (the incoming phase without the contour's growth)."""
    m3, h3, lo3 = _m3(g.m), _d3(g.h, 1.0), _d3(g.lo)
    kap, kp = _c(q.ravel(), np.complex128)
    e3 = _d3(eta)
    b = np.empty(g.N, dtype=np.complex128)
    lib().or_rhs_phase(g.dim, m3.ctypes.data, lo3.ctypes.data, h3.ctypes.data,
                       float(gamma), float(k0), kp, e3.ctypes.data, b.ctypes.data)
    return b.reshape(g.shape)


def ff_integrand(g: Grid, gamma, k0, q, eta, u=None):
    """s_j = q_j (u_in,j + u_j)."""
    m3, h3, lo3 = _m3(g.m), _d3(g.h, 1.0), _d3(g.lo)
    kap, kp = _c(q.ravel(), np.complex128)
    e3 = _d3(eta)
    s = np.empty(g.N, dtype=np.complex128)
    if u is None:
        up = None
    else:
        uu, up = _c(u.ravel(), np.complex128)
    lib().or_ff_integrand(g.dim, m3.ctypes.data, lo3.ctypes.data, h3.ctypes.data,
                          float(gamma), float(k0), kp, e3.ctypes.data, up, s.ctypes.data)
    return s.reshape(g.shape)


def ff_contract(g: Grid, gamma, k0, s, dirs, method="separable", want_absum=False):
    """F_m = e^{i d gamma} prod h sum_j exp(-i k0 e^{ig} alpha_m.x_j) s_j."""
    dirs = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1, g.dim))
    M = dirs.shape[0]
    m3, h3, lo3 = _m3(g.m), _d3(g.h, 1.0), _d3(g.lo)
    ss, sp = _c(s.ravel(), np.complex128)
    F = np.empty(M, dtype=np.complex128)
    if method == "dense":
        ab = np.empty(M, dtype=np.float64) if want_absum else None
        lib().or_ff_dense(g.dim, m3.ctypes.data, lo3.ctypes.data, h3.ctypes.data,
                          float(gamma), float(k0), sp, M, dirs.ctypes.data, F.ctypes.data,
                          None if ab is None else ab.ctypes.data)
        return (F, ab) if want_absum else F
    lib().or_ff_separable(g.dim, m3.ctypes.data, lo3.ctypes.data, h3.ctypes.data,
                          float(gamma), float(k0), sp, M, dirs.ctypes.data, F.ctypes.data)
    return F


def farfield(g: Grid, gamma, k0, q, eta, u, dirs, method="separable"):
    """The full far-field map of a (solved) scattered wave u."""
    s = ff_integrand(g, gamma, k0, q, eta, u)
    return ff_contract(g, gamma, k0, s, dirs, method=method)
