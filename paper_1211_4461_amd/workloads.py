"""Seeded synthetic inputs: scatterers, potentials, incoming and outgoing
directions, and the grid/box/angle parameters of each workload.

This module holds no step of the method (no operator, smoother, transfer,
solve or quadrature).  It only evaluates the *given* coefficient functions at
the interior nodes, so that the GPU library and the CPU oracle are fed the
same arrays.  The workloads follow the paper's problems:

* Helmholtz (-Lap - k^2(z)) u = k0^2 chi(z) u_in(z) on the rotated grid
  z = e^{i gamma} x (Sec. 2.1, Sec. 3.1 eq. helmholtz_cc); the library input
  is the contrast k^2(z) - k0^2 = k0^2 chi(z) at every interior node.
* Schroedinger (-1/2 Lap + V - E) psi = phi, rewritten with
  k^2 = 2(E - V) (Sec. 5); the library input is V(z) at every interior node.

Two ways of evaluating chi at the nodes are provided:

* ``continued``: chi(z) with z = e^{i gamma} x and the bilinear continuation
  (z-c).(z-c) of |x-c|^2 (the analytic continuation the contour method
  assumes, Sec. 3.1);
* ``sampled``: chi(x) at the real node, used where the continued bumps would
  be amplified beyond any floating-point range (off-centre narrow bumps).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

HELMHOLTZ = 0
SCHRODINGER = 1


def interior_axes(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]):
    """Real coordinates of the interior nodes x_i = lo + i h, i = 1..n-1."""
    out = []
    for nk, lk, hk in zip(n, lo, hi):
        h = (hk - lk) / nk
        out.append(lk + h * np.arange(1, nk, dtype=np.float64))
    return out


def mesh(n, lo, hi):
    """Coordinate arrays in the library layout (x fastest): returns
    [X, Y] with shape (ny, nx) in 2D, [X, Y, Z] with shape (nz, ny, nx)."""
    ax = interior_axes(n, lo, hi)
    grids = np.meshgrid(*ax[::-1], indexing="ij")
    return grids[::-1]


def rotate(X, gamma):
    """Rotated coordinates z = e^{i gamma} x."""
    return [np.exp(1j * gamma) * x for x in X]


def gauss_continued(X, gamma, amp, width, centre):
    """amp * exp(-(z-c).(z-c)/w^2) at z = e^{i gamma} x (bilinear form)."""
    Z = rotate(X, gamma)
    q = sum((z - c) ** 2 for z, c in zip(Z, centre))
    return amp * np.exp(-q / width ** 2)


def gauss_sampled(X, amp, width, centre):
    """amp * exp(-|x-c|^2/w^2) at the real node."""
    q = sum((x - c) ** 2 for x, c in zip(X, centre))
    return amp * np.exp(-q / width ** 2)


def directions_2d(M: int):
    """alpha_m = 2 pi m / M, m = 0..M-1 (0 = forward along +x)."""
    a = 2.0 * np.pi * np.arange(M) / M
    return np.stack([np.cos(a), np.sin(a)], axis=1)


def directions_3d(n_azimuth: int, n_polar: int):
    """(sin t cos p, sin t sin p, cos t), p = 2 pi a / n_azimuth,
    t = (q + 1/2) pi / n_polar; polar-major order (all azimuths of one polar
    angle are consecutive)."""
    p = 2.0 * np.pi * np.arange(n_azimuth) / n_azimuth
    t = (np.arange(n_polar) + 0.5) * np.pi / n_polar
    T, P = np.meshgrid(t, p, indexing="ij")
    cz = np.cos(T)
    # identical cos(t) values for all azimuths of one polar angle
    return np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), cz], axis=-1).reshape(-1, 3)


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: int
    lo: float
    hi: float
    gamma: float
    kind: int
    k0: float
    energy: float
    coef: np.ndarray            # k0^2 chi (Helmholtz) or V (Schroedinger), x fastest
    eta: np.ndarray             # incoming direction (unit vector)
    dirs: np.ndarray            # outgoing directions, (M, dim)
    tol: float = 1e-10
    nu1: int = 2
    nu2: int = 2
    omega: float = 0.8
    params: Optional[dict] = None

    @property
    def shape(self):
        return (self.n - 1,) * self.dim

    @property
    def N(self):
        return (self.n - 1) ** self.dim

    def box(self):
        return [self.lo] * self.dim, [self.hi] * self.dim


def _eta(dim, angle=0.0):
    e = np.zeros(dim)
    e[0], e[1] = math.cos(angle), math.sin(angle)
    return e


# ---------------------------------------------------------------------------
# The five workloads.  Sizes and distributions are those of the paper's
# problem class at the scales the benchmark runs; see the design notes for the
# readings (intervals vs nodes, continuation, k0 for the stress variants).
# ---------------------------------------------------------------------------

def small_2d(n: int = 64, k0: float = 2.0, M: int = 180) -> Workload:
    """2D Helmholtz, box [-5,5]^2, n intervals, chi = 0.5 exp(-z.z) continued
    and cut to zero where the real |x| > 4, gamma = 30 deg, eta = +x."""
    gamma = math.pi / 6
    lo, hi = -5.0, 5.0
    X = mesh([n] * 2, [lo] * 2, [hi] * 2)
    chi = gauss_continued(X, gamma, 0.5, 1.0, (0.0, 0.0))
    r2 = X[0] ** 2 + X[1] ** 2
    chi = np.where(r2 > 16.0, 0.0, chi)
    coef = (k0 ** 2) * chi
    return Workload("small_2d", 2, n, lo, hi, gamma, HELMHOLTZ, k0, 0.0,
                    np.ascontiguousarray(coef, dtype=np.complex128), _eta(2),
                    directions_2d(M))


def bumps(seed: int, count: int = 8, rmax: float = 6.0):
    """Seeded Gaussian bumps: amplitude U[0.2,0.8], width U[0.5,1.5], centre
    area-uniform in |c| < rmax; draw order per bump: A, w, r, theta."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        A = rng.uniform(0.2, 0.8)
        w = rng.uniform(0.5, 1.5)
        r = rmax * math.sqrt(rng.uniform(0.0, 1.0))
        th = rng.uniform(0.0, 2.0 * math.pi)
        out.append((A, w, (r * math.cos(th), r * math.sin(th))))
    return out


def bumps_2d(n: int = 2048, seed: int = 1, k0: Optional[float] = 1.0,
             M: int = 360, lo: float = -10.0, hi: float = 10.0) -> Workload:
    """2D Helmholtz with 8 seeded Gaussian bumps sampled at the real nodes
    (real kappa), gamma = 30 deg.  k0 = None selects the stress wavenumber
    k0 h = 0.5."""
    gamma = math.pi / 6
    h = (hi - lo) / n
    if k0 is None:
        k0 = 0.5 / h
    X = mesh([n] * 2, [lo] * 2, [hi] * 2)
    chi = np.zeros_like(X[0])
    bl = bumps(seed)
    for A, w, c in bl:
        chi += gauss_sampled(X, A, w, c)
    coef = (k0 ** 2) * chi
    return Workload("bumps_2d", 2, n, lo, hi, gamma, HELMHOLTZ, k0, 0.0,
                    np.ascontiguousarray(coef, dtype=np.complex128), _eta(2),
                    directions_2d(M), params={"bumps": bl, "seed": seed})


def gauss_3d(n: int = 512, k0: Optional[float] = 1.0, n_az: int = 128,
             n_pol: int = 64, lo: float = -6.0, hi: float = 6.0) -> Workload:
    """3D Helmholtz, chi = 0.5 exp(-z.z/2) continued, gamma = 30 deg,
    eta = +x, directions on an azimuth x polar grid."""
    gamma = math.pi / 6
    h = (hi - lo) / n
    if k0 is None:
        k0 = 0.5 / h
    ax = interior_axes([n] * 3, [lo] * 3, [hi] * 3)
    # separable evaluation keeps host memory at one complex array
    e1 = np.exp(-(np.exp(1j * gamma) * ax[0]) ** 2 / 2.0)
    coef = np.empty((n - 1,) * 3, dtype=np.complex128)
    exy = e1[None, :] * e1[:, None]
    for iz in range(n - 1):
        coef[iz] = (k0 ** 2 * 0.5 * e1[iz]) * exy
    eta = np.array([1.0, 0.0, 0.0])
    return Workload("gauss_3d", 3, n, lo, hi, gamma, HELMHOLTZ, k0, 0.0, coef, eta,
                    directions_3d(n_az, n_pol))


def wells(seed: int, count: int = 3, depth=(0.5, 2.0)):
    """Seeded Gaussian wells: depth U[depth], width 1, centre area-uniform in
    |c| < 2; draw order per well: D, r, theta."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        D = rng.uniform(depth[0], depth[1])
        r = 2.0 * math.sqrt(rng.uniform(0.0, 1.0))
        th = rng.uniform(0.0, 2.0 * math.pi)
        out.append((D, (r * math.cos(th), r * math.sin(th))))
    return out


def schrodinger_potential(n: int, seed: int = 3, lo: float = -10.0, hi: float = 10.0,
                          gamma: float = math.pi / 6, deep: bool = False):
    """V(z) = -B exp(-z.z) - sum_i D_i exp(-(z-c_i).(z-c_i)) on the contour.

    deep=True: B = 2, D_i ~ U[0.5, 2].  Those wells hold bound states below
    -E, which complex scaling leaves on the real axis, and plain Jacobi
    V-cycles diverge on them (the breakdown the paper reports for bound-state
    energies, Sec. 5.4).  deep=False (default): the same shape scaled by 1/10,
    B = 0.2, D_i ~ U[0.05, 0.2], which stays in the V-cycle's convergence
    regime for E >= 0.5."""
    X = mesh([n] * 2, [lo] * 2, [hi] * 2)
    scale = 1.0 if deep else 0.1
    V = gauss_continued(X, gamma, -2.0 * scale, 1.0, (0.0, 0.0))
    for D, c in wells(seed, depth=(0.5 * scale, 2.0 * scale)):
        V = V + gauss_continued(X, gamma, -D, 1.0, c)
    return np.ascontiguousarray(V, dtype=np.complex128)


def schrodinger_batch(seed: int = 3, n_dirs: int = 32, energies=(0.5, 1.0, 2.0),
                      sizes=(256, 512, 1024), M: int = 360,
                      lo: float = -10.0, hi: float = 10.0) -> List[Workload]:
    """96 instances: 32 equispaced incoming directions x 3 energies, each on a
    grid drawn by seed from ``sizes`` (the same grid for every direction of
    one energy would make the batch uniform; here each instance draws its own
    n).  Returns the instances in (energy, direction) order."""
    gamma = math.pi / 6
    rng = np.random.default_rng(seed + 1000)
    ns = rng.choice(np.asarray(sizes), size=len(energies) * n_dirs)
    pots = {}
    out = []
    dirs = directions_2d(M)
    for ie, E in enumerate(energies):
        for d in range(n_dirs):
            n = int(ns[ie * n_dirs + d])
            if n not in pots:
                pots[n] = schrodinger_potential(n, seed, lo, hi, gamma)
            ang = 2.0 * math.pi * d / n_dirs
            out.append(Workload(f"schr_E{E}_d{d}_n{n}", 2, n, lo, hi, gamma, SCHRODINGER,
                                math.sqrt(2.0 * E), E, pots[n], _eta(2, ang), dirs,
                                params={"seed": seed}))
    return out


def radial_2d(n: int, L: float = 10.0, k0: float = 2.0, amp: float = 0.5,
              width: float = 1.0, gamma: float = math.pi / 6, M: int = 180) -> Workload:
    """Radially symmetric continued Gaussian chi = amp exp(-z.z/w^2) on
    [-L, L]^2 with no cut-off (a physics instance with a partial-wave
    reference)."""
    X = mesh([n] * 2, [-L] * 2, [L] * 2)
    chi = gauss_continued(X, gamma, amp, width, (0.0, 0.0))
    coef = (k0 ** 2) * chi
    return Workload("radial_2d", 2, n, -L, L, gamma, HELMHOLTZ, k0, 0.0,
                    np.ascontiguousarray(coef, dtype=np.complex128), _eta(2),
                    directions_2d(M), params={"amp": amp, "width": width})


def radial_3d(n: int, L: float = 12.0, k0: float = 1.0, amp: float = 0.5,
              width: float = math.sqrt(2.0), gamma: float = math.pi / 6,
              n_az: int = 16, n_pol: int = 8) -> Workload:
    """3D radially symmetric continued Gaussian chi = amp exp(-z.z/w^2)."""
    ax = interior_axes([n] * 3, [-L] * 3, [L] * 3)
    e1 = np.exp(-(np.exp(1j * gamma) * ax[0]) ** 2 / width ** 2)
    coef = (k0 ** 2 * amp) * (e1[:, None, None] * e1[None, :, None] * e1[None, None, :])
    return Workload("radial_3d", 3, n, -L, L, gamma, HELMHOLTZ, k0, 0.0,
                    np.ascontiguousarray(coef, dtype=np.complex128),
                    np.array([1.0, 0.0, 0.0]), directions_3d(n_az, n_pol),
                    params={"amp": amp, "width": width})


def gamma_from_ecs(theta: float) -> float:
    """Rotation angle of the full complex grid linked to an ECS layer angle
    theta (Sec. 3.3, eq. thetagamma; Table gammatheta: pi/6 -> 9.9 deg,
    pi/4 -> 14.6 deg)."""
    return math.atan(math.sin(theta) / (2.0 + math.cos(theta)))


def two_spheres(dim: int, n: int, k0: float, gamma: float, L: float = 20.0,
                M: int = 360, n_az: int = 16, n_pol: int = 8) -> Workload:
    """The model scatterer of the paper's Helmholtz experiments (Sec. 4):
    k0^2 chi = -1/5 (exp(-|x - c+|^2) + exp(-|x - c-|^2)), c+- = (0, +-4[, 0])
    (eq. chi2D in 2D, eq. chi3D in 3D), continued to z = e^{i gamma} x, on
    [-L, L]^d with eta = +x.  The contrast k0^2 chi does not depend on k0."""
    X = mesh([n] * dim, [-L] * dim, [L] * dim)
    coef = np.zeros(X[0].shape, dtype=np.complex128)
    for cy in (4.0, -4.0):
        c = (0.0, cy, 0.0)[:dim]
        coef += gauss_continued(X, gamma, -0.2, 1.0, c)
    dirs = directions_2d(M) if dim == 2 else directions_3d(n_az, n_pol)
    eta = np.zeros(dim)
    eta[0] = 1.0
    return Workload(f"two_spheres_{dim}d", dim, n, -L, L, gamma, HELMHOLTZ, k0, 0.0,
                    np.ascontiguousarray(coef, dtype=np.complex128), eta, dirs,
                    tol=1e-6, nu1=1, nu2=1)


# The model of Sec. 5.2 (eq. partialwave2d) and the energies of the
# complex-contour points of Fig. single_and_double: the bound-state energy
# lambda_0 = -1.02150069 of the 1D Hamiltonian at h = 0.05 plus 0.2 j.
ION_LAMBDA0 = -1.02150069
ION_ENERGIES = tuple(ION_LAMBDA0 + 0.2 * j for j in range(1, 21))


def ionization_2d(E: float, n: int = 256, h: float = 0.05, theta: float = math.pi / 7,
                  coarsest_n: int = 32) -> Workload:
    """The 2D radial partial-wave model of Sec. 5.2 at total energy E, on the
    contour grid of [0, n h]^2: V1(x) = -4.5 exp(-x^2), V2(y) = -4.5 exp(-y^2),
    V12 = 2 exp(-(x+y)^2), source phi = exp(-3 (x+y)^2), all continued to
    z = e^{i gamma} x, with gamma from the ECS angle theta = pi/7 through
    eq. thetagamma (8.5 deg, Sec. 5.4).  The paper's grid is [0,15]^2 with
    300 points (h = 0.05); a power-of-two grid keeps h and takes the box
    n h.  The coarsest multigrid level keeps h <= 0.4 (coarsest_n
    intervals), fine enough for the wells' bound states.  params: src (phi),
    v12, v1 (the one-body potential at the axis nodes, both axes)."""
    L = n * h
    gamma = gamma_from_ecs(theta)
    X, Y = mesh([n, n], [0.0, 0.0], [L, L])
    zx, zy = rotate([X, Y], gamma)
    z = np.exp(1j * gamma) * interior_axes([n], [0.0], [L])[0]
    v1 = -4.5 * np.exp(-z * z)
    s = zx + zy
    v12 = 2.0 * np.exp(-s * s)
    V = -4.5 * np.exp(-zx * zx) - 4.5 * np.exp(-zy * zy) + v12
    src = np.exp(-3.0 * s * s)
    c = lambda a: np.ascontiguousarray(a, dtype=np.complex128)
    return Workload(f"ionization_2d_E{E:+.4f}_n{n}", 2, n, 0.0, L, gamma, SCHRODINGER, 0.0, float(E), c(V),
                    np.array([1.0, 0.0]), np.zeros((0, 2)), tol=1e-10, nu1=1, nu2=1,
                    params={"src": c(src), "v12": c(v12), "v1": c(v1), "coarsest_n": coarsest_n, "h": h})


def random_field(n: int, seed: int, kh: float, lo: float = -10.0, hi: float = 10.0):
    """A random bump field (the bumps_2d law) at wavenumber k0 = kh / h;
    used as training input for the learned smoother."""
    return bumps_2d(n=n, seed=seed, k0=kh / ((hi - lo) / n), lo=lo, hi=hi)
