"""FP64 CPU oracle for the ionisation observables of the 2D radial
partial-wave Schroedinger model (Sec. 5.1-5.4 of arXiv 1211.4461).

TEST INFRASTRUCTURE ONLY: the reference that the HIP library's ionisation
entry points are checked against.  Only the tests, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it.  Plain numpy/scipy
in double precision; it shares no code with the GPU library.

Conventions (the same discrete problem as the multigrid oracle):
  * one axis of the contour grid: n intervals on [lo, hi], h = (hi-lo)/n,
    interior nodes z_i = lo + i h e^{i gamma}, i = 1..n-1 (lo = 0 for the
    radial coordinates of eq. partialwave2d, whose Dirichlet condition at 0
    is the grid's boundary value), h~ = h e^{i gamma};
  * 2D fields are (ny-1, nx-1) arrays, x fastest;
  * the Schroedinger equation (-1/2 Lap + V - E) u = phi is solved in its
    Helmholtz form (-Lap - 2(E - V)) u = 2 phi (Sec. 5 introduction), on the
    contour -Lap = e^{-2i gamma} (-Lap_h) (Sec. 5.2, rotated stencil).

Readings of the paper taken here:
  * test-function normalisation (eq. testfunction "normalized with 1/sqrt k"):
    the regular solution whose free-wave amplitude is 1/sqrt(k), i.e.
    phi_k ~ sin(k x + delta)/sqrt(k) where the potential has died out.  On
    the grid, the free recurrence keeps the invariant
        A^2 = (p_i^2 + p_{i+1}^2 - 2 c p_i p_{i+1}) / (1 - c^2),
        c = 1 - h~^2 k^2 / 2,
    (the squared amplitude of p_i = A sin(theta i + delta), cos theta = c),
    evaluated at the first node past the last one where |V| > 1e-13; A takes
    the root with positive real part.
  * bound state (eq. boundstate): the eigenvector of the rotated 1D
    Hamiltonian normalised by the contour integral sum phi^2 h~ = 1 (the
    continuation of int phi^2 dx = 1), sign with Re phi_1 > 0.
  * channel wavenumbers: k_n = sqrt(2(E - Re lambda_n)); double-ionisation
    energies eps_m = (m + 1/2) E / M (midpoint rule over [0, E]),
    k1 = sqrt(2 eps), k2 = sqrt(2(E - eps)) (eq. double-ionization).
  * cross sections (Fig. single_and_double): half the outgoing probability
    flux into each kind of channel, which is the scale of the printed points
    (the prefactor 8 pi^2 / k0^2 of the paper's sigma(k1, k2) needs the
    incident momentum of the underlying collision, which this model does not
    define):  single 4 |s_0|^2, double (4/pi) int_0^E |f|^2 d eps, total
    Im <phi, u> (the optical theorem: the total flux is 2 Im <phi, u>).
"""
from __future__ import annotations

import math

import numpy as np

V_NEGLIGIBLE = 1e-13


def axis(n: int, lo: float, hi: float, gamma: float):
    """(h, h~, z): spacing, rotated spacing, contour nodes of one axis."""
    h = (hi - lo) / n
    ht = h * np.exp(1j * gamma)
    z = lo + ht * np.arange(1, n)
    return h, ht, z


def hamiltonian_1d(n: int, lo: float, hi: float, gamma: float, v):
    """Dense rotated 1D Hamiltonian -1/2 e^{-2i gamma} D2/h^2 + diag(V(z_i))
    with Dirichlet ends (Sec. 5.2, the rotated stencil)."""
    h, ht, _ = axis(n, lo, hi, gamma)
    m = n - 1
    c = 1.0 / (ht * ht)
    H = np.zeros((m, m), dtype=np.complex128)
    for i in range(m):
        H[i, i] = c + v[i]
        if i > 0:
            H[i, i - 1] = -0.5 * c
        if i + 1 < m:
            H[i, i + 1] = -0.5 * c
    return H


def bound_state(n: int, lo: float, hi: float, gamma: float, v, shift: float):
    """eq. boundstate on the contour: the eigenpair of the rotated 1D
    Hamiltonian whose eigenvalue lies nearest to ``shift``; returns
    (lambda, phi) with sum phi^2 h~ = 1 and Re phi_1 > 0."""
    _, ht, _ = axis(n, lo, hi, gamma)
    H = hamiltonian_1d(n, lo, hi, gamma, np.asarray(v, dtype=np.complex128))
    w, V = np.linalg.eig(H)
    i = int(np.argmin(np.abs(w - shift)))
    phi = V[:, i]
    phi = phi / np.sqrt(np.sum(phi * phi) * ht)
    if phi[0].real < 0:
        phi = -phi
    return complex(w[i]), phi


def reference_index(v, tau: float = V_NEGLIGIBLE) -> int:
    """0-based index of the first node past the last one with |V| > tau."""
    big = np.nonzero(np.abs(np.asarray(v)) > tau)[0]
    return int(big[-1]) + 1 if big.size else 0


def test_function(n: int, lo: float, hi: float, gamma: float, v, k: float):
    """eq. testfunction on the contour: the regular solution of
    (-1/2 d^2/dz^2 + V - k^2/2) phi = 0 with phi(lo) = 0, by the three-point
    recurrence of the rotated stencil, normalised to free-wave amplitude
    1/sqrt(k) (reading above)."""
    _, ht, _ = axis(n, lo, hi, gamma)
    v = np.asarray(v, dtype=np.complex128)
    m = n - 1
    p = np.zeros(m, dtype=np.complex128)
    prev = 0.0 + 0.0j
    p[0] = 1.0
    for i in range(m - 1):
        # -1/2 (p_{i+1} - 2 p_i + p_{i-1}) / h~^2 + (V_i - k^2/2) p_i = 0
        p[i + 1] = 2.0 * p[i] - prev + ht * ht * (2.0 * v[i] - k * k) * p[i]
        prev = p[i]
    r = reference_index(v)
    if r + 1 >= m:
        raise ValueError("the potential does not die out inside the box")
    c = 1.0 - 0.5 * ht * ht * k * k
    a2 = (p[r] ** 2 + p[r + 1] ** 2 - 2.0 * c * p[r] * p[r + 1]) / (1.0 - c * c)
    A = np.sqrt(a2)
    if A.real < 0:
        A = -A
    return p / (A * math.sqrt(k))


def test_functions(n: int, lo: float, hi: float, gamma: float, v, ks):
    return np.stack([test_function(n, lo, hi, gamma, v, float(k)) for k in ks])


def wavenumbers(E: float, lam: complex, M: int):
    """(k_n, k1[M], k2[M], w[M]): the single-ionisation channel wavenumber
    (None below its threshold) and the midpoint nodes and weights of the
    double-ionisation energy integral (empty for E <= 0)."""
    lr = complex(lam).real
    kn = math.sqrt(2.0 * (E - lr)) if E > lr else None
    if E <= 0.0 or M <= 0:
        z = np.zeros(0)
        return kn, z, z, z
    eps = (np.arange(M) + 0.5) * (E / M)
    return kn, np.sqrt(2.0 * eps), np.sqrt(2.0 * (E - eps)), np.full(M, E / M)


def amplitudes(gamma: float, hx: float, hy: float, src, v12, u, tx, ty):
    """eq. single-ionization / eq. double-ionization on the contour:
    a_m = h~x h~y sum_{j,i} tx[m, i] ty[m, j] (phi - V12 u)[j, i]; and the
    optical-theorem product <phi, u> = h~x h~y sum phi u.  Plain sums."""
    pre = hx * hy * np.exp(2j * gamma)
    rho = np.asarray(src) - np.asarray(v12) * np.asarray(u)
    tx = np.atleast_2d(tx)
    ty = np.atleast_2d(ty)
    amp = np.array([pre * np.sum(ty[m][:, None] * tx[m][None, :] * rho) for m in range(tx.shape[0])])
    opt = pre * np.sum(np.asarray(src) * np.asarray(u))
    return amp, complex(opt)


def cross_sections(s0, f, w, opt):
    """(single, double, total) from the amplitudes (reading above)."""
    single = 4.0 * abs(s0) ** 2 if s0 is not None else 0.0
    double = (4.0 / math.pi) * float(np.sum(np.asarray(w) * np.abs(np.asarray(f)) ** 2)) if len(w) else 0.0
    return single, double, float(np.imag(opt))


# ---------------------------------------------------------------- the model

def model_fields(n: int, L: float, gamma: float):
    """The Sec. 5.2 model on the contour grid of [0, L]^2: V1(x) = -4.5 e^{-x^2},
    V2(y) = -4.5 e^{-y^2}, V12 = 2 e^{-(x+y)^2}, phi = e^{-3 (x+y)^2}.
    Returns (v1 axis, V total, V12, phi) with 2D arrays (n-1, n-1), x fastest."""
    _, _, z = axis(n, 0.0, L, gamma)
    v1 = -4.5 * np.exp(-z * z)
    Zy, Zx = np.meshgrid(z, z, indexing="ij")
    s = Zx + Zy
    v12 = 2.0 * np.exp(-s * s)
    V = v1[None, :] + v1[:, None] + v12
    src = np.exp(-3.0 * s * s)
    return v1, V, v12, src


def solve_direct(n: int, L: float, gamma: float, V, E: float, src):
    """u of (-1/2 Lap + V - E) u = phi on the contour grid of [0, L]^2 by a
    sparse direct solve of the Helmholtz form (-Lap - 2(E - V)) u = 2 phi."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    _, ht, _ = axis(n, 0.0, L, gamma)
    m = n - 1
    D2 = sp.diags([np.ones(m - 1), -2.0 * np.ones(m), np.ones(m - 1)], [-1, 0, 1]) / (ht * ht)
    I = sp.identity(m)
    A = -(sp.kron(I, D2) + sp.kron(D2, I)) - sp.diags(2.0 * (E - np.asarray(V).ravel()))
    return spl.spsolve(A.tocsc(), 2.0 * np.asarray(src).ravel()).reshape(m, m)


def observables(n: int, L: float, gamma: float, E: float, M: int, u=None, shift: float = -1.0):
    """All cross sections of the model at energy E: bound state, test
    functions, amplitudes, cross sections (u from ``solve_direct`` unless
    given).  Returns a dict."""
    v1, V, v12, src = model_fields(n, L, gamma)
    if u is None:
        u = solve_direct(n, L, gamma, V, E, src)
    lam, phi0 = bound_state(n, 0.0, L, gamma, v1, shift)
    kn, k1, k2, w = wavenumbers(E, lam, M)
    h = L / n
    s0 = None
    if kn is not None:
        a, opt = amplitudes(gamma, h, h, src, v12, u, test_functions(n, 0.0, L, gamma, v1, [kn]), phi0[None, :])
        s0 = a[0]
    f = np.zeros(0, dtype=np.complex128)
    if len(k1):
        f, opt = amplitudes(gamma, h, h, src, v12, u, test_functions(n, 0.0, L, gamma, v1, k1),
                            test_functions(n, 0.0, L, gamma, v1, k2))
    if kn is None and not len(k1):
        _, opt = amplitudes(gamma, h, h, src, v12, u, np.zeros((1, n - 1)), np.zeros((1, n - 1)))
    single, double, total = cross_sections(s0, f, w, opt)
    return dict(lam=lam, kn=kn, s0=s0, f=f, k1=k1, k2=k2, w=w, opt=opt, single=single, double=double,
                total=total, u=u)
