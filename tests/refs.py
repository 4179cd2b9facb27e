"""Independent restatements used to pin the oracle (tests only).

Nothing here calls the oracle: the operator is assembled from Kronecker
products as the paper writes it (Sec. 3.2, L = kron(I,T) + kron(T,I) with
T = tridiag(-1, 2, -1)), the transfer operators from their 1D matrices, and
the physics references from closed forms and the partial-wave expansion.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
from scipy import special
from scipy.integrate import solve_ivp


# ------------------------------------------------------------------ matrices

def T1(m):
    return sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1], format="csr")


def I1(m):
    return sp.identity(m, format="csr")


def kron_operator(m, h, gamma, kappa):
    """A = e^{-2ig} sum_k kron(..., T_k / h_k^2, ...) - diag(kappa), x fastest."""
    dim = len(m)
    rot = np.exp(-2j * gamma)
    A = None
    for k in range(dim):
        mats = []
        # x is the fastest index, so the x factor is the LAST kron factor
        for ax in reversed(range(dim)):
            mats.append(T1(m[ax]) / h[ax] ** 2 if ax == k else I1(m[ax]))
        term = mats[0]
        for mm in mats[1:]:
            term = sp.kron(term, mm, format="csr")
        A = term if A is None else A + term
    return (rot * A - sp.diags(np.asarray(kappa).ravel())).tocsr()


def fw_1d(mf):
    """1D full weighting (1/4, 1/2, 1/4), coarse I <- fine 2I-1, 2I, 2I+1."""
    mc = (mf - 1) // 2
    R = np.zeros((mc, mf))
    for I in range(mc):
        f = 2 * I + 1
        R[I, f - 1], R[I, f], R[I, f + 1] = 0.25, 0.5, 0.25
    return R


def kron_list(mats_x_first):
    """kron with the x matrix last (x fastest)."""
    out = None
    for M in reversed(mats_x_first):
        out = M if out is None else np.kron(out, M)
    return out


def fw(mf):
    return kron_list([fw_1d(m) for m in mf])


def prolong(mf):
    """Linear interpolation is 2 x (1D full weighting)^T per axis."""
    return kron_list([2.0 * fw_1d(m).T for m in mf])


def inject_index(mf):
    """Fine interior indices (x fastest, flattened) of the coarse nodes."""
    mc = [(m - 1) // 2 for m in mf]
    idx = [2 * np.arange(c) + 1 for c in mc]
    grids = np.meshgrid(*idx[::-1], indexing="ij")[::-1]
    flat = np.zeros_like(grids[0])
    stride = 1
    for k, gk in enumerate(grids):
        flat = flat + gk * stride
        stride *= mf[k]
    return flat.ravel()


def dense_gmres_step(A, b, u, m):
    """The least-residual update of u in the Krylov space of its residual,
    span{r, A r, ..., A^{m-1} r}, by a dense least-squares solve over the
    explicit (column-normalised) power basis."""
    r = b - A @ u
    nr = np.linalg.norm(r)
    if nr == 0.0:
        return u
    K = [r / nr]
    for _ in range(1, m):
        v = A @ K[-1]
        K.append(v / np.linalg.norm(v))
    K = np.stack(K, 1)
    c, *_ = np.linalg.lstsq(A @ K, r, rcond=None)
    return u + K @ c


def color_mask(m):
    """True at the "red" points (0-based interior indices summing to an even
    number), x fastest."""
    idx = np.meshgrid(*[np.arange(mk) for mk in m[::-1]], indexing="ij")
    return (sum(idx) % 2 == 0).ravel()


def dense_rbgs(A, b, u, red):
    """Red-black Gauss-Seidel as a block solve in the red/black ordering:
    u_r = D_r^{-1} (b_r - A_rb u_b), then u_b = D_b^{-1} (b_b - A_br u_r)."""
    u = u.copy()
    for c in (red, ~red):
        o = ~c
        D = np.diag(A)[c]
        u[c] = (b[c] - A[np.ix_(c, o)] @ u[o]) / D
    return u


def dense_vcycle(m, h, gamma, kappa, b, u, nu1, nu2, omega, coarsest_n=8, krylov_m=0, rbgs=False):
    """One V(nu1, nu2) cycle written with dense matrices (krylov_m > 0:
    GMRES(krylov_m) smoothing steps, rbgs: red-black Gauss-Seidel sweeps
    instead of omega-Jacobi sweeps)."""
    m = list(m)
    A = kron_operator(m, h, gamma, kappa).toarray()
    if min(mk + 1 for mk in m) <= coarsest_n:
        return np.linalg.solve(A, b)
    D = np.diag(A)

    red = color_mask(m)

    def smooth(u):
        if krylov_m:
            return dense_gmres_step(A, b, u, krylov_m)
        if rbgs:
            return dense_rbgs(A, b, u, red)
        return u + omega * (b - A @ u) / D

    for _ in range(nu1):
        u = smooth(u)
    r = b - A @ u
    R = fw(m)
    bc = R @ r
    mc = [(mk - 1) // 2 for mk in m]
    kc = np.asarray(kappa).ravel()[inject_index(m)]
    ec = dense_vcycle(mc, [2 * hk for hk in h], gamma, kc, bc, np.zeros_like(bc),
                      nu1, nu2, omega, coarsest_n, krylov_m, rbgs)
    u = u + prolong(m) @ ec
    for _ in range(nu2):
        u = smooth(u)
    return u


def prolong_sparse(mf):
    """prolong(mf) as a sparse matrix (large fine grids)."""
    out = None
    for m in mf:                 # x first; kron puts later factors slower
        M = sp.csr_matrix(2.0 * fw_1d(m).T)
        out = M if out is None else sp.kron(M, out, format="csr")
    return out


def dense_fmg(m, h, gamma, kappa, b, k, nu1, nu2, omega, coarsest_n=8):
    """Full-multigrid initial guess for the grid with interior counts m,
    written with the matrices above: the right-hand side and kappa of each
    coarser grid are the finer ones at the coarse nodes, the coarsest system
    is solved exactly, each level in between runs k dense V-cycles from the
    interpolated coarser solution, and the guess is the interpolated
    solution of the first coarse level."""
    m = list(m)
    if min(mk + 1 for mk in m) <= coarsest_n:
        return np.linalg.solve(kron_operator(m, h, gamma, kappa).toarray(), b)
    idx = inject_index(m)
    mc = [(mk - 1) // 2 for mk in m]
    hc = [2 * hk for hk in h]
    kc, bc = np.asarray(kappa).ravel()[idx], np.asarray(b).ravel()[idx]
    if min(mk + 1 for mk in mc) <= coarsest_n:
        uc = np.linalg.solve(kron_operator(mc, hc, gamma, kc).toarray(), bc)
    else:
        uc = dense_fmg(mc, hc, gamma, kc, bc, k, nu1, nu2, omega, coarsest_n)
        for _ in range(k):
            uc = dense_vcycle(mc, hc, gamma, kc, bc, uc, nu1, nu2, omega, coarsest_n)
    return prolong_sparse(m) @ uc


# ------------------------------------------------------------------ physics

def born_2d(k0, amp, sigma, alpha_dirs, eta):
    """Fourier transform of k0^2 amp exp(-|x|^2/sigma^2) at k0 (alpha - eta):
    k0^2 amp pi sigma^2 exp(-k0^2 sigma^2 |alpha - eta|^2 / 4)."""
    d2 = np.sum((alpha_dirs - eta[None, :]) ** 2, axis=1)
    return k0 ** 2 * amp * math.pi * sigma ** 2 * np.exp(-(k0 ** 2) * sigma ** 2 * d2 / 4.0)


def born_nd(k0, amp, sigma, alpha_dirs, eta):
    d = alpha_dirs.shape[1]
    d2 = np.sum((alpha_dirs - eta[None, :]) ** 2, axis=1)
    return k0 ** 2 * amp * (math.pi * sigma ** 2) ** (d / 2) * np.exp(-(k0 ** 2) * sigma ** 2 * d2 / 4.0)


def partial_wave_2d(k0, chi, angles, mmax=25, r0=1e-3, r1=9.0):
    """Far field of a radially symmetric real scatterer k^2 = k0^2 (1 + chi(r))
    in the normalisation F = -4i sum_m t_m e^{i m phi}, with t_m from the
    regular radial solution matched to J_m + t_m H_m^(1) at r1."""
    def rhs(r, y, m):
        R, dR = y[0] + 1j * y[1], y[2] + 1j * y[3]
        ddR = -dR / r - (k0 ** 2 * (1.0 + chi(r)) - m * m / (r * r)) * R
        return [dR.real, dR.imag, ddR.real, ddR.imag]

    t = np.zeros(mmax + 1, dtype=np.complex128)
    for m in range(mmax + 1):
        # regular start R ~ r^m, scaled to R(r0) = 1 (only R'/R matters)
        kap0 = k0 ** 2 * (1.0 + chi(r0))
        dR0 = m / r0 if m > 0 else -0.5 * kap0 * r0
        sol = solve_ivp(rhs, (r0, r1), [1.0, 0.0, dR0, 0.0], args=(m,), rtol=1e-12,
                        atol=1e-14, method="DOP853")
        R = sol.y[0, -1] + 1j * sol.y[1, -1]
        dR = sol.y[2, -1] + 1j * sol.y[3, -1]
        beta = dR / R
        x = k0 * r1
        J, dJ = special.jv(m, x), special.jvp(m, x)
        H, dH = special.hankel1(m, x), special.h1vp(m, x)
        t[m] = (k0 * dJ - beta * J) / (beta * H - k0 * dH)
    F = np.zeros(len(angles), dtype=np.complex128)
    for m in range(mmax + 1):
        F += (1 if m == 0 else 2) * t[m] * np.cos(m * angles)
    return -4j * F, t
