"""Training data and training loop of the learned smoother.

Data: (error, residual) pairs from plain weighted-Jacobi V-cycles of the
library on seeded random bump fields (the bumps law of the 2048^2 workload,
k0 h drawn from a range), plus white-noise errors.  For each field the converged solution
u* is computed first; the iterates u_k of a fresh solve from u = 0 give
e_k = u* - u_k and r_k = b - A u_k.  32 x 32 patches at random positions
are cut out and scaled as the smoother sees them: r / s, e / (s h^2),
kappa h^2, with s the RMS of r over the whole grid.

Training: Adam on minibatches of patches through ml_train_step (the
library's forward and backward kernels).  Everything numerical runs in the
library; torch only holds the device arrays and cuts patches.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import ffmg
from . import workloads as W

PATCH = 32


def init_weights(seed: int, scale: float = 1.0):
    """Complex Gaussian initialisation, variance scale^2 / fan-in per part."""
    rng = np.random.default_rng(seed)
    out = []
    for s in ffmg.NET_SHAPES:
        sd = scale * math.sqrt(1.0 / (9 * s[2]))
        out.append(rng.normal(0.0, sd, s) + 1j * rng.normal(0.0, sd, s))
    return out


def jacobi_init(seed: int, gamma: float = math.pi / 6, omega: float = 0.8, noise: float = 0.1):
    """Weights that start as one weighted-Jacobi sweep of the contour operator
    (kappa h^2 neglected against the Laplacian's diagonal): channel 0 carries
    r~ through the centre taps (gate 1) and layer 3 scales it by
    omega / (4 e^{-2 i gamma}); the other channels start as small noise and
    do not feed channel 0."""
    W1, W2, W3 = init_weights(seed, noise)
    c = omega / (4.0 * np.exp(-2j * gamma))
    W1[:, 0, :] = 0.0
    W2[:, 0, :] = 0.0
    W2[:, :, 0] = 0.0
    W3[:, :, 0] = 0.0
    W1[4, 0, 0] = 1.0
    W2[4, 0, 0] = 1.0
    W3[4, 0, 0] = c
    return [W1, W2, W3]


def phase_rhs(w, torch, device="cuda", h=None):
    """b = q exp(i k0 cos(gamma) eta.x) from the library (mg_rhs_phase): the
    plane wave's phase without the contour's exponential growth, for k0 h
    near 0.5 where the contour wave itself would exceed the floating-point
    range.  h: a handle of the workload (one is set up if None)."""
    own = h is None
    if own:
        h = ffmg.setup_workload(w, device=device, options=ffmg.default_options())[0]
    b = torch.empty((w.n - 1,) * w.dim, dtype=torch.complex128, device=device)
    ffmg.mg_rhs_phase(h, w.eta, b)
    if own:
        torch.cuda.synchronize()
        h.destroy()
    return b


@dataclass
class PatchSet:
    rt: object     # (count, 32, 32) complex64, r / s
    kt: object     # kappa h^2
    et: object     # e / (s h^2)

    @property
    def count(self):
        return self.rt.shape[0]


def make_patches(torch, n_fields=48, n=256, kh=(0.02, 0.6), iterates=3, patches_per_iterate=64, noise_sets=2,
                 smooth_sets=0, seed=1000, iterate_kh_max=0.6, kh_dist="uniform", device="cuda"):
    """(residual, error) patches from plain V-cycle iterates; fields use seeds
    seed, seed + 1, ...; k0 h uniform (or log-uniform) in kh.  Per field two sequences of
    iterates from u = 0 are sampled: V(2,2) cycles, and V(2,0) cycles, whose
    iterates are the state right after the coarse-grid correction (the
    interpolation leaves high-frequency error there, which is what the
    smoother has to remove).  noise_sets white-noise errors e (with r = A e)
    per field add every frequency with equal weight, smooth_sets smooth
    random errors the step must not amplify.  The k0 h range covers
    the coarse levels of a hierarchy too (k0 h doubles per level); iterates
    are sampled only for k0 h <= iterate_kh_max, where the plain cycle on the
    field's own grid converges, white noise for every field."""
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    R, K, E = [], [], []
    m = n - 1

    def cut(r, e, kap, s, hh, count):
        ys = rng.integers(0, m - PATCH + 1, count)
        xs = rng.integers(0, m - PATCH + 1, count)
        for y0, x0 in zip(ys, xs):
            sl = (slice(int(y0), int(y0) + PATCH), slice(int(x0), int(x0) + PATCH))
            R.append(r[sl] / s)
            E.append(e[sl] / (s * hh * hh))
            K.append(kap[sl])

    for f in range(n_fields):
        if kh_dist == "log":
            khf = float(np.exp(rng.uniform(np.log(kh[0]), np.log(kh[1]))))
        else:
            khf = float(rng.uniform(kh[0], kh[1]))
        w = W.random_field(n, seed + f, khf)
        hs = [ffmg.setup_workload(w, device=device, options=ffmg.default_options())[0],
              ffmg.setup_workload(w, device=device, options=ffmg.default_options(nu2=0))[0]]
        hh = (w.hi - w.lo) / w.n
        b = phase_rhs(w, torch, device, h=hs[0])
        kap = torch.from_numpy(np.ascontiguousarray((w.k0 ** 2 + w.coef) * hh * hh)).to(device)
        Au = torch.empty_like(b)
        if khf <= iterate_kh_max:
            ustar = torch.zeros_like(b)
            ffmg.mg_solve(hs[0], b, ustar, tol=1e-12)
        for h in (hs if khf <= iterate_kh_max else []):
            u = torch.zeros_like(b)
            for k in range(iterates):
                ffmg.mg_vcycle(h, b, u)
                r = ffmg.mg_residual(h, b, u, Au)
                e = ustar - u
                s = float(torch.sqrt(torch.mean(torch.abs(r) ** 2)))
                if s > 0:
                    cut(r, e, kap, s, hh, patches_per_iterate)
        # smooth random errors (a coarse random field interpolated to the
        # grid): what the step must not amplify
        for _ in range(smooth_sets):
            c = torch.randn((2, 1, m // 8 + 2, m // 8 + 2), generator=gen, device=device, dtype=torch.float64)
            c = torch.nn.functional.interpolate(c, size=(m, m), mode="bilinear", align_corners=True)[:, 0]
            e = torch.complex(c[0], c[1]).contiguous()
            ffmg.mg_apply(hs[0], e, Au)
            s = float(torch.sqrt(torch.mean(torch.abs(Au) ** 2)))
            cut(Au, e, kap, s, hh, patches_per_iterate)
        # white-noise errors: every frequency the smoother has to damp
        for _ in range(noise_sets):
            e = torch.complex(torch.randn(b.shape, generator=gen, device=device, dtype=torch.float64),
                              torch.randn(b.shape, generator=gen, device=device, dtype=torch.float64))
            ffmg.mg_apply(hs[0], e, Au)
            s = float(torch.sqrt(torch.mean(torch.abs(Au) ** 2)))
            cut(Au, e, kap, s, hh, patches_per_iterate)
        for h in hs:
            h.destroy()
    stack = lambda L: torch.stack(L).to(torch.complex64).contiguous()
    return PatchSet(stack(R), stack(K), stack(E))


def train(torch, net: "ffmg.Net", data: PatchSet, steps=1500, batch=256, lr=1e-3, lr_final=1e-4, seed=0,
          border=4, log_every=0):
    """Adam with a cosine learning-rate decay; returns the loss history
    (every log_every steps, or the first and last)."""
    g = torch.Generator(device=data.rt.device)
    g.manual_seed(seed)
    hist = []
    for it in range(steps):
        idx = torch.randint(0, data.count, (batch,), generator=g, device=data.rt.device)
        rt, kt, et = data.rt[idx].contiguous(), data.kt[idx].contiguous(), data.et[idx].contiguous()
        a = lr_final + 0.5 * (lr - lr_final) * (1.0 + math.cos(math.pi * it / max(steps - 1, 1)))
        want = (log_every and it % log_every == 0) or it == 0 or it == steps - 1
        L = net.train_step(rt, kt, et, a, border=border, want_loss=bool(want))
        if want:
            hist.append((it, L))
    return hist
