"""Seeded synthetic inputs for the posterior-mean system of the CMB source-separation model.

This module only *draws* inputs: grid shapes, hyperparameters, the mixing matrix, per-pixel
noise weights, simulated observations and the standard-normal draws used for perturbation
sampling.  It contains none of the solver's arithmetic (no stencil, no mixing contraction, no
right-hand-side assembly, no solve), so that the CPU oracle and the GPU path can both consume the
same inputs without sharing any computation.

Model being simulated (Section 2.1, eq. (model)): every pixel j carries k source values s_j and
f observed brightnesses y_j = A s_j + eps_j, with independent Gaussian noise whose precision at
frequency f and pixel p is W[f, p].  The paper's own simulation draws i.i.d. normal sources
(Section 4, experiment set-up); the default here draws smooth Gaussian random fields instead and
keeps i.i.d. sources as a variant.

Distributions of the named workloads (seed = 1000 + workload index, fixed draw order):
  kappa_j ~ U(0.1, 1), tau_j ~ U(0.5, 2)      (k each)
  A[f, j] ~ U(0.2, 1.5)                        (f x k, row-major: row f is a_f)
  sigma_f ~ U(0.5, 2)                          (noise level of frequency f)
  weights: homoscedastic  W[f, p] = sigma_f^-2
           heteroscedastic W[f, p] = sigma_f^-2 * omega[f, p], omega ~ lognormal(0, 0.5) i.i.d.
           separable       W[f, p] = sigma_f^-2 * omega[p]   (one omega per pixel, shared over f)
           masked          additionally W[:, p] = 0 for pixels drawn Bernoulli(mask_frac)
  sources S_j: Gaussian random field with spectrum (1 + (l |k|)^2)^-2, unit variance
  Y[f] = sum_j A[f, j] S_j + W[f]^-1/2 eps_f  (Y = 0 where W = 0)
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Problem",
    "make_problem",
    "workload",
    "WORKLOADS",
    "po_draws",
    "random_maps",
]


@dataclass
class Problem:
    """One posterior-mean system on an ny x nx grid, periodic or one HEALPix-like face.

    Pixel p = iy * nx + ix.  Arrays are float64 numpy arrays:
      kappa[k], tau[k]   prior hyperparameters of component j (Q_j = tau_j (kappa_j^2 I - Lap)^2)
      A[f, k]            mixing matrix, row f = a_f
      W[f, n_pix]        per-pixel noise precision (>= 0; 0 = masked pixel)
      Y[f, n_pix]        observed maps, stacked by map
    """

    ny: int
    nx: int
    k: int
    f: int
    kappa: np.ndarray
    tau: np.ndarray
    A: np.ndarray
    W: np.ndarray
    Y: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)
    boundary: str = "periodic"     # "periodic" (torus) or "face" (links only inside the grid)

    @property
    def n_pix(self) -> int:
        return self.ny * self.nx

    @property
    def n(self) -> int:
        return self.k * self.ny * self.nx


def _gaussian_field(rng: np.random.Generator, ny: int, nx: int, corr: float) -> np.ndarray:
    """Unit-variance stationary Gaussian random field on the periodic grid.

    White noise filtered in Fourier space by (1 + (corr |k|)^2)^-1 (amplitude), i.e. a power
    spectrum (1 + (corr |k|)^2)^-2; a generic smoothness model for diffuse sources, not tied to
    the prior of the solver.
    """
    white = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None] * 2.0 * np.pi
    kx = np.fft.fftfreq(nx)[None, :] * 2.0 * np.pi
    amp = 1.0 / (1.0 + corr * corr * (kx * kx + ky * ky))
    fld = np.fft.ifft2(np.fft.fft2(white) * amp).real
    sd = fld.std()
    if sd > 0:
        fld = fld / sd
    return fld


def make_problem(
    ny: int,
    nx: int,
    k: int,
    f: int,
    seed: int,
    noise: str = "hetero",
    mask_frac: float = 0.0,
    sources: str = "field",
    kappa: Optional[np.ndarray] = None,
    tau: Optional[np.ndarray] = None,
    A: Optional[np.ndarray] = None,
    sigma: Optional[np.ndarray] = None,
    name: str = "",
    boundary: str = "periodic",
) -> Problem:
    """Draw one problem.  Draw order is fixed: kappa, tau, A, sigma, weights/mask, sources, noise.

    noise: 'homo' | 'hetero' | 'separable'.  Explicit kappa/tau/A/sigma override the draws but the
    corresponding random numbers are still consumed, so the other draws do not shift.
    """
    rng = np.random.default_rng(seed)
    n_pix = ny * nx
    kap = rng.uniform(0.1, 1.0, size=k)
    ta = rng.uniform(0.5, 2.0, size=k)
    Am = rng.uniform(0.2, 1.5, size=(f, k))
    sig = rng.uniform(0.5, 2.0, size=f)
    if kappa is not None:
        kap = np.asarray(kappa, dtype=np.float64).reshape(k).copy()
    if tau is not None:
        ta = np.asarray(tau, dtype=np.float64).reshape(k).copy()
    if A is not None:
        Am = np.asarray(A, dtype=np.float64).reshape(f, k).copy()
    if sigma is not None:
        sig = np.asarray(sigma, dtype=np.float64).reshape(f).copy()
    base = 1.0 / (sig * sig)
    if noise == "homo":
        W = np.repeat(base[:, None], n_pix, axis=1)
    elif noise == "hetero":
        W = base[:, None] * rng.lognormal(0.0, 0.5, size=(f, n_pix))
    elif noise == "separable":
        nsep = rng.lognormal(0.0, 0.5, size=(1, n_pix))
        W = base[:, None] * nsep
    else:
        raise ValueError(f"unknown noise law {noise!r}")
    W = np.ascontiguousarray(W, dtype=np.float64)
    if mask_frac > 0.0:
        masked = rng.random(n_pix) < mask_frac
        W[:, masked] = 0.0
    corr = max(2.0, min(ny, nx) / 32.0)
    if sources == "field":
        S = np.stack([_gaussian_field(rng, ny, nx, corr).ravel() for _ in range(k)])
    elif sources == "iid":
        S = rng.standard_normal((k, n_pix))
    else:
        raise ValueError(f"unknown source law {sources!r}")
    eps = rng.standard_normal((f, n_pix))
    with np.errstate(divide="ignore"):
        sd = np.where(W > 0, 1.0 / np.sqrt(np.where(W > 0, W, 1.0)), 0.0)
    Y = Am @ S + sd * eps
    Y[W == 0] = 0.0
    meta = {"seed": seed, "noise": noise, "mask_frac": mask_frac, "sources": sources}
    if noise == "separable" and mask_frac == 0.0:
        # the factors of W[f, p] = t_f n_p (W holds exactly their rounded products)
        meta["t"] = base.copy()
        meta["n"] = nsep[0].copy()
    if boundary not in ("periodic", "face"):
        raise ValueError(f"unknown boundary {boundary!r}")
    return Problem(ny, nx, k, f, kap, ta, Am, W, np.ascontiguousarray(Y), name=name, meta=meta,
                   boundary=boundary)


# Named workloads.  Sizes follow the paper's per-patch pixel counts (N = 4^h, App. A) and its
# numbers of maps (9) and sources (4); tolerances and precisions are the solver settings each
# workload is run with.
WORKLOADS = {
    "tiny_64": dict(index=0, ny=64, nx=64, k=3, f=6, noise="homo", tol=1e-10, precision="f64"),
    "het_1024": dict(index=1, ny=1024, nx=1024, k=3, f=9, noise="hetero", tol=1e-8,
                     precision="f64+mixed"),
    "masked_2048": dict(index=2, ny=2048, nx=2048, k=4, f=9, noise="hetero", mask_frac=0.1,
                        tol=1e-8, precision="mixed"),
    "batched_8grids": dict(index=3, sizes=[256, 384, 512, 640, 768, 896, 1024, 1024], nrhs=8,
                           k=3, f=6, noise="hetero", tol=1e-8, precision="mixed"),
    "grad_512": dict(index=4, ny=512, nx=512, k=4, f=9, noise="hetero", tol=1e-10,
                     precision="f64"),
    # the case the paper solves in Sylvester form (Section 3.3): separable noise t_f n_p and one
    # kappa shared by the components (the first kappa draw of the seed)
    "sylv_1024": dict(index=5, ny=1024, nx=1024, k=4, f=9, noise="separable",
                      common_kappa=True, tol=1e-8, precision="f64"),
    # a full sky at HEALPix level 10: the 12 base faces (1024 x 1024 pixels each, links only
    # inside a face, App. A), 4 sources, 9 maps, solved as 12 independent problems in one call
    "healpix_sky_1024": dict(index=6, sizes=[1024] * 12, nrhs=1, k=4, f=9, noise="hetero",
                             boundary="face", tol=1e-8, precision="f64+mixed"),
    # repeated solves over a hyperparameter sweep (the INLA-style use named as future work in
    # the conclusion): `steps` solves with kappa_j scaled by (1 + dk)^s and tau_j by (1 - dt)^s
    "sweep_1024": dict(index=7, ny=1024, nx=1024, k=3, f=9, noise="hetero", tol=1e-8,
                       steps=10, dk=0.01, dt=0.01, precision="f64+mixed"),
}


def sweep_parameters(prob: Problem, steps: int, dk: float, dt: float):
    """(kappa, tau) of each solve of a hyperparameter sweep around the drawn values."""
    return [(prob.kappa * (1.0 + dk) ** s, prob.tau * (1.0 - dt) ** s) for s in range(steps)]


def workload(name: str, scale: Optional[int] = None) -> List[Problem]:
    """Problems of a named workload (a list: one entry, or one per grid for the batched one).

    scale, if given, replaces the grid side (used for shrunken test variants of a workload with the
    same laws); for the batched workload it divides every side by `scale`.
    """
    cfg = WORKLOADS[name]
    seed = 1000 + cfg["index"]
    if "sizes" in cfg:
        out = []
        for g, side in enumerate(cfg["sizes"]):
            s = side if scale is None else max(4, side // scale)
            out.append(make_problem(s, s, cfg["k"], cfg["f"], seed * 100 + g, noise=cfg["noise"],
                                    name=f"{name}[{g}]",
                                    boundary=cfg.get("boundary", "periodic")))
        return out
    ny = cfg["ny"] if scale is None else scale
    nx = cfg["nx"] if scale is None else scale
    kappa = None
    if cfg.get("common_kappa"):
        # make_problem's first draw, repeated for every component
        kappa = np.full(cfg["k"], np.random.default_rng(seed).uniform(0.1, 1.0, size=cfg["k"])[0])
    return [make_problem(ny, nx, cfg["k"], cfg["f"], seed, noise=cfg["noise"],
                         mask_frac=cfg.get("mask_frac", 0.0), kappa=kappa, name=name)]


def po_draws(prob: Problem, nrhs: int, seed: int):
    """Standard-normal draws for perturbation-optimisation sampling.

    Returns (xi [nrhs, k, n_pix], zeta [nrhs, f, n_pix]); xi perturbs the prior term and zeta the
    likelihood term.  The solver side turns them into a right-hand-side perturbation.
    """
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((nrhs, prob.k, prob.n_pix))
    zeta = rng.standard_normal((nrhs, prob.f, prob.n_pix))
    return xi, zeta


def random_maps(prob: Problem, seed: int, nrhs: Optional[int] = None) -> np.ndarray:
    """Standard-normal component maps [k, n_pix] (or [nrhs, k, n_pix])."""
    rng = np.random.default_rng(seed)
    shape = (prob.k, prob.n_pix) if nrhs is None else (nrhs, prob.k, prob.n_pix)
    return rng.standard_normal(shape)
