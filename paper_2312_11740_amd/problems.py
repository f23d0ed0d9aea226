"""Seeded synthetic inputs for the pressure-projection solve.

This module only draws inputs: level-set fields of spherical bubbles, density pairs,
surface-tension coefficients and right-hand sides.  It holds none of the solver's
arithmetic (no face coefficients, curvature, jump term or solve), so the GPU path and
the CPU oracle can both take their inputs from it.

The paper's workloads (flow boiling, impinging jet; Sec. 2) and their data are not
available; these bubble fields stand in for them at the paper's gas/liquid density
ratio of 1e-3 (Sec. 4, Fig. 13).  Fields are float64 arrays of shape (n, n, n)
indexed [k, j, i], so that x is the fastest-varying index in memory, with cell
centres at ((i+1/2)/n, (j+1/2)/n, (k+1/2)/n) on the unit cube.

The level set is phi(x) = min_b (|x - c_b| - r_b): negative inside the bubbles,
positive outside.  The "-" side (phi <= 0) carries rho_neg, the "+" side rho_pos.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "cell_centres",
    "bubble_phi",
    "draw_bubbles",
    "single_bubble_problem",
    "many_bubbles_problem",
    "random_bubbles_problem",
    "rising_bubble_problem",
    "refine_near_interface",
    "CONFIGS",
]


@dataclass
class Problem:
    """One projection problem: phi and f on an n^3 grid plus the phase constants."""

    n: int
    phi: np.ndarray          # (n, n, n) float64, [k, j, i]
    f: np.ndarray            # (n, n, n) float64
    rho_neg: float           # density where phi <= 0 (inside bubbles)
    rho_pos: float           # density where phi > 0
    sigma: float             # surface-tension coefficient
    centres: list = field(default_factory=list)
    radii: list = field(default_factory=list)
    seed: int | None = None


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def bubble_phi(n: int, centres, radii) -> np.ndarray:
    """phi = min over bubbles of (distance to centre - radius), shape (n, n, n) [k, j, i]."""
    x = cell_centres(n)
    X = x[None, None, :]
    Y = x[None, :, None]
    Z = x[:, None, None]
    phi = np.full((n, n, n), np.inf)
    for (cx, cy, cz), r in zip(centres, radii):
        d = np.sqrt((X - cx) ** 2 + (Y - cy) ** 2 + (Z - cz) ** 2) - r
        np.minimum(phi, d, out=phi)
    return phi


def _fits(c, r, centres, radii, h, cmin, cmax):
    c = np.asarray(c)
    # keep every bubble at least 2h inside the walls and 4h away from every other one,
    # so that the curvature stencil never sees a wall or the kink between two bubbles
    if np.any(c - r < 2 * h) or np.any(c + r > 1 - 2 * h):
        return False
    for c2, r2 in zip(centres, radii):
        if np.linalg.norm(c - np.asarray(c2)) - r - r2 < 4 * h:
            return False
    return True


def draw_bubbles(rng: np.random.Generator, count: int, rmin: float, rmax: float,
                 cmin: float, cmax: float, n: int, max_tries: int = 100000):
    """Draw `count` non-overlapping bubbles, each as (cx, cy, cz, r), by rejection."""
    h = 1.0 / n
    centres, radii = [], []
    tries = 0
    while len(centres) < count:
        cx, cy, cz = rng.uniform(cmin, cmax, size=3)
        r = rng.uniform(rmin, rmax)
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d bubbles" % count)
        if _fits((cx, cy, cz), r, centres, radii, h, cmin, cmax):
            centres.append((float(cx), float(cy), float(cz)))
            radii.append(float(r))
    return centres, radii


def single_bubble_problem(n: int = 32) -> Problem:
    """One sphere of radius 0.25 at the centre, rho = 1 inside and 10 outside, no surface
    tension; f is the cell value of div((1/rho) grad p*) within each phase for the
    manufactured p* = cos(pi x) cos(pi y) cos(pi z), i.e. -3 pi^2 p* / rho, made
    zero-mean."""
    x = cell_centres(n)
    phi = bubble_phi(n, [(0.5, 0.5, 0.5)], [0.25])
    pstar = (np.cos(np.pi * x)[None, None, :] * np.cos(np.pi * x)[None, :, None]
             * np.cos(np.pi * x)[:, None, None])
    rho_neg, rho_pos = 1.0, 10.0
    rho = np.where(phi > 0.0, rho_pos, rho_neg)
    f = -3.0 * np.pi ** 2 * pstar / rho
    f -= f.mean()
    return Problem(n, phi, f, rho_neg, rho_pos, 0.0, [(0.5, 0.5, 0.5)], [0.25])


def _uniform_rhs(rng: np.random.Generator, n: int) -> np.ndarray:
    f = rng.uniform(-1.0, 1.0, size=(n, n, n))
    f -= f.mean()
    return f


def many_bubbles_problem(n: int = 128, count: int = 20, seed: int = 1, ratio: float = 1000.0,
                         sigma: float = 0.01) -> Problem:
    """`count` bubbles, centres uniform in [0.15, 0.85]^3, radii uniform in [0.04, 0.12];
    liquid density 1 outside, gas density 1/ratio inside; f uniform in [-1, 1],
    zero-mean."""
    rng = np.random.default_rng(seed)
    centres, radii = draw_bubbles(rng, count, 0.04, 0.12, 0.15, 0.85, n)
    phi = bubble_phi(n, centres, radii)
    f = _uniform_rhs(rng, n)
    return Problem(n, phi, f, 1.0 / ratio, 1.0, sigma, centres, radii, seed)


def random_bubbles_problem(seed: int, n: int = 64, sigma: float = 0.01) -> Problem:
    """Batched/learned workload: count uniform in {1..8}, radii uniform in [0.05, 0.15],
    centres uniform in [0.15, 0.85]^3, density ratio log-uniform in [10, 1000]."""
    rng = np.random.default_rng(seed)
    count = int(rng.integers(1, 9))
    centres, radii = draw_bubbles(rng, count, 0.05, 0.15, 0.15, 0.85, n)
    ratio = 10.0 ** rng.uniform(1.0, 3.0)
    phi = bubble_phi(n, centres, radii)
    f = _uniform_rhs(rng, n)
    return Problem(n, phi, f, 1.0 / ratio, 1.0, sigma, centres, radii, seed)


def rising_bubble_problem(t: int, n: int = 256, sigma: float = 0.01,
                          ratio: float = 1000.0) -> Problem:
    """Step t of the rising-bubble sequence: radius 0.1 at (0.5, 0.5, 0.2 + 0.004 t),
    density ratio 1000, f uniform in [-1, 1] drawn with seed 40000 + t."""
    rng = np.random.default_rng(40000 + t)
    c = (0.5, 0.5, 0.2 + 0.004 * t)
    phi = bubble_phi(n, [c], [0.1])
    f = _uniform_rhs(rng, n)
    return Problem(n, phi, f, 1.0 / ratio, 1.0, sigma, [c], [0.1], 40000 + t)


CONFIGS = {
    "single_bubble_32": dict(n=32, rho_ratio=10.0, sigma=0.0, rtol=1e-10),
    "bubbles20_128": dict(n=128, rho_ratio=1000.0, sigma=0.01, rtol=1e-10),
    "batched_64x64": dict(n=64, batch=64, seeds=(20000, 20064), sigma=0.01, rtol=1e-10),
    "learned_64": dict(n=64, train=(0, 4000), held_out=(10000, 10500), sigma=0.01),
    "rising_bubble_256": dict(n=256, steps=100, rho_ratio=1000.0, sigma=0.01, rtol=1e-10),
}


def refine_near_interface(phi0: np.ndarray, nb: int, band: float) -> np.ndarray:
    """Refinement flags of the blocks of nb^3 cells of phi0 ((n, n, n), [k, j, i]): 1 where
    some cell centre of the block lies within `band` of the interface (|phi| < band), the
    refinement around phi = 0 of Fig. 2.  Returns uint8 of shape (n/nb,)*3, [bk, bj, bi]."""
    n = phi0.shape[0]
    m = n // nb
    near = np.abs(phi0) < band
    return near.reshape(m, nb, m, nb, m, nb).any(axis=(1, 3, 5)).astype(np.uint8)


def to_grid(a) -> np.ndarray:
    """Contiguous float64 copy in [k, j, i] layout."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def sphere_volume_fraction(r: float) -> float:  # used by tests of the generator
    return 4.0 / 3.0 * math.pi * r ** 3
