"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module only produces initial fields (density, velocity, or raw
population arrays) and run parameters.  It contains none of the method's
arithmetic (no quasiequilibrium, collision, entropy or limiter): each side
(the GPU library and the CPU oracle) builds its own f* from the fields here.

Randomness comes from splitmix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), implemented below from its
published definition so that streams are reproducible on any machine.

Workloads follow the paper's test problems (Sec. 4.3 shock tube, Sec. 4.4
lid-driven cavity) and the periodic flows used for the large-grid runs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEFAULT_SEED = 0x07040043
_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, count: int) -> np.ndarray:
    """`count` successive splitmix64 outputs (uint64) starting from `seed`."""
    with np.errstate(over="ignore"):
        idx = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & _MASK64) + idx * np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, count: int) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of splitmix64."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def beta_from_nu(nu: float) -> float:
    """Over-relaxation parameter for kinematic viscosity nu (lattice units).

    The lattices have c_s^2 = 1/3 and the LBGK viscosity is
    nu = c_s^2 (1/(2 beta) - 1/2), hence beta = 1/(6 nu + 1)."""
    return 1.0 / (6.0 * nu + 1.0)


def nu_from_beta(beta: float) -> float:
    return (1.0 / (2.0 * beta) - 0.5) / 3.0


# ---- raw population fields (parity tests) ----------------------------------

# shape of a rest state used to give random populations realistic magnitudes
_SHAPE = {3: np.array([2 / 3, 1 / 6, 1 / 6]),
          9: np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)}


def random_populations(q: int, nx: int, ny: int, seed: int = DEFAULT_SEED, rho0: float = 1.0,
                       amp: float = 0.05, spike_frac: float = 0.02, spike_amp: float = 0.4,
                       negative_frac: float = 0.0) -> np.ndarray:
    """Positive populations f[i, y, x] = rho0 * shape_i * (1 + noise).

    `amp` sets the bulk relative perturbation; a fraction `spike_frac` of the
    sites gets `spike_amp` instead (strongly nonequilibrium sites that the
    limiters act on); `negative_frac` of the sites get one negative entry."""
    n = nx * ny
    r = uniform(seed, q * n + 2 * n).reshape(-1)
    noise = (2.0 * r[: q * n].reshape(q, ny, nx) - 1.0)
    spikes = (r[q * n: q * n + n] < spike_frac).reshape(ny, nx)
    scale = np.where(spikes, spike_amp, amp)
    f = rho0 * _SHAPE[q][:, None, None] * (1.0 + scale[None] * noise)
    if negative_frac > 0:
        neg = (r[q * n + n:] < negative_frac).reshape(ny, nx)
        f[q - 1][neg] = -0.01 * rho0 * _SHAPE[q][q - 1]
    return np.ascontiguousarray(f)


def random_flow(nx: int, ny: int, seed: int = DEFAULT_SEED, rho0: float = 1.0, drho: float = 0.02,
                umax: float = 0.05, dim: int = 2):
    """Random density and velocity fields (rho [ny, nx], u [dim, ny, nx])."""
    n = nx * ny
    r = uniform(seed ^ 0x5A5A, (1 + dim) * n).reshape(1 + dim, ny, nx)
    rho = rho0 * (1.0 + drho * (2 * r[0] - 1))
    u = umax * (2 * r[1:] - 1)
    return rho, np.ascontiguousarray(u)


# ---- physical workloads -----------------------------------------------------

def shock_tube(nx: int = 800, split: int = 400, rho_left: float = 1.0, rho_right: float = 0.5):
    """1:2 athermal shock tube (Sec. 4.3): rho_left for x < split, u = 0."""
    rho = np.where(np.arange(nx) < split, rho_left, rho_right).astype(np.float64)[None, :]
    u = np.zeros((1, 1, nx))
    return rho, u


def cavity_rest(nx: int, ny: int | None = None, rho0: float = 2.7):
    """Fluid at rest with uniform density (Sec. 4.4.1)."""
    ny = nx if ny is None else ny
    return np.full((ny, nx), rho0), np.zeros((2, ny, nx))


def taylor_green(n: int, u0: float = 0.05, mode: int = 1, rho0: float = 1.0, perturb: float = 1e-3,
                 seed: int = DEFAULT_SEED, ny: int | None = None):
    """Taylor-Green vortex plus a seeded random-phase divergence-free perturbation.

    u = U0 (sin kx cos ky, -cos kx sin ky), k = 2 pi mode / n, with the
    pressure term rho = rho0 - (3 rho0 U0^2 / 4)(cos 2kx + cos 2ky).  The
    perturbation is u' = curl(psi'), psi' = sum_{1 <= |m|_inf <= 4}
    cos(2 pi (mx x + my y)/n + theta_m), theta from splitmix64, scaled to
    max |u'| = perturb."""
    ny = n if ny is None else ny
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    kx, ky = 2 * math.pi * mode / n, 2 * math.pi * mode / ny
    ux = u0 * np.sin(kx * x) * np.cos(ky * y)
    uy = -u0 * np.cos(kx * x) * np.sin(ky * y)
    rho = rho0 - 0.75 * rho0 * u0 * u0 * (np.cos(2 * kx * x) + np.cos(2 * ky * y))
    if perturb > 0:
        modes = [(mx, my) for mx in range(-4, 5) for my in range(-4, 5) if max(abs(mx), abs(my)) >= 1]
        theta = 2 * math.pi * uniform(seed, len(modes))
        px = np.zeros((ny, n))
        py = np.zeros((ny, n))
        for (mx, my), th in zip(modes, theta):
            arg = 2 * math.pi * (mx * x / n + my * y / ny) + th
            s = -np.sin(arg)
            # u' = d psi/dy, v' = -d psi/dx
            px += s * (2 * math.pi * my / ny)
            py -= s * (2 * math.pi * mx / n)
        scale = perturb / max(np.sqrt(px * px + py * py).max(), 1e-300)
        ux = ux + scale * px
        uy = uy + scale * py
    rho = np.broadcast_to(rho, (ny, n)).copy()
    return rho, np.ascontiguousarray(np.stack([ux, uy]))


def double_shear_layer(n: int, u0: float = 0.05, kappa: float = 80.0, eps: float = 0.05, rho0: float = 1.0):
    """Periodic double shear layer: u_x = U0 tanh(kappa (y/n - 1/4)) for y <= n/2,
    U0 tanh(kappa (3/4 - y/n)) above; u_y = eps U0 sin(2 pi (x/n + 1/4))."""
    x = np.arange(n, dtype=np.float64)[None, :]
    y = np.arange(n, dtype=np.float64)[:, None]
    yn = y / n
    ux = np.where(y <= n / 2, u0 * np.tanh(kappa * (yn - 0.25)), u0 * np.tanh(kappa * (0.75 - yn)))
    uy = eps * u0 * np.sin(2 * math.pi * (x / n + 0.25))
    ux = np.broadcast_to(ux, (n, n))
    uy = np.broadcast_to(uy, (n, n))
    return np.full((n, n), rho0), np.ascontiguousarray(np.stack([ux, uy]))


@dataclass
class CavitySpec:
    n: int
    re: float
    nu: float
    beta: float
    probe: tuple


@dataclass
class CavityBatch:
    specs: list = field(default_factory=list)

    @property
    def sites(self) -> int:
        return sum(s.n * s.n for s in self.specs)


def cavity_batch(count: int = 256, sizes=(64, 100, 128, 192, 256), re_range=(2000.0, 7500.0),
                 u0: float = 0.1, seed: int = DEFAULT_SEED) -> CavityBatch:
    """Ensemble of lid-driven cavities: N from `sizes`, Re uniform in `re_range`,
    nu = u0 N / Re; probe at the node nearest (N/16, 13N/16) (Sec. 4.4.2)."""
    r = uniform(seed ^ 0xCA71, 2 * count).reshape(count, 2)
    specs = []
    for k in range(count):
        n = int(sizes[min(int(r[k, 0] * len(sizes)), len(sizes) - 1)])
        re = re_range[0] + (re_range[1] - re_range[0]) * r[k, 1]
        nu = u0 * n / re
        probe = (int(round((n - 1) / 16)), int(round(13 * (n - 1) / 16)))
        specs.append(CavitySpec(n=n, re=re, nu=nu, beta=beta_from_nu(nu), probe=probe))
    return CavityBatch(specs)
