"""Seeded synthetic inputs for the multiscale kernel solver.

This module only *generates data*: point hierarchies, support radii and
target-function samples. It contains none of the method's arithmetic (no
kernel evaluation, no neighbour search, no solve), so both the CPU oracle and
the GPU path can take their inputs from here without sharing any of the
computation that is being checked.

Workloads (all synthetic; the paper's own experiments are synthetic too):

* ``grid_hierarchy``      -- nested uniform grids on [0,1]^2 (the paper's
  Section 5 setting: Table 1 grids with spacing 2^-l, mu = 1/2, nu = 4).
* ``halton_hierarchy``    -- prefix-nested 2-D Halton points (bases 2, 3).
* ``uniform3d_hierarchy`` -- prefix-nested 3-D points from a SplitMix64 stream.
* ``fourier_target``      -- a seeded sum of random Fourier modes.
* ``franke``              -- the Franke test function printed in Section 5.
* ``gauss_sine``          -- exp(-|x-c|^2/0.1) + sin(2 pi x) cos(2 pi y).

Random numbers come from a project-written SplitMix64 (Steele, Lea, Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): every draw is
a pure function of (seed, index), so any prefix of a stream is reproducible.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Hierarchy",
    "splitmix64",
    "uniform01",
    "halton",
    "grid_points",
    "grid_hierarchy",
    "table1_hierarchy",
    "halton_hierarchy",
    "uniform3d_hierarchy",
    "FourierTarget",
    "fourier_target",
    "franke",
    "gauss_sine",
    "config_hierarchy",
    "batch_hierarchies",
    "NU_2D_40",
    "NU_3D_60",
]

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# nu such that the expected number of same-level points within delta_j = nu*h_j
# of an interior point (itself included) is 40 in 2-D (pi nu^2 = 40) and 60 in
# 3-D (4/3 pi nu^3 = 60), with h_j = N_j^(-1/d) at unit density.
NU_2D_40 = math.sqrt(40.0 / math.pi)
NU_3D_60 = (45.0 / math.pi) ** (1.0 / 3.0)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of the SplitMix64 stream of ``seed``.

    Output i is mix(seed + (i+1)*golden) with the published finaliser
    z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27; z *= 0x94D049BB133111EB;
    z ^= z>>31 (all arithmetic mod 2^64).
    """
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    """53-bit doubles in [0, 1): (z >> 11) * 2^-53 of the SplitMix64 stream."""
    z = splitmix64(seed, start, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _radical_inverse(n: np.ndarray, base: int) -> np.ndarray:
    """van der Corput radical inverse of the integers ``n`` in ``base``."""
    n = n.astype(np.int64).copy()
    out = np.zeros(n.shape, dtype=np.float64)
    f = 1.0
    inv = 1.0 / base
    while np.any(n > 0):
        f *= inv
        out += f * (n % base)
        n //= base
    return out


def halton(count: int, start: int = 1) -> np.ndarray:
    """2-D Halton points with bases (2, 3) for indices start .. start+count-1.

    The default start=1 skips the origin (index 0).
    """
    n = np.arange(start, start + count, dtype=np.int64)
    return np.stack([_radical_inverse(n, 2), _radical_inverse(n, 3)], axis=1)


def grid_points(m: int) -> np.ndarray:
    """The (2^m+1)^2 points k*2^-m, k = 0..2^m, of [0,1]^2, x fastest."""
    n = (1 << m) + 1
    t = np.arange(n, dtype=np.float64) * (2.0 ** -m)  # exact binary fractions
    yy, xx = np.meshgrid(t, t, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel()], axis=1)


@dataclass
class Hierarchy:
    """A multilevel point set: level l holds ``points[offsets[l]:offsets[l+1]]``.

    ``delta[l]`` is the support radius of level l's kernel. Levels are stored
    coarse to fine. ``name`` describes the recipe.
    """

    dim: int
    points: np.ndarray  # float64 [N][dim], all levels concatenated
    offsets: np.ndarray  # int64 [L+1]
    delta: np.ndarray  # float64 [L]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def levels(self) -> int:
        return int(self.delta.shape[0])

    @property
    def n_total(self) -> int:
        return int(self.offsets[-1])

    def level_points(self, l: int) -> np.ndarray:
        return self.points[self.offsets[l]:self.offsets[l + 1]]

    def sizes(self) -> list[int]:
        return [int(self.offsets[l + 1] - self.offsets[l]) for l in range(self.levels)]


def _stack(levels: list[np.ndarray], delta, dim, name, **meta) -> Hierarchy:
    offs = np.zeros(len(levels) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(p) for p in levels])
    pts = np.ascontiguousarray(np.concatenate(levels, axis=0), dtype=np.float64)
    return Hierarchy(dim, pts, offs, np.asarray(delta, dtype=np.float64), name, meta)


def grid_hierarchy(levels: int = 4, first_exponent: int = 3, nu_spacing: float = 4.0) -> Hierarchy:
    """Nested grids with spacing s_j = 2^-(first_exponent + j), delta_j = nu*s_j.

    Default: 4 levels with spacing 1/8 .. 1/64 (81, 289, 1089, 4225 points)
    and delta = 4 * spacing, so exact ties at distance delta do occur.
    """
    pts, dl = [], []
    for j in range(levels):
        m = first_exponent + j
        pts.append(grid_points(m))
        dl.append(nu_spacing * (2.0 ** -m))
    return _stack(pts, dl, 2, f"grid{levels}", spacing_exp0=first_exponent)


def table1_hierarchy(levels: int, nu: float = 4.0) -> Hierarchy:
    """The paper's Table 1 grids: spacing 2^-l for l = 1..L.

    The fill distance of the grid with spacing s is s/sqrt(2) and the support
    radius is delta_l = nu * fill distance (Assumption 2, nu = 4).
    """
    pts, dl = [], []
    for l in range(1, levels + 1):
        pts.append(grid_points(l))
        dl.append(nu * (2.0 ** -l) / math.sqrt(2.0))
    return _stack(pts, dl, 2, f"table1_L{levels}")


def halton_hierarchy(levels: int = 8, n0: int = 64, ratio: int = 4, nu: float = NU_2D_40,
                     start: int = 1, sizes: list[int] | None = None) -> Hierarchy:
    """Prefix-nested 2-D Halton hierarchy: level j = first n0*ratio^j points.

    h_j = N_j^(-1/2) and delta_j = nu * h_j. ``sizes`` overrides the level
    sizes (still prefixes of one Halton run starting at index ``start``).
    """
    if sizes is None:
        sizes = [n0 * ratio ** j for j in range(levels)]
    top = halton(max(sizes), start=start)
    pts = [top[:n] for n in sizes]
    dl = [nu * n ** -0.5 for n in sizes]
    return _stack(pts, dl, 2, f"halton_L{len(sizes)}", start=start, sizes=list(sizes))


def uniform3d_hierarchy(levels: int = 5, n0: int = 512, ratio: int = 8, nu: float = NU_3D_60,
                        seed: int = 2000) -> Hierarchy:
    """Prefix-nested 3-D hierarchy from one seeded uniform stream on [0,1)^3.

    Point i takes stream outputs 3i, 3i+1, 3i+2 as (x, y, z). Level j holds the
    first n0*ratio^j points; h_j = N_j^(-1/3), delta_j = nu * h_j.
    """
    sizes = [n0 * ratio ** j for j in range(levels)]
    top = uniform01(seed, 0, 3 * max(sizes)).reshape(-1, 3)
    pts = [top[:n] for n in sizes]
    dl = [nu * n ** (-1.0 / 3.0) for n in sizes]
    return _stack(pts, dl, 3, f"uniform3d_L{levels}", seed=seed)


@dataclass
class FourierTarget:
    """f(x) = sum_m c_m cos(2 pi k_m . x + theta_m)."""

    k: np.ndarray  # int [M][d]
    c: np.ndarray  # float64 [M]
    theta: np.ndarray  # float64 [M]

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.asarray(x, dtype=np.float64)
        out = np.zeros(x.shape[0], dtype=np.float64)
        for km, cm, tm in zip(self.k, self.c, self.theta):
            out += cm * np.cos(2.0 * math.pi * (x @ km.astype(np.float64)) + tm)
        return out

    def torch_eval(self, x):
        """Same sum evaluated with torch ops (for large device-resident batches)."""
        import torch

        k = torch.as_tensor(self.k, dtype=torch.float64, device=x.device)
        c = torch.as_tensor(self.c, dtype=torch.float64, device=x.device)
        th = torch.as_tensor(self.theta, dtype=torch.float64, device=x.device)
        ph = 2.0 * math.pi * (x.to(torch.float64) @ k.T) + th
        return torch.cos(ph) @ c


def fourier_target(seed: int, dim: int = 2, modes: int = 32, kmax: float = 8.0) -> FourierTarget:
    """Seeded random Fourier target.

    k_m is uniform over the nonzero integer vectors with |k| <= kmax (listed in
    lexicographic order), c_m = g_m / |k_m|^2 with g_m standard normal
    (Box-Muller), theta_m uniform in [0, 2 pi).
    """
    r = int(math.floor(kmax))
    axes = [np.arange(-r, r + 1)] * dim
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, dim)
    n2 = (grid ** 2).sum(axis=1)
    cand = grid[(n2 > 0) & (n2 <= kmax * kmax)]
    u = uniform01(seed, 0, 4 * modes).reshape(modes, 4)
    idx = np.minimum((u[:, 0] * len(cand)).astype(np.int64), len(cand) - 1)
    k = cand[idx]
    u1 = np.maximum(u[:, 1], 2.0 ** -53)
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u[:, 2])
    c = g / (k ** 2).sum(axis=1).astype(np.float64)
    theta = 2.0 * math.pi * u[:, 3]
    return FourierTarget(k, c, theta)


def franke(x: np.ndarray) -> np.ndarray:
    """The Franke function as printed in Section 5 (eq. Franke)."""
    X, Y = x[:, 0], x[:, 1]
    return (0.75 * np.exp(-((9 * X - 2) ** 2 + (9 * Y - 2) ** 2) / 4.0)
            + 0.75 * np.exp(-((9 * X + 1) ** 2) / 49.0 - (9 * Y + 1) / 10.0)
            + 0.5 * np.exp(-((9 * X - 7) ** 2 + (9 * Y - 3) ** 2) / 4.0)
            - 0.2 * np.exp(-(9 * X - 4) ** 2 - (9 * Y - 7) ** 2))


def gauss_sine(x: np.ndarray) -> np.ndarray:
    """exp(-((x-1/2)^2+(y-1/2)^2)/0.1) + sin(2 pi x) cos(2 pi y)."""
    X, Y = x[:, 0], x[:, 1]
    return (np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.1)
            + np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y))


def batch_hierarchies(count: int = 64, seed: int = 4000, n_min: int = 10_000, n_max: int = 200_000,
                      levels_choice=(5, 6, 7)) -> list[tuple[Hierarchy, np.ndarray]]:
    """Independent 2-D Halton hierarchies of uneven sizes.

    Hierarchy h starts its Halton run at index 1 + 10^6 h, has L_h levels drawn
    from ``levels_choice`` and a top level of N_top,h points drawn uniformly
    in [n_min, n_max]; level l holds ceil(N_top,h * 4^(l - L_h + 1)) points
    (prefix-nested), delta_l = sqrt(40/pi) * N_l^(-1/2). Its target is the
    32-mode Fourier sum with seed ``seed + h``. Draws use SplitMix64(seed).
    """
    u = uniform01(seed, 0, 2 * count).reshape(count, 2)
    out = []
    for h in range(count):
        L = int(levels_choice[min(int(u[h, 0] * len(levels_choice)), len(levels_choice) - 1)])
        ntop = int(n_min + math.floor(u[h, 1] * (n_max - n_min + 1)))
        sizes = [int(math.ceil(ntop * 4.0 ** (l - L + 1))) for l in range(L)]
        hh = halton_hierarchy(sizes=sizes, start=1 + 1_000_000 * h)
        out.append((hh, fourier_target(seed + h, 2)(hh.points)))
    return out


def config_hierarchy(name: str, levels: int | None = None) -> tuple[Hierarchy, np.ndarray]:
    """Named workloads -> (hierarchy, target samples f on all points).

    ``grid4``     4 nested grids (81..4225 points), delta = 4*spacing, gauss_sine.
    ``halton``    2-D Halton, 64*4^j points (default 8 levels, 1,398,080 points),
                  nu = sqrt(40/pi), 32-mode Fourier target seed 1000.
    ``uniform3d`` 3-D uniform stream seed 2000, 512*8^j points (default 5 levels,
                  2,396,672 points), nu = (45/pi)^(1/3), Fourier target seed 2001.
    ``table1``    the paper's Table 1 grids (default 7 levels), Franke target.
    """
    if name == "grid4":
        h = grid_hierarchy(levels or 4)
        return h, gauss_sine(h.points)
    if name == "halton":
        h = halton_hierarchy(levels or 8)
        return h, fourier_target(1000, 2)(h.points)
    if name == "uniform3d":
        h = uniform3d_hierarchy(levels or 5)
        return h, fourier_target(2001, 3)(h.points)
    if name == "table1":
        h = table1_hierarchy(levels or 7)
        return h, franke(h.points)
    raise ValueError(f"unknown workload {name!r}")
