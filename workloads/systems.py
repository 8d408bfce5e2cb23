"""Seeded synthetic particle systems.

The paper's own systems (an equilibrated 1000-water GROMACS box replicated
27 times, a cloud-wall system and an isolated cloud; sections 7-9) are not
available, so these generators stand in for them with the same kind of
structure: uniform random ions with +/-1 charges, and a 3-site water model
with SPC/E-like charges (-0.8476 on O, +0.4238 on H, section 8.1) at liquid
density, O sites placed by random sequential addition with a 2.5 A O-O
exclusion and molecules given uniform random orientations.

All randomness comes from ``numpy.random.default_rng(seed)`` (PCG64) and all
positions are generated in float64 and wrapped into [0, L).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

Q_O = -0.8476
Q_H = 0.4238
OH_BOND = 1.0               # Angstrom
HOH_ANGLE = 109.47          # degrees
WATER_DENSITY = 0.0334      # molecules per cubic Angstrom
OO_MIN = 2.5                # Angstrom, random-sequential-addition exclusion


def ions(N: int, L: float, seed: int):
    """N ions uniform in [0, L)^3; the first N//2 carry +1, the rest -1
    (N odd leaves one extra -1, i.e. a net charge of -1)."""
    rng = np.random.default_rng(seed)
    x = rng.random((N, 3)) * L
    q = np.empty(N)
    q[: N // 2] = 1.0
    q[N // 2:] = -1.0
    return x, q


def _random_rotations(rng, n):
    """n uniform random rotation matrices (normalised 4D Gaussian quaternions)."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, a, b, c = qv.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (b * b + c * c)
    R[:, 0, 1] = 2 * (a * b - c * w)
    R[:, 0, 2] = 2 * (a * c + b * w)
    R[:, 1, 0] = 2 * (a * b + c * w)
    R[:, 1, 1] = 1 - 2 * (a * a + c * c)
    R[:, 1, 2] = 2 * (b * c - a * w)
    R[:, 2, 0] = 2 * (a * c - b * w)
    R[:, 2, 1] = 2 * (b * c + a * w)
    R[:, 2, 2] = 1 - 2 * (a * a + b * b)
    return R


def _rsa_sites(rng, n: int, L: float, dmin: float):
    """Random sequential addition of n points in a periodic cube with minimum
    periodic distance dmin, done in batches: each batch of uniform proposals
    is tested against the accepted points (through a cell grid with cells of
    side >= dmin, at most ``cap`` points per cell) and against the earlier
    proposals of the same batch; a proposal that fails either test is
    dropped."""
    nc = max(3, int(math.floor(L / dmin)))
    cs = L / nc
    cap = 8
    grid = np.full((nc, nc, nc, cap, 3), np.nan)
    fill = np.zeros((nc, nc, nc), dtype=np.int64)
    pts = np.empty((n, 3))
    count = 0
    d2 = dmin * dmin
    off = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1)
                    for k in (-1, 0, 1)])
    rounds = 0
    while count < n:
        rounds += 1
        if rounds > 100000:
            raise RuntimeError("random sequential addition did not converge")
        B = int(min(4096, max(64, 2 * (n - count))))
        cand = rng.random((B, 3)) * L
        ci = np.minimum((cand / cs).astype(np.int64), nc - 1)
        nb = (ci[:, None, :] + off[None, :, :]) % nc            # B,27,3
        neigh = grid[nb[..., 0], nb[..., 1], nb[..., 2]]       # B,27,cap,3
        dd = neigh - cand[:, None, None, :]
        dd -= L * np.round(dd / L)
        r2 = np.einsum("bkcd,bkcd->bkc", dd, dd)
        ok = ~np.any(r2 < d2, axis=(1, 2))                     # nan compares False
        idx = np.nonzero(ok)[0]
        if idx.size:
            c = cand[idx]
            dd = c[:, None, :] - c[None, :, :]
            dd -= L * np.round(dd / L)
            r2 = np.einsum("ijd,ijd->ij", dd, dd)
            clash = np.triu(r2 < d2, k=1)
            keep = ~np.any(clash, axis=0)                      # no earlier clash
            idx = idx[keep]
        idx = idx[: n - count]
        for b in idx:
            cx, cy, cz = ci[b]
            k = fill[cx, cy, cz]
            if k >= cap:
                continue
            grid[cx, cy, cz, k] = cand[b]
            fill[cx, cy, cz] = k + 1
            pts[count] = cand[b]
            count += 1
    return pts


def water(L: float, seed: int, density: float = WATER_DENSITY):
    """Rigid 3-site water at ``density`` molecules/A^3 in a periodic cube of
    side L.  Returns (x[3n,3], q[3n]) ordered O, H, H per molecule (neutral)."""
    rng = np.random.default_rng(seed)
    nmol = int(math.floor(density * L ** 3))
    O = _rsa_sites(rng, nmol, L, OO_MIN)
    half = math.radians(HOH_ANGLE) / 2.0
    body = np.array([[math.sin(half), 0.0, math.cos(half)],
                     [-math.sin(half), 0.0, math.cos(half)]]) * OH_BOND
    R = _random_rotations(rng, nmol)
    H = O[:, None, :] + np.einsum("nij,kj->nki", R, body)
    x = np.empty((nmol, 3, 3))
    x[:, 0] = O
    x[:, 1:] = H
    x = np.mod(x.reshape(-1, 3), L)
    x[x >= L] = 0.0  # mod can round up to L for tiny negative inputs
    q = np.tile([Q_O, Q_H, Q_H], nmol)
    return x, q


def nacl_lattice(ncell: int, a: float = 1.0):
    """Rock-salt crystal: ncell^3 conventional cells, nearest-neighbour
    distance a, box L = 2 a ncell, N = 8 ncell^3 ions, charge (-1)^(i+j+k)."""
    n = 2 * ncell
    idx = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n),
                               indexing="ij"), -1).reshape(-1, 3)
    x = idx.astype(np.float64) * a
    q = np.where(idx.sum(1) % 2 == 0, 1.0, -1.0)
    return x, q, float(n * a)


@dataclass(frozen=True)
class SystemSpec:
    """A named workload: system recipe plus SE parameters."""
    name: str
    kind: str           # "ions" or "water"
    N: int              # requested atoms (ions) or resulting atoms (water)
    L: float
    xi: float
    M: int
    P: tuple = field(default=(8,))
    seed: int = 0

    def generate(self):
        if self.kind == "ions":
            return ions(self.N, self.L, self.seed)
        if self.kind == "water":
            return water(self.L, self.seed)
        raise ValueError(self.kind)


# The five workloads: small ionic case, three water boxes, one large ionic box.
CONFIGS = {
    "ions_1k": SystemSpec("ions_1k", "ions", 1000, 10.0, 1.5, 32, (8,), 1001),
    "water_L40": SystemSpec("water_L40", "water", 6411, 40.0, 0.3, 40, (6, 10), 1002),
    "water_L60": SystemSpec("water_L60", "water", 21642, 60.0, 0.3, 64, (8,), 1003),
    "water_L100": SystemSpec("water_L100", "water", 100200, 100.0, 0.3, 96, (6, 8, 12), 1004),
    "ions_1M": SystemSpec("ions_1M", "ions", 1000000, 220.0, 0.35, 192, (8,), 1005),
}


def make_system(name: str):
    """(x, q, spec) for a named workload."""
    spec = CONFIGS[name]
    x, q = spec.generate()
    return x, q, spec
