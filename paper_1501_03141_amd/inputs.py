"""Seeded synthetic workloads for the PDEP chi0 path.

This module only draws random numbers and evaluates the synthetic potential on the
grid.  It contains none of the method's arithmetic (no plane-wave sphere, no
transforms, no solves): the trial block generator receives the Miller list from the
caller.  Both the CPU oracle side and the HIP side consume exactly the arrays built
here, so the arrays are the definition of each workload.

Workloads stand in for the paper's systems (molecules, solids, interfaces at the
Gamma point, N_pdep of the same order as the number of occupied bands; Sec. 3, 4):

* ``tiny``       10^3 bohr, 16^3 grid, 5 Ha, 4 wells, N_v=4,   N_pdep=8
* ``small``      15^3 bohr, 32^3 grid, 10 Ha, 16 wells, N_v=32, N_pdep=64
* ``medium``     20^3 bohr, 48^3 grid, 12 Ha, 64 wells, N_v=128, N_pdep=128
* ``interface``  20x20x40 bohr, 48x48x96 grid, 12 Ha, two slabs of wells,
                 N_v=512, N_pdep=256
* serving stream: jobs on 24^3/32^3/48^3 grids, N_v in 8..128, N_pdep in 16..64.

Potential (Hartree): V(r) = -sum_a A_a sum_{m in {-1,0,1}^3}
exp(-|r - R_a - L*m|^2 / (2 w_a^2)), with per-well draw order (R_a, A_a, w_a).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    L: tuple            # cell lengths (bohr), orthorhombic
    n: tuple            # FFT grid
    ecut: float         # wavefunction cutoff (Ha): 1/2 |G|^2 <= ecut
    n_wells: int
    n_v: int
    n_pdep: int
    cg_tol: float       # final relative Sternheimer residual
    seed: int
    depth: tuple = (1.0, 3.0)
    width: tuple = (0.8, 1.5)
    slabs: Optional[tuple] = None   # ((count, zlo, zhi, dlo, dhi), ...)

    @property
    def volume(self) -> float:
        return float(self.L[0] * self.L[1] * self.L[2])

    @property
    def n_grid(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])


WORKLOADS = {
    "tiny": Workload("tiny", (10.0, 10.0, 10.0), (16, 16, 16), 5.0, 4, 4, 8, 1e-12, 1502),
    "small": Workload("small", (15.0, 15.0, 15.0), (32, 32, 32), 10.0, 16, 32, 64, 1e-10, 1503),
    "medium": Workload("medium", (20.0, 20.0, 20.0), (48, 48, 48), 12.0, 64, 128, 128, 1e-8, 1504),
    "interface": Workload("interface", (20.0, 20.0, 40.0), (48, 48, 96), 12.0, 224, 512, 256, 1e-8,
                          1505, slabs=((128, 0.0, 20.0, 3.0, 5.0), (96, 20.0, 40.0, 0.5, 1.5))),
}


def with_seed(w: Workload, seed: int) -> Workload:
    return dataclasses.replace(w, seed=int(seed))


def draw_wells(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Well parameters, one row (Rx, Ry, Rz, A, width) per Gaussian."""
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    rows = []
    if w.slabs is None:
        for _ in range(w.n_wells):
            R = [rng.uniform(0.0, w.L[d]) for d in range(3)]
            A = rng.uniform(*w.depth)
            s = rng.uniform(*w.width)
            rows.append(R + [A, s])
    else:
        for (count, zlo, zhi, dlo, dhi) in w.slabs:
            for _ in range(count):
                R = [rng.uniform(0.0, w.L[0]), rng.uniform(0.0, w.L[1]), rng.uniform(zlo, zhi)]
                A = rng.uniform(dlo, dhi)
                s = rng.uniform(*w.width)
                rows.append(R + [A, s])
    return np.asarray(rows, dtype=np.float64).reshape(-1, 5)


def well_potential(L: Sequence[float], n: Sequence[int], wells: np.ndarray) -> np.ndarray:
    """Sum of periodic-imaged attractive Gaussians on the grid r = (i L / n), C order."""
    L = [float(x) for x in L]
    n = [int(x) for x in n]
    axes = [np.arange(n[d]) * (L[d] / n[d]) for d in range(3)]
    V = np.zeros(n, dtype=np.float64)
    for (Rx, Ry, Rz, A, s) in wells:
        inv2s2 = 1.0 / (2.0 * s * s)
        # separable: exp(-(dx^2+dy^2+dz^2)/(2s^2)) summed over the 27 images
        f = []
        for d, R in enumerate((Rx, Ry, Rz)):
            acc = np.zeros(n[d])
            for m in (-1, 0, 1):
                dd = axes[d] - R - L[d] * m
                acc += np.exp(-dd * dd * inv2s2)
            f.append(acc)
        V -= A * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    return V


def vloc(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    return well_potential(w.L, w.n, draw_wells(w, seed))


def canonical_half(miller: np.ndarray) -> np.ndarray:
    """Boolean mask of the canonical half of the nonzero Miller indices:
    mx > 0, or mx == 0 and my > 0, or mx == my == 0 and mz > 0."""
    m = np.asarray(miller)
    mx, my, mz = m[:, 0], m[:, 1], m[:, 2]
    return (mx > 0) | ((mx == 0) & (my > 0)) | ((mx == 0) & (my == 0) & (mz > 0))


def trial_block(miller: np.ndarray, n_pert: int, seed: int) -> np.ndarray:
    """Random-normal trial potentials on the given (G != 0) Miller list.

    For G in the canonical half, phi(G) = (a + i b)/sqrt(2), a, b ~ N(0, 1) drawn in
    list order (perturbation outer); phi(-G) = conj(phi(G)), so each potential is real
    in r.  Returns complex128 [n_pert, len(miller)].  The list must be closed under
    G -> -G and must not contain G = 0.
    """
    m = np.asarray(miller, dtype=np.int64)
    if np.any(np.all(m == 0, axis=1)):
        raise ValueError("trial_block: Miller list must exclude G = 0")
    half = canonical_half(m)
    idx = {tuple(r): k for k, r in enumerate(m.tolist())}
    neg = np.array([idx[(-a, -b, -c)] for (a, b, c) in m.tolist()], dtype=np.int64)
    hpos = np.nonzero(half)[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    ab = rng.standard_normal((n_pert, hpos.size, 2))
    vals = (ab[..., 0] + 1j * ab[..., 1]) / math.sqrt(2.0)
    phi = np.zeros((n_pert, m.shape[0]), dtype=np.complex128)
    phi[:, hpos] = vals
    phi[:, neg[hpos]] = np.conj(vals)
    return phi


@dataclasses.dataclass(frozen=True)
class ServingJob:
    job_id: int
    workload: Workload
    arrival_s: float


def serving_stream(n_jobs: int = 300, rate_hz: float = 1.0, base_seed: int = 1506,
                   grids: Sequence[int] = (24, 32, 48)) -> List[ServingJob]:
    """Poisson stream of PDEP jobs of mixed grid and band sizes.

    Cell edge L = n * 20/48 bohr (10, 13.33, 20), ecut 12 Ha, wells = round(64 * vol/8000),
    N_v ~ U{8..128}, N_pdep ~ U{16..64}; job k uses seed base_seed + 1 + k for its wells.
    """
    rng = np.random.Generator(np.random.PCG64(base_seed))
    t = 0.0
    jobs = []
    for k in range(n_jobs):
        t += rng.exponential(1.0 / rate_hz)
        g = int(grids[rng.integers(0, len(grids))])
        nv = int(rng.integers(8, 129))
        npd = int(rng.integers(16, 65))
        Ledge = g * 20.0 / 48.0
        nw = int(round(64.0 * Ledge ** 3 / 8000.0))
        wl = Workload(f"job{k}", (Ledge,) * 3, (g,) * 3, 12.0, nw, nv, npd, 1e-8, base_seed + 1 + k)
        jobs.append(ServingJob(k, wl, t))
    return jobs


def random_grid_potentials(n: Sequence[int], n_pert: int, seed: int) -> np.ndarray:
    """Real random-normal potentials on the grid, [n_pert, N_g] (test input for the
    grid-level density-response hook)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n_pert, int(np.prod(n))))
