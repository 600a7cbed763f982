"""Plane-wave basis, grid and the model Kohn-Sham Hamiltonian, written out densely.

Test infrastructure only (see the package docstring).

Conventions (Hartree units, orthorhombic cell of edges L, grid n, N_g = prod(n)):
* G = 2 pi (mx/Lx, my/Ly, mz/Lz) for integer Miller indices m;
* basis sphere S = {G : 1/2 |G|^2 <= E_cut}, listed lexicographically in (mx, my, mz)
  with mz fastest (the plane-wave expansion of Sec. 2.1 with its cutoff; the
  boundary case never occurs for the workloads here, so "<" and "<=" agree);
* grid points r_j = (ix Lx/nx, iy Ly/ny, iz Lz/nz), C order (ix, iy, iz);
* Inv(c)(r_j) = sum_{G in S} c_G exp(i G.r_j)      (sphere -> grid)
* Fwd(f)(G)   = N_g^-1 sum_j f(r_j) exp(-i G.r_j)   (grid -> sphere);
* H = diag(1/2 |G|^2) + Fwd(V_loc * Inv(.)) restricted to S (KS equation of Sec. 2 with
  a local potential only).  Products on the grid alias exactly as the discrete
  transforms make them; that aliasing is part of the model.
"""
from __future__ import annotations

import math
import os

import numpy as np
import scipy.fft as sfft

# threads of the batched FFTs (pocketfft through scipy.fft, run over the batch): the
# ORACLE_FFT_WORKERS or OMP_NUM_THREADS setting, else every CPU
FFT_WORKERS = (int(os.environ.get("ORACLE_FFT_WORKERS", "0") or 0)
               or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1))


def sphere(L, ecut):
    """Miller indices of S, int64 [N_pw, 3], lexicographic with mz fastest."""
    L = np.asarray(L, dtype=np.float64)
    nmax = [int(math.floor(math.sqrt(2.0 * ecut) * L[d] / (2.0 * math.pi))) + 1 for d in range(3)]
    rng = [np.arange(-k, k + 1) for k in nmax]
    mx, my, mz = np.meshgrid(*rng, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1).astype(np.int64)
    G = 2.0 * math.pi * m / L[None, :]
    keep = 0.5 * np.sum(G * G, axis=1) <= ecut
    return m[keep]


def gvectors(L, miller):
    return 2.0 * math.pi * np.asarray(miller, dtype=np.float64) / np.asarray(L, dtype=np.float64)[None, :]


def kinetic(L, miller):
    G = gvectors(L, miller)
    return 0.5 * np.sum(G * G, axis=1)


def grid_index(n, miller):
    """Flat C-order grid index of each G (Miller index taken modulo the grid)."""
    m = np.asarray(miller, dtype=np.int64)
    return ((m[:, 0] % n[0]) * n[1] + (m[:, 1] % n[1])) * n[2] + (m[:, 2] % n[2])


def nonzero_mask(miller):
    return np.any(np.asarray(miller) != 0, axis=1)


def dft_matrix(n, miller):
    """E[j, g] = exp(i G_g . r_j), N_g x N_pw, phases reduced exactly in integers."""
    n = [int(x) for x in n]
    m = np.asarray(miller, dtype=np.int64)
    ix, iy, iz = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    frac = (((ix[:, None] * m[None, :, 0]) % n[0]) / n[0]
            + ((iy[:, None] * m[None, :, 1]) % n[1]) / n[1]
            + ((iz[:, None] * m[None, :, 2]) % n[2]) / n[2])
    return np.exp(2j * math.pi * frac)


def inv_naive(E, c):
    """Sphere -> grid by the naive DFT; c is [N_pw] or [N_pw, k]."""
    return E @ c


def fwd_naive(E, f):
    """Grid -> sphere by the naive DFT; f is [N_g] or [N_g, k]."""
    return (E.conj().T @ f) / E.shape[0]


def hamiltonian_naive(E, kin, vloc_flat):
    """Dense H = diag(T) + E^H diag(V) E / N_g."""
    H = (E.conj().T @ (vloc_flat[:, None] * E)) / E.shape[0]
    H[np.diag_indices_from(H)] += kin
    return H


# --- FFT route (pocketfft via scipy.fft); pinned equal to the naive DFT by the tests -----

def inv_fft(n, idx, c):
    """Sphere -> grid with a library FFT: N_g * ifftn of the scattered coefficients.
    c is [N_pw] or [k, N_pw]; returns grid(s) of shape n or [k, *n]."""
    n = tuple(int(x) for x in n)
    c = np.asarray(c)
    batch = c.ndim == 2
    cc = c if batch else c[None, :]
    g = np.zeros((cc.shape[0], int(np.prod(n))), dtype=np.complex128)
    g[:, idx] = cc
    out = sfft.ifftn(g.reshape((cc.shape[0],) + n), axes=(1, 2, 3), workers=FFT_WORKERS) * float(np.prod(n))
    return out if batch else out[0]


def fwd_fft(n, idx, f):
    """Grid -> sphere with a library FFT: fftn / N_g gathered at the sphere indices.
    f has shape n or [k, *n]; returns [N_pw] or [k, N_pw]."""
    n = tuple(int(x) for x in n)
    f = np.asarray(f)
    batch = f.ndim == 4
    ff = f if batch else f[None]
    F = sfft.fftn(ff, axes=(1, 2, 3), workers=FFT_WORKERS).reshape(ff.shape[0], -1) / float(np.prod(n))
    out = F[:, idx]
    return out if batch else out[0]


def hamiltonian_fft(n, miller, kin, vloc):
    """Dense H from the Fourier coefficients of V: H[g, g'] = V~(G_g - G_g') + delta T."""
    n = [int(x) for x in n]
    Vt = np.fft.fftn(np.asarray(vloc, dtype=np.float64).reshape(n)) / float(np.prod(n))
    m = np.asarray(miller, dtype=np.int64)
    d0 = (m[:, None, 0] - m[None, :, 0]) % n[0]
    d1 = (m[:, None, 1] - m[None, :, 1]) % n[1]
    d2 = (m[:, None, 2] - m[None, :, 2]) % n[2]
    H = Vt[d0, d1, d2].astype(np.complex128)
    H[np.diag_indices_from(H)] += kin
    return H
