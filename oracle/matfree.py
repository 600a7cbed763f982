"""Matrix-free FP64 version of the same chi0bar chain (FFT-based H, conjugate gradient).

Test infrastructure only (see the package docstring).

This is the chain of the response module with the dense matrices replaced by
numpy FFTs (pinned equal to the naive DFT on small grids) and the direct solves
replaced by preconditioned conjugate gradient, which is what the paper proposes for the
Sternheimer equation (Sec. 2.3, after Eq. stern).  It is used to time a CPU baseline
and for sampled checks on cells where the dense matrices do not fit.

Preconditioner: K_G = 1/max(1/2|G|^2 - e_v, 0.1) followed by P_c (the paper names a
preconditioned CG without fixing K; K changes iteration counts only).
Stopping rule per band: ||P_c(b - A x)|| <= tol ||b||, x0 = 0; b = 0 gives x = 0.
"""
from __future__ import annotations

import numpy as np

from . import planewave as pw
from .response import GroundState, Model, project_c  # noqa: F401


def h_apply(model: Model, X: np.ndarray, shift: np.ndarray) -> np.ndarray:
    """(H - shift_k) x_k for the rows of X [k, N_pw], with H applied through the FFT."""
    f = pw.inv_fft(model.n, model.idx, X)
    f *= model.vloc[None]
    out = pw.fwd_fft(model.n, model.idx, f)
    out += (model.kin[None, :] - shift[:, None]) * X
    return out


def cg_bands(model: Model, eps: np.ndarray, C: np.ndarray, B: np.ndarray, tol: float,
             maxit: int = 5000, precondition: bool = True):
    """Solve P_c (H - e_v) P_c x_v = b_v for a set of bands at once: row k of B has
    shift eps[k]; C [N_v, N_pw] holds every occupied band (P_c removes all of them).
    Returns (X, iterations)."""
    X = np.zeros_like(B)
    R = project_c(C, B.copy())
    bnorm = np.linalg.norm(B, axis=1)
    active = bnorm > 0
    if precondition:
        K = 1.0 / np.maximum(0.1, model.kin[None, :] - eps[:, None])
        Z = project_c(C, K * R)
    else:
        K = None
        Z = R.copy()
    P = Z.copy()
    rz = np.real(np.sum(np.conj(R) * Z, axis=1))
    it = 0
    for it in range(1, maxit + 1):
        rn = np.linalg.norm(R, axis=1)
        done = (~active) | (rn <= tol * np.where(bnorm > 0, bnorm, 1.0))
        if np.all(done):
            return X, it - 1
        AP = project_c(C, h_apply(model, P, eps))
        pap = np.real(np.sum(np.conj(P) * AP, axis=1))
        alpha = np.where(done, 0.0, rz / np.where(pap != 0, pap, 1.0))
        X += alpha[:, None] * P
        R -= alpha[:, None] * AP
        Z = project_c(C, K * R) if precondition else R.copy()
        rz_new = np.real(np.sum(np.conj(R) * Z, axis=1))
        beta = np.where(done, 0.0, rz_new / np.where(rz != 0, rz, 1.0))
        P = Z + beta[:, None] * P
        rz = rz_new
    return X, maxit


def chi0bar_apply_cg(model: Model, gs: GroundState, phi: np.ndarray, tol: float,
                     bands=None, precondition: bool = True):
    """chi0bar on a block phi [k, N_pw'] through FFT + CG.  If `bands` is given, only
    those occupied bands are solved (a timing sample; the result is then partial).
    Returns (result [k, N_pw'], total CG iterations)."""
    phi = np.atleast_2d(phi)
    k = phi.shape[0]
    full = np.zeros((k, model.n_pw), dtype=np.complex128)
    full[:, model.nz] = phi * model.coul[None, :]
    dV = np.real(pw.inv_fft(model.n, model.idx, full))           # [k, *n]
    sel = np.arange(gs.C.shape[0]) if bands is None else np.asarray(bands)
    Usub = gs.U[sel].reshape((len(sel),) + tuple(model.n))
    out = np.empty((k, int(np.sum(model.nz))), dtype=np.complex128)
    iters = 0
    for i in range(k):
        W = pw.fwd_fft(model.n, model.idx, dV[i][None] * Usub)
        B = -project_c(gs.C, W)
        X, it = cg_bands(model, gs.eps[sel], gs.C, B, tol, precondition=precondition)
        iters += it
        dpsi = pw.inv_fft(model.n, model.idx, X)
        dn = (4.0 / model.volume) * np.real(np.sum(np.conj(Usub) * dpsi, axis=0))
        F = pw.fwd_fft(model.n, model.idx, dn.astype(np.complex128))
        out[i] = F[model.nz] * model.coul
    return out, iters
