"""Ground state, Sternheimer response, density response and chi0bar, densely.

Test infrastructure only (see the package docstring).  FP64 throughout.

The result of the PDEP/DFPT chain has a plain definition, and this module writes that
definition out with dense matrices and direct solves:

* ground state: the N_v lowest eigenpairs of the dense H (KS equation, Sec. 2);
* Sternheimer (Sec. 2.3, Eq. stern): for a real potential dV(r) and occupied band v,
  b_v = -P_c Fwd(dV * u_v) and dc_v solves P_c (H - e_v) P_c dc_v = b_v in range(P_c),
  P_c = 1 - sum_v |c_v><c_v|.  Solved by LU of H - e_v + sigma P_v with
  sigma = e_{N_v} - e_1 + 1, which is positive definite and agrees with the projected
  system on range(P_c);
* sum over states (Eq. AdlerWiser at omega = 0, body): dc_v = sum_{c > N_v}
  c_c <c_c|Fwd(dV u_v)> / (e_v - e_c), from the full diagonalisation;
* density response (Eq. deltani at Gamma, two spins, u_v = Omega^{1/2} psi_v):
  dn(r) = (4/Omega) Re sum_v conj(u_v(r)) Inv(dc_v)(r);
* chi0bar on S' = S minus G=0 (Eq. chiisamatrixinpdep with V_pert = phi~):
  phi~(G) = sqrt(4 pi)/|G| phi(G), dV = Inv(phi~) (real), and
  (chi0bar phi)(G) = sqrt(4 pi)/|G| Fwd(dn)(G).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.linalg as sla

from . import planewave as pw


@dataclasses.dataclass
class Model:
    L: tuple
    n: tuple
    ecut: float
    vloc: np.ndarray          # real grid, shape n
    miller: np.ndarray        # S, lexicographic
    kin: np.ndarray           # 1/2 |G|^2 on S
    idx: np.ndarray           # flat grid index of each G in S
    nz: np.ndarray            # mask of S' inside S
    coul: np.ndarray          # sqrt(4 pi)/|G| on S'
    E: Optional[np.ndarray]   # naive DFT matrix (small cells only)

    @property
    def n_grid(self) -> int:
        return int(np.prod(self.n))

    @property
    def volume(self) -> float:
        return float(self.L[0] * self.L[1] * self.L[2])

    @property
    def n_pw(self) -> int:
        return int(self.miller.shape[0])

    def inv(self, c):
        """Sphere -> grid; c is [N_pw] or [k, N_pw]; returns flat grid(s)."""
        if self.E is not None:
            out = pw.inv_naive(self.E, np.asarray(c).T).T
        else:
            out = pw.inv_fft(self.n, self.idx, c).reshape(np.asarray(c).shape[:-1] + (-1,))
        return out

    def fwd(self, f):
        """Grid -> sphere; f is flat [N_g] or [k, N_g]."""
        f = np.asarray(f)
        if self.E is not None:
            return pw.fwd_naive(self.E, f.T).T
        ff = f.reshape(f.shape[:-1] + tuple(self.n))
        return pw.fwd_fft(self.n, self.idx, ff)


def make_model(L, n, ecut, vloc, naive: Optional[bool] = None) -> Model:
    """naive=None picks the naive DFT for grids up to 16^3."""
    miller = pw.sphere(L, ecut)
    kin = pw.kinetic(L, miller)
    idx = pw.grid_index(n, miller)
    nz = pw.nonzero_mask(miller)
    G = pw.gvectors(L, miller[nz])
    coul = math.sqrt(4.0 * math.pi) / np.sqrt(np.sum(G * G, axis=1))
    if naive is None:
        naive = int(np.prod(n)) <= 4096
    E = pw.dft_matrix(n, miller) if naive else None
    return Model(tuple(L), tuple(int(x) for x in n), float(ecut),
                 np.asarray(vloc, dtype=np.float64).reshape(n), miller, kin, idx, nz, coul, E)


def hamiltonian(model: Model) -> np.ndarray:
    if model.E is not None:
        return pw.hamiltonian_naive(model.E, model.kin, model.vloc.ravel())
    return pw.hamiltonian_fft(model.n, model.miller, model.kin, model.vloc)


@dataclasses.dataclass
class GroundState:
    eps: np.ndarray     # [N_v] occupied energies, ascending
    C: np.ndarray       # [N_v, N_pw] occupied coefficients (band-major rows)
    U: np.ndarray       # [N_v, N_g] u_v(r) = Inv(c_v)
    gap: float          # e_{N_v+1} - e_{N_v}
    eps_all: Optional[np.ndarray] = None
    C_all: Optional[np.ndarray] = None   # [N_pw, N_pw] columns = eigenvectors
    H: Optional[np.ndarray] = None


def ground_state(model: Model, n_v: int, full: bool = False) -> GroundState:
    H = hamiltonian(model)
    if full:
        w, V = np.linalg.eigh(H)
        eps, C = w[:n_v], V[:, :n_v].T.copy()
        gap = float(w[n_v] - w[n_v - 1])
        gs = GroundState(eps, C, model.inv(C), gap, w, V, H)
    else:
        w, V = sla.eigh(H, subset_by_index=[0, n_v])
        gs = GroundState(w[:n_v].copy(), V[:, :n_v].T.copy(), None, float(w[n_v] - w[n_v - 1]), None, None, H)
        gs.U = model.inv(gs.C)
    return gs


def project_c(C, x):
    """P_c x = x - sum_v c_v (c_v^H x); x is [k, N_pw], C is [N_v, N_pw]."""
    return x - (x @ C.conj().T) @ C


def rhs(model: Model, gs: GroundState, dV) -> np.ndarray:
    """b_v = -P_c Fwd(dV * u_v), [N_v, N_pw]."""
    w = model.fwd(np.asarray(dV, dtype=np.float64).ravel()[None, :] * gs.U)
    return -project_c(gs.C, w)


def solve_direct(model: Model, gs: GroundState, b: np.ndarray) -> np.ndarray:
    """Solve P_c (H - e_v) P_c x_v = b_v on range(P_c), one LU per band."""
    H = gs.H if gs.H is not None else hamiltonian(model)
    sigma = float(gs.eps[-1] - gs.eps[0] + 1.0)
    Pv = gs.C.T @ gs.C.conj()                       # sum_v |c_v><c_v|
    out = np.empty_like(b)
    for v in range(gs.C.shape[0]):
        A = H - gs.eps[v] * np.eye(H.shape[0]) + sigma * Pv
        out[v] = np.linalg.solve(A, b[v])
    return project_c(gs.C, out)


def solve_direct_many(model: Model, gs: GroundState, B: np.ndarray) -> np.ndarray:
    """Like solve_direct for many perturbations at once; B is [n_pert, N_v, N_pw]."""
    H = gs.H if gs.H is not None else hamiltonian(model)
    sigma = float(gs.eps[-1] - gs.eps[0] + 1.0)
    Pv = gs.C.T @ gs.C.conj()
    out = np.empty_like(B)
    for v in range(gs.C.shape[0]):
        A = H - gs.eps[v] * np.eye(H.shape[0]) + sigma * Pv
        lu = sla.lu_factor(A)
        out[:, v, :] = sla.lu_solve(lu, B[:, v, :].T).T
    n_pert = B.shape[0]
    return project_c(gs.C, out.reshape(-1, B.shape[2])).reshape(B.shape)


def solve_sos(gs: GroundState, w: np.ndarray) -> np.ndarray:
    """Sum over empty states: dc_v = sum_c c_c (c_c^H w_v)/(e_v - e_c), w_v = Fwd(dV u_v)."""
    if gs.C_all is None:
        raise ValueError("solve_sos needs the full diagonalisation (ground_state(full=True))")
    n_v = gs.C.shape[0]
    Cc = gs.C_all[:, n_v:]
    ec = gs.eps_all[n_v:]
    out = np.empty_like(w)
    for v in range(n_v):
        coef = (Cc.conj().T @ w[v]) / (gs.eps[v] - ec)
        out[v] = Cc @ coef
    return out


def density_response(model: Model, gs: GroundState, dC: np.ndarray) -> np.ndarray:
    """dn(r) = (4/Omega) Re sum_v conj(u_v) Inv(dc_v); dC is [N_v, N_pw]; flat real grid."""
    dpsi = model.inv(dC)
    return (4.0 / model.volume) * np.real(np.sum(np.conj(gs.U) * dpsi, axis=0))


def chi0_real(model: Model, gs: GroundState, dV, method: str = "direct") -> np.ndarray:
    """Density response (flat real grid) to a real potential dV on the grid."""
    b = rhs(model, gs, dV)
    if method == "direct":
        dC = solve_direct(model, gs, b)
    elif method == "sos":
        w = model.fwd(np.asarray(dV, dtype=np.float64).ravel()[None, :] * gs.U)
        dC = solve_sos(gs, w)
    else:
        raise ValueError(method)
    return density_response(model, gs, dC)


def perturbation_grid(model: Model, phi: np.ndarray) -> np.ndarray:
    """dV = Inv(phi~) on the grid, phi~ = sqrt(4 pi)/|G| phi on S'; real part (phi is
    Hermitian-symmetric, so the imaginary part is rounding only).  phi: [k, N_pw']."""
    phi = np.atleast_2d(phi)
    full = np.zeros((phi.shape[0], model.n_pw), dtype=np.complex128)
    full[:, model.nz] = phi * model.coul[None, :]
    return np.real(model.inv(full))


def project_density(model: Model, dn: np.ndarray) -> np.ndarray:
    """(chi0bar phi)(G) = sqrt(4 pi)/|G| Fwd(dn)(G) on S'; dn: [k, N_g]."""
    F = model.fwd(np.atleast_2d(dn).astype(np.complex128))
    return F[:, model.nz] * model.coul[None, :]


def chi0bar_apply(model: Model, gs: GroundState, phi: np.ndarray, method: str = "direct") -> np.ndarray:
    """chi0bar applied to a block of Hermitian-symmetric potentials phi [k, N_pw']."""
    phi = np.atleast_2d(phi)
    dV = perturbation_grid(model, phi)                       # [k, N_g]
    k = phi.shape[0]
    n_v = gs.C.shape[0]
    W = model.fwd((dV[:, None, :] * gs.U[None, :, :]).reshape(k * n_v, -1)).reshape(k, n_v, -1)
    if method == "direct":
        B = -project_c(gs.C, W.reshape(k * n_v, -1)).reshape(W.shape)
        dC = solve_direct_many(model, gs, B)
    elif method == "sos":
        dC = np.stack([solve_sos(gs, W[i]) for i in range(k)])
    else:
        raise ValueError(method)
    dpsi = model.inv(dC.reshape(k * n_v, -1)).reshape(k, n_v, -1)
    dn = (4.0 / model.volume) * np.real(np.sum(np.conj(gs.U)[None] * dpsi, axis=1))
    return project_density(model, dn)


def real_basis(model: Model) -> np.ndarray:
    """Orthonormal basis of Hermitian-symmetric vectors on S': for each G in the canonical
    half, (e_G + e_-G)/sqrt2 and i(e_G - e_-G)/sqrt2.  Returns complex [N', N']."""
    m = model.miller[model.nz]
    mx, my, mz = m[:, 0], m[:, 1], m[:, 2]
    half = (mx > 0) | ((mx == 0) & (my > 0)) | ((mx == 0) & (my == 0) & (mz > 0))
    pos = {tuple(r): k for k, r in enumerate(m.tolist())}
    Np = m.shape[0]
    Bm = np.zeros((Np, Np), dtype=np.complex128)
    col = 0
    s = 1.0 / math.sqrt(2.0)
    for k in np.nonzero(half)[0]:
        kn = pos[tuple((-m[k]).tolist())]
        Bm[col, k] = s
        Bm[col, kn] = s
        Bm[col + 1, k] = 1j * s
        Bm[col + 1, kn] = -1j * s
        col += 2
    assert col == Np
    return Bm


def chi0bar_matrix(model: Model, gs: GroundState, method: str = "direct"):
    """Full chi0bar in the real basis (real symmetric [N', N']) and the basis rows."""
    Bm = real_basis(model)
    K = chi0bar_apply(model, gs, Bm, method=method)          # rows: chi0bar b_a
    M = np.real(Bm.conj() @ K.T)                              # M[a, b] = <b_a | chi0bar b_b>
    return M, Bm


def pdep_exact(model: Model, gs: GroundState, n_pdep: int):
    """Exact PDEP: the n_pdep lowest (most negative) eigenvalues of chi0bar and the
    eigenvectors on S' (rows), from the full matrix.  Returns (lam ascending, Phi, M)."""
    M, Bm = chi0bar_matrix(model, gs)
    Ms = 0.5 * (M + M.T)
    lam, Y = np.linalg.eigh(Ms)
    Phi = Y[:, :n_pdep].T @ Bm
    return lam[:n_pdep], Phi, Ms


def rayleigh_ritz(model: Model, gs: GroundState, X: np.ndarray):
    """Ritz values of chi0bar on span(X) (X rows Hermitian-symmetric, not necessarily
    orthonormal): eigenvalues of (X^H X)^{-1/2} X^H chi0bar X (X^H X)^{-1/2}."""
    AX = chi0bar_apply(model, gs, X)
    S = np.real(X.conj() @ X.T)
    M = np.real(X.conj() @ AX.T)
    M = 0.5 * (M + M.T)
    return sla.eigh(M, S, eigvals_only=True)


def subspace_iteration(model: Model, gs: GroundState, X0: np.ndarray, n_iter: int = 50,
                       tol: float = 1e-10):
    """Plain Rayleigh-Ritz subspace iteration X <- orth(chi0bar X).  chi0bar is negative
    semidefinite, so its most negative eigenvalues are the largest in magnitude and
    dominate the power iteration.  An independent route to the lowest PDEP eigenvalues on cells where the full matrix
    is too large.  Returns (lam ascending, iterations)."""
    X = np.atleast_2d(X0).astype(np.complex128)
    lam_old = None
    for it in range(1, n_iter + 1):
        AX = chi0bar_apply(model, gs, X)
        S = np.real(X.conj() @ X.T)
        M = np.real(X.conj() @ AX.T)
        M = 0.5 * (M + M.T)
        lam, Y = sla.eigh(M, S)
        X = Y.T @ X
        AX = Y.T @ AX
        if lam_old is not None and np.max(np.abs(lam - lam_old)) < tol:
            return lam, it
        lam_old = lam
        X = AX
        # orthonormalise (real coefficients keep Hermitian symmetry)
        S = np.real(X.conj() @ X.T)
        Lc = np.linalg.cholesky(S)
        X = np.linalg.solve(Lc, X)
    return lam_old, n_iter


# --- reducible polarizability (RPA, Hartree term only) -------------------------------------

def chibar_from_chi0bar(M: np.ndarray) -> np.ndarray:
    """The reducible symmetrised polarizability from the irreducible one by linear algebra
    (Eq. linearalgebrachichi0): chibar = (1 - chi0bar)^{-1} chi0bar, M a square matrix of
    chi0bar in any orthonormal basis."""
    return np.linalg.solve(np.eye(M.shape[0]) - M, M)


def hartree_potential(model: Model, dnG: np.ndarray) -> np.ndarray:
    """Linear change of the Hartree potential (Eq. LFHartree) in G space on S':
    dV_H(G) = 4 pi dn(G) / |G|^2 (Hartree units, e^2 = 1)."""
    return model.coul[None, :] ** 2 * dnG


def chibar_apply_scf(model: Model, gs: GroundState, phi: np.ndarray, tol: float = 1e-12,
                     maxit: int = 500, mixing: float = 0.4):
    """Reducible chibar on a block phi [k, N_pw'] by the self-consistent DFPT loop of
    Fig. pdepscheme (right panel): the Sternheimer perturbation is the applied potential
    phi~ plus the linear change of the Hartree potential of the density response (the
    Hartree term of Eq. LF, Eq. LFHartree; RPA), dV_H(G) = 4 pi dn(G)/|G|^2, taken on S'
    like the potentials themselves.  Each pass solves the Sternheimer equations for the
    current total perturbation, forms dn (Eq. deltani) and its Hartree potential, and
    mixes it linearly into the next perturbation; at self-consistency sqrt(4 pi)/|G|
    dn(G) on S' is chibar phi (Eq. chiisamatrixinpdep with the screened response).  A
    pass multiplies the error by 1 - mixing (1 - lambda) on each eigenvector of chi0bar,
    so the loop converges for mixing < 2 / eps_max (eps_max = 1 - lambda_min).  Returns
    (chibar phi [k, N_pw'], passes)."""
    phi = np.atleast_2d(phi)
    coul = model.coul[None, :]                     # sqrt(4 pi)/|G| on S'
    vH = np.zeros_like(phi, dtype=np.complex128)   # Hartree potential on S'
    out = None
    for it in range(1, maxit + 1):
        pert = phi * coul + vH                     # phi~ + dV_H
        full = np.zeros((phi.shape[0], model.n_pw), dtype=np.complex128)
        full[:, model.nz] = pert
        dV = np.real(model.inv(full))
        dn = np.stack([chi0_real(model, gs, dV[i]) for i in range(phi.shape[0])])
        dnG = model.fwd(dn.astype(np.complex128))[:, model.nz]
        vH_new = hartree_potential(model, dnG)
        new = coul * dnG
        if out is not None and np.max(np.linalg.norm(new - out, axis=1) / np.linalg.norm(new, axis=1)) <= tol:
            return new, it
        out = new
        vH = (1.0 - mixing) * vH + mixing * vH_new
    return out, maxit


def eps_inverse_eigenvalues(lam: np.ndarray) -> np.ndarray:
    """Eigenvalues of the inverse dielectric matrix from those of chi0bar: chibar has the
    eigenvalues lambda / (1 - lambda) on the same eigenvectors (Eq. linearalgebrachichi0)
    and eps^-1 = 1 + chibar (Eq. epsilonandchi), hence 1 / (1 - lambda)."""
    return 1.0 / (1.0 - np.asarray(lam))
