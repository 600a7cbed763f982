"""G0W0 quasiparticle energies of occupied states at Gamma: the exchange term, the
correlation self-energy by contour deformation (Sec. 2.5, Eqs. contourdeformationfinal
and fcontour) and the solution of the quasiparticle equation (Eq. QPenergies) by the
secant method from the linearised root (Eq. QPconZ), written out with every state of the
dense diagonalisation.

Test infrastructure only (see the package docstring).  FP64.

Notation (Hartree units, u = Omega^1/2 psi on the grid, two spins):

* V_i = Re Inv(phi~_i), phi~_i = sqrt(4 pi)/|G| phi_i on S' (the basis potentials);
* W_p(r, r'; w) = Xi(w) + (1/Omega) sum_ij V_i(r) Lambda_ij(w) V_j(r') (Eq. Wchihb),
  Lambda and Xi from F, U, B by Eq. Bfinal (headwings.lambda_xi);
* pair coefficients b_mi = <c_m| Fwd(V_i u_n)> = (1/N_g) sum_r conj(u_m) V_i u_n, so
  that S_m(w) = <psi_n psi_m| W_p(w) |psi_m psi_n> = Xi(w) delta_mn
  + (1/Omega) b_m^H Lambda(w) b_m;
* G_KS(z) = sum_m |psi_m><psi_m| / (z - e_m) off the real axis (Eq. Glehmann);
* Sigma_C(E) = -(1/2pi) int dw' sum_m S_m(iw') / (E + iw' - e_m)
  + sum_m f_m S_m(e_m - E)  (Eq. contourdeformationfinal), f_m = +1 for
  e_F < e_m < E, -1 for E < e_m < e_F, else 0 (Eq. fcontour).  S_m(iw') is real and even
  in w', so the integral is -(1/pi) sum_m int_0^inf S_m(iw') d_m / (d_m^2 + w'^2) dw' with
  d_m = E - e_m, taken as
      -sgn(d_m) S_m(0) / 2 - (1/pi) int_0^inf [S_m(iw') - S_m(0)] d_m / (d_m^2 + w'^2) dw'
  (the first term integrates the Lorentzian exactly; the remainder stays smooth as
  d_m -> 0).  sgn(0) = +1: the limit E -> e_m from above, which with the strict
  inequalities of f_m keeps Sigma_C continuous at E = e_m.  The residues need W_p at the
  real frequency w = e_m - E, where it has the poles of Eq. AdlerWiser: there every
  transition enters as [1/(D + w - i eta) + 1/(D - w - i eta)] / 2 (D = e_c - e_v) with
  a finite broadening eta, which makes Lambda, Xi and the residue complex; the imaginary
  axis is taken at eta -> 0, where everything is real.  Im Sigma_C is the broadening's
  trace of the continuum (a lifetime), the QP equation uses Re Sigma_C;
* Sigma_X = -sum_{m occ} [I_BZ delta_mn + (4 pi / Omega) sum_{G in S'} |rho_mn(G)|^2 / |G|^2],
  rho_mn = Fwd(conj(u_m) u_n): the bare exchange on the set S' of the basis potentials,
  the G = 0 term by the integral I_BZ of 4 pi / q^2 over the region around q = 0 (the
  one Xi uses);
* E = e_n + Sigma_X + Sigma_C(E) - V_xc (Eq. QPenergies); Eq. QPconZ with
  Z = 1 / (1 - dSigma_C/dE at e_n) by a central difference starts the secant iteration.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from .headwings import bz_coulomb_integral, commutator_vectors, lambda_xi
from .lanczos import rhs_vectors
from .response import GroundState, Model


class Screening:
    """Lambda(w) and Xi(w) of Eq. Bfinal for the basis phi [k, N_pw'], from the full
    diagonalisation (sums over every empty state, Eq. AdlerWiser with the dipole elements
    through the commutator, as headwings.head_wings_body_sos).  at(w) is the imaginary
    frequency i w, where each transition carries D / (D^2 + w^2); at(w, real=True, eta)
    the real frequency w, where it carries [1/(D + w - i eta) + 1/(D - w - i eta)] / 2."""

    def __init__(self, model: Model, gs: GroundState, phi: np.ndarray):
        if gs.C_all is None:
            raise ValueError("Screening needs ground_state(full=True)")
        n_v = gs.C.shape[0]
        Cc = gs.C_all[:, n_v:]
        ec = gs.eps_all[n_v:]
        g = commutator_vectors(model, gs)                  # [3, N_v, N_pw]
        W = rhs_vectors(model, gs, phi)                    # [k, N_v, N_pw]
        s4 = math.sqrt(4.0 * math.pi)
        D, Y = [], []
        for v in range(n_v):
            d = ec - gs.eps[v]
            R = (Cc.conj().T @ g[:, v, :].T) / d[:, None]  # <c|r_a|v>
            P = Cc.conj().T @ W[:, v, :].T                 # <c|V_j|v>
            D.append(d)
            Y.append(np.concatenate([s4 * R, P], axis=1))
        self.D = np.concatenate(D)                         # transition energies e_c - e_v
        self.Y = np.concatenate(Y)                         # [transitions, 3 + k]
        self.k = W.shape[0]
        self.L = model.L
        self.volume = model.volume
        self.cache = {}

    def blocks(self, w: float, real: bool = False, eta: float = 0.0):
        """(F [3, 3], U [3, k], B [k, k]) at one frequency (complex when real=True)."""
        D = self.D
        if real:
            f = 0.5 * (1.0 / (D + w - 1j * eta) + 1.0 / (D - w - 1j * eta))
        else:
            f = D / (D * D + w * w)
        # sum_t f_t Re[conj(Y_ti) Y_tj]
        Yr, Yi = self.Y.real, self.Y.imag
        E = (-4.0 / self.volume) * (Yr.T @ (f[:, None] * Yr) + Yi.T @ (f[:, None] * Yi))
        return E[:3, :3], E[:3, 3:], E[3:, 3:]

    def at(self, w: float, real: bool = False, eta: float = 0.0):
        """(Lambda [k, k], Xi) at one frequency."""
        key = (float(w), bool(real), float(eta) if real else 0.0)
        if key not in self.cache:
            F, U, B = self.blocks(w, real, eta)
            lam, xi, _ = lambda_xi(F, U, B, self.L)
            self.cache[key] = (lam, xi)
        return self.cache[key]


def pair_coefficients(model: Model, gs: GroundState, phi: np.ndarray, n: int) -> np.ndarray:
    """b[m, i] = <c_m| Fwd(V_i u_n)> for every state m of the full diagonalisation, [N_pw, k]."""
    phi = np.atleast_2d(phi)
    full = np.zeros((phi.shape[0], model.n_pw), dtype=np.complex128)
    full[:, model.nz] = phi * model.coul[None, :]
    V = np.real(model.inv(full))                           # [k, N_g]
    un = model.inv(gs.C_all[:, n])
    Y = model.fwd(V * un[None, :])                         # [k, N_pw]
    return gs.C_all.conj().T @ Y.T


def pair_strengths(b: np.ndarray, lam: np.ndarray, xi, n: int, volume: float) -> np.ndarray:
    """S_m = <psi_n psi_m| W_p |psi_m psi_n> for every m (rows of b); complex when Lambda is."""
    S = np.einsum("mi,ij,mj->m", b.conj(), lam, b) / volume
    S[n] += xi
    return S


def sigma_x(model: Model, gs: GroundState, n: int) -> float:
    """Bare exchange <psi_n|Sigma_X|psi_n> over the occupied states."""
    n_v = gs.C.shape[0]
    un = model.inv(gs.C_all[:, n])
    total = 0.0
    for m in range(n_v):
        um = model.inv(gs.C_all[:, m])
        rho = model.fwd(np.conj(um) * un)[model.nz]
        total += float(np.sum(model.coul ** 2 * np.abs(rho) ** 2))
    head = bz_coulomb_integral(model.L) if n < n_v else 0.0
    return -total / model.volume - head


def sigma_c(E: float, n: int, eps_all: np.ndarray, e_fermi: float, b: np.ndarray, screen, volume: float,
            eta: float = 1e-3, epsabs: float = 1e-13, epsrel: float = 1e-11) -> complex:
    """<psi_n|Sigma_C(E)|psi_n> by contour deformation.  eps_all [M] and b [M, k] list every
    state; screen(w, real, eta) -> (Lambda, Xi) gives W_p at the imaginary frequency i w
    (real=False) or at the real frequency w with broadening eta."""
    d = E - np.asarray(eps_all, dtype=np.float64)
    lam0, xi0 = screen(0.0, False, 0.0)
    S0 = np.real(pair_strengths(b, lam0, xi0, n, volume))
    sgn = np.where(d >= 0.0, 1.0, -1.0)
    lorentz = -0.5 * float(np.sum(sgn * S0))

    def remainder(w):
        lam, xi = screen(w, False, 0.0)
        S = np.real(pair_strengths(b, lam, xi, n, volume))
        den = d * d + w * w
        kern = np.divide(d, den, out=np.zeros_like(d), where=den > 0.0)
        return float(np.sum((S - S0) * kern))

    rem, _ = integrate.quad(remainder, 0.0, np.inf, epsabs=epsabs, epsrel=epsrel, limit=500)
    res = 0.0 + 0.0j
    for m, em in enumerate(eps_all):
        if e_fermi < em < E:
            f = 1.0
        elif E < em < e_fermi:
            f = -1.0
        else:
            continue
        lam, xi = screen(abs(em - E), True, eta)
        res += f * complex(pair_strengths(b[m:m + 1], lam, xi if m == n else 0.0, 0, volume)[0])
    return lorentz - rem / math.pi + res


def qp_solve(sigma, eps_n: float, vxc: float = 0.0, h: float = 1e-3, tol: float = 1e-9, maxit: int = 40):
    """sigma(E) = Sigma_X + Re Sigma_C(E).  Eq. QPconZ gives e_lin = e_n + Z (sigma(e_n) - V_xc)
    with 1/Z = 1 - dsigma/dE(e_n) (central difference of step h); the secant method on
    g(E) = e_n + sigma(E) - V_xc - E then starts from the points e_n and e_lin."""
    s0 = sigma(eps_n)
    ds = (sigma(eps_n + h) - sigma(eps_n - h)) / (2.0 * h)
    z = 1.0 / (1.0 - ds)
    e_lin = eps_n + z * (s0 - vxc)
    x0, g0 = eps_n, s0 - vxc
    x1 = e_lin
    g1 = eps_n + sigma(x1) - vxc - x1
    it = 0
    for it in range(1, maxit + 1):
        if g1 == 0.0 or g1 == g0:
            break
        x2 = x1 - g1 * (x1 - x0) / (g1 - g0)
        x0, g0 = x1, g1
        x1 = x2
        g1 = eps_n + sigma(x1) - vxc - x1
        if abs(x1 - x0) <= tol:
            break
    return {"sigma_ks": s0, "z": z, "e_lin": e_lin, "e_qp": x1, "iterations": it, "residual": g1}


def quasiparticle(model: Model, gs: GroundState, phi: np.ndarray, n: int, e_fermi: float, vxc: float = 0.0,
                  screen=None, eta: float = 1e-3, **kw):
    """Sigma_X, Sigma_C(e_n), Z, e_lin and the secant root for the occupied state n."""
    if screen is None:
        screen = Screening(model, gs, phi).at
    b = pair_coefficients(model, gs, phi, n)
    sx = sigma_x(model, gs, n)
    seen = {}

    def sig(E):
        seen[E] = sigma_c(E, n, gs.eps_all, e_fermi, b, screen, model.volume, eta=eta)
        return sx + seen[E].real
    out = qp_solve(sig, float(gs.eps_all[n]), vxc, **kw)
    out["sigma_x"] = sx
    out["sigma_c_ks"] = seen[float(gs.eps_all[n])]
    out["sigma_c_qp"] = seen[out["e_qp"]] if out["e_qp"] in seen else sigma_c(
        out["e_qp"], n, gs.eps_all, e_fermi, b, screen, model.volume, eta=eta)
    return out
