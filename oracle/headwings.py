"""Head, wings and body of chi0bar at q -> 0 and imaginary frequencies, and the
reducible Lambda, Xi of Eq. Bfinal, written out densely.

Test infrastructure only (see the package docstring).  FP64.

In the q -> 0 limit (Table limitqchi0) the head of chi0bar is sum q_a F_ab q_b / q^2,
the wings -i sum_a q_a U_aj / q (and its Hermitian conjugate), the body B_ij.  With the
commutator vectors g^a_v = [H, r_a] psi_v, which for a local potential are -d/dr_a psi_v,
i.e. -i G_a c_v(G) in the plane-wave basis, the auxiliary functions
xi^a_v = P_c r_a psi_v solve (H - e_v) xi^a_v = P_c g^a_v (Eq. commu), and their
overlaps with the empty states are the dipole matrix elements <c|r_a|v> =
<c|g^a_v> / (e_c - e_v).  At omega = i u, with D = e_c - e_v and
f(D) = D / (D^2 + u^2) (Eq. AdlerWiser, two spins, both time orderings):

    F_ab(iu) = -(16 pi / Omega) sum_vc f(D) Re conj(<c|r_a|v>) <c|r_b|v>        (Eq. finalF)
    U_aj(iu) = -(4 / Omega) sqrt(4 pi) sum_vc f(D) Re conj(<c|r_a|v>) <c|V_j|v> (Eq. finalU1)
    B_ij(iu) = -(4 / Omega) sum_vc f(D) Re conj(<c|V_i|v>) <c|V_j|v>            (Eq. finalB)

with V_j = Re Inv(sqrt(4 pi)/|G| phi_j).  Everything is real: the orbitals, phi and g
are real in r.  From them Eq. Bfinal gives Lambda = (1 - B)^-1 B +
(1/k) (1 - B)^-1 mu (1 - B)^-1, k = 1 - f - Tr[mu (1 - B)^-1], f = (1/3) Tr F,
mu_ij = (1/3) sum_a U_ai U_aj (U_ia = U_ai, Hermiticity of chi0bar), and
Xi = (1 - k)/k times the integral of 4 pi / q^2 over the region around q = 0, here the
Brillouin zone of the Gamma-only cell, the box |q_a| <= pi / L_a.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from . import planewave as pw
from .lanczos import rhs_vectors
from .response import GroundState, Model, project_c, solve_direct


def commutator_vectors(model: Model, gs: GroundState) -> np.ndarray:
    """g[a, v] = [H, r_a] psi_v = -i G_a c_v(G) for a local potential (Eq. commu), [3, N_v, N_pw]."""
    G = pw.gvectors(model.L, model.miller)               # [N_pw, 3]
    return np.stack([-1j * G[None, :, a] * gs.C for a in range(3)])


def dipole_vectors(model: Model, gs: GroundState) -> np.ndarray:
    """xi[a, v] = P_c r_a psi_v: the solutions of (H - e_v) xi = P_c g^a_v on range(P_c)."""
    g = commutator_vectors(model, gs)
    return np.stack([solve_direct(model, gs, project_c(gs.C, g[a])) for a in range(3)])


def head_wings_body_sos(model: Model, gs: GroundState, phi: np.ndarray, u):
    """(F [nf, 3, 3], U [nf, 3, k], B [nf, k, k]) from the full diagonalisation of H,
    the dipole elements taken through the commutator, <c|r|v> = <c|g_v> / (e_c - e_v)."""
    if gs.C_all is None:
        raise ValueError("head_wings_body_sos needs ground_state(full=True)")
    n_v = gs.C.shape[0]
    Cc = gs.C_all[:, n_v:]
    ec = gs.eps_all[n_v:]
    g = commutator_vectors(model, gs)
    W = rhs_vectors(model, gs, phi)                       # [k, N_v, N_pw]
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    k = W.shape[0]
    F = np.zeros((u.size, 3, 3))
    U = np.zeros((u.size, 3, k))
    B = np.zeros((u.size, k, k))
    s4 = math.sqrt(4.0 * math.pi)
    for v in range(n_v):
        D = ec - gs.eps[v]
        R = (Cc.conj().T @ g[:, v, :].T) / D[:, None]     # <c|r_a|v>, [n_c, 3]
        P = Cc.conj().T @ W[:, v, :].T                    # <c|V_j|v>, [n_c, k]
        for f, uf in enumerate(u):
            w = D / (D * D + uf * uf)
            F[f] += np.real(R.conj().T @ (w[:, None] * R))
            U[f] += np.real(R.conj().T @ (w[:, None] * P))
            B[f] += np.real(P.conj().T @ (w[:, None] * P))
    return (-16.0 * math.pi / model.volume) * F, (-4.0 / model.volume) * s4 * U, (-4.0 / model.volume) * B


def head_wings_body_resolvent(model: Model, gs: GroundState, phi: np.ndarray, u):
    """The same three blocks without empty states: the dipole vectors from the
    Sternheimer solve of Eq. commu and f(A_v) applied by a dense linear solve with
    A_v = H - e_v + sigma P_v (equal to P_c (H - e_v) P_c on range(P_c))."""
    n_v = gs.C.shape[0]
    X = dipole_vectors(model, gs)                          # [3, N_v, N_pw]
    W = rhs_vectors(model, gs, phi)                        # [k, N_v, N_pw]
    s4 = math.sqrt(4.0 * math.pi)
    Y = np.concatenate([s4 * X, W], axis=0)                # rows: 3 directions, then k potentials
    H = gs.H
    sigma = float(gs.eps[-1] - gs.eps[0] + 1.0)
    Pv = gs.C.T @ gs.C.conj()
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    E = np.zeros((u.size, Y.shape[0], Y.shape[0]))
    for v in range(n_v):
        A = H - gs.eps[v] * np.eye(H.shape[0]) + sigma * Pv
        AY = A @ Y[:, v, :].T
        for f, uf in enumerate(u):
            Z = np.linalg.solve(A @ A + uf * uf * np.eye(H.shape[0]), AY)    # f(A) y
            E[f] += np.real(Y[:, v, :].conj() @ Z)
    E *= -4.0 / model.volume
    return E[:, :3, :3], E[:, :3, 3:], E[:, 3:, 3:]


def bz_coulomb_integral(L) -> float:
    """int d^3q / (2 pi)^3 4 pi / q^2 over the box |q_a| <= h_a = pi / L_a.  The box is
    the union of the six pyramids over its faces; on the pyramid of the face q_a = h_a,
    q = q_a (1, s, t) with |s| <= h_b / h_a, |t| <= h_c / h_a, and the radial integral is
    h_a times the smooth integral of 1 / (1 + s^2 + t^2) over that rectangle."""
    h = np.pi / np.asarray(L, dtype=np.float64)
    total = 0.0
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        sb, sc = h[b] / h[a], h[c] / h[a]
        val, _ = integrate.dblquad(lambda t, s: 1.0 / (1.0 + s * s + t * t), -sb, sb, -sc, sc,
                                   epsabs=1e-14, epsrel=1e-13)
        total += 2.0 * h[a] * val
    return total * 4.0 * math.pi / (2.0 * math.pi) ** 3


def lambda_xi(F: np.ndarray, U: np.ndarray, B: np.ndarray, L):
    """Eq. Bfinal at one frequency: (Lambda [k, k], Xi, k)."""
    n = B.shape[0]
    M = np.linalg.inv(np.eye(n) - B)                      # (1 - B)^-1
    mu = (U.T @ U) / 3.0                                  # mu_ij = 1/3 sum_a U_ai U_aj
    f = np.trace(F) / 3.0
    kk = 1.0 - f - np.trace(mu @ M)
    Lam = M @ B + (M @ mu @ M) / kk
    Xi = (1.0 - kk) / kk * bz_coulomb_integral(L)
    return Lam, Xi, kk
