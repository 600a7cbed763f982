"""The body of chi0bar at imaginary frequencies in a basis of potentials, two ways.

Test infrastructure only (see the package docstring).  FP64.

With w_jv = P_c Fwd(V_j u_v) (the Sternheimer right-hand side of Eq. stern for the
perturbation V_j = Inv(phi~_j), up to sign) and A_v = P_c (H - e_v) P_c on range(P_c),
the static chi0bar of the response module is

    chi0bar_ij = -(4/Omega) sum_v Re <w_iv| A_v^-1 |w_jv>,

and the Adler-Wiser form (Eq. AdlerWiser, body, q = 0) at the imaginary frequency
omega = i u replaces 2 / (e_v - e_c) by 1/(e_v - e_c + i u) + 1/(e_v - e_c - i u):

    B_ij(iu) = -(4/Omega) sum_v Re <w_iv| A_v (A_v^2 + u^2)^-1 |w_jv>      (Eq. finalB)

* body_sos: that definition written out with the full diagonalisation of H (sum over
  the empty states c, Eq. AdlerWiser);
* body_lanczos: the deflated Lanczos route of Sec. 2.4: for every (j, v) a Lanczos chain
  of the deflated Hamiltonian P_c H P_c started at |R> = w_jv / ||w_jv|| (q_1 = R,
  alpha_n = <q_n|H~|q_n>, beta_{n+1} q_{n+1} = (H~ - alpha_n) q_n - beta_n q_{n-1}) gives
  T = U D U^t, and <L| f(H~) |R> = sum_{n1 n2} <L|q_n1> U_n1n2 f(d_n2) U_1n2 (Eq. MCfinal)
  with L = w_iv and f(d) = (d - e_v) / ((d - e_v)^2 + u^2).
"""
from __future__ import annotations

import numpy as np

from .response import GroundState, Model, project_c


def rhs_vectors(model: Model, gs: GroundState, phi: np.ndarray) -> np.ndarray:
    """w[j, v] = P_c Fwd(V_j u_v) with V_j = Re Inv(phi~_j); phi [k, N_pw'] -> [k, N_v, N_pw]."""
    phi = np.atleast_2d(phi)
    full = np.zeros((phi.shape[0], model.n_pw), dtype=np.complex128)
    full[:, model.nz] = phi * model.coul[None, :]
    V = np.real(model.inv(full))                                        # [k, N_g]
    k, n_v = phi.shape[0], gs.C.shape[0]
    W = model.fwd((V[:, None, :] * gs.U[None, :, :]).reshape(k * n_v, -1))
    return project_c(gs.C, W).reshape(k, n_v, -1)


def body_sos(model: Model, gs: GroundState, phi: np.ndarray, u) -> np.ndarray:
    """B[f, i, j] at the imaginary frequencies u[f], from the full diagonalisation."""
    if gs.C_all is None:
        raise ValueError("body_sos needs the full diagonalisation (ground_state(full=True))")
    W = rhs_vectors(model, gs, phi)
    n_v = gs.C.shape[0]
    Cc = gs.C_all[:, n_v:]                  # empty states (columns)
    ec = gs.eps_all[n_v:]
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    out = np.zeros((u.size, W.shape[0], W.shape[0]))
    for v in range(n_v):
        P = Cc.conj().T @ W[:, v, :].T      # <c|w_jv>, [n_c, k]
        d = ec - gs.eps[v]                  # e_c - e_v > 0
        for f, uf in enumerate(u):
            g = d / (d * d + uf * uf)
            out[f] += np.real(P.conj().T @ (g[:, None] * P))
    return -(4.0 / model.volume) * out


def lanczos_chain(apply_h, r: np.ndarray, n_steps: int):
    """Lanczos chain of a Hermitian operator from r (normalised inside): returns the
    vectors Q [n, N] (rows), the diagonal alpha [n] and the off-diagonal beta [n - 1]
    of T = Q^H H Q.  Stops early (shorter outputs) when the chain closes."""
    q = r / np.linalg.norm(r)
    Q, alpha, beta = [q], [], []
    q_prev = np.zeros_like(q)
    b = 0.0
    for n in range(n_steps):
        z = apply_h(q)
        a = float(np.real(np.vdot(q, z)))
        alpha.append(a)
        if n == n_steps - 1:
            break
        z = z - a * q - b * q_prev
        b = float(np.linalg.norm(z))
        if b <= 1e-14 * abs(a) + 1e-300:
            break
        beta.append(b)
        q_prev, q = q, z / b
        Q.append(q)
    return np.array(Q), np.array(alpha), np.array(beta)


def body_lanczos(model: Model, gs: GroundState, phi: np.ndarray, u, n_lanczos: int = 40) -> np.ndarray:
    """B[f, i, j] at the imaginary frequencies u[f] by one Lanczos chain per (j, v)."""
    W = rhs_vectors(model, gs, phi)
    H = gs.H
    n_v = gs.C.shape[0]
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    k = W.shape[0]
    out = np.zeros((u.size, k, k))

    def h_tilde(x):                          # P_c H P_c
        return project_c(gs.C, (H @ project_c(gs.C, x[None, :])[0])[None, :])[0]
    for v in range(n_v):
        for j in range(k):
            r = W[j, v]
            rn = np.linalg.norm(r)
            if rn == 0.0:
                continue
            Q, a, b = lanczos_chain(h_tilde, r, n_lanczos)
            T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
            d, U = np.linalg.eigh(T)
            ov = np.real(W[:, v, :].conj() @ Q.T)             # <L_i|q_n>, [k, n]
            for f, uf in enumerate(u):
                x = d - gs.eps[v]
                g = x / (x * x + uf * uf) * U[0, :]
                out[f, :, j] += rn * (ov @ (U @ g))
    return -(4.0 / model.volume) * out
