"""Pins of the oracle's G0W0 module (exchange, contour-deformation Sigma_C, QP solver)
against facts that do not come from the module itself: a closed-form GW self-energy for a
screened interaction given as a sum of poles, closed-form exchange for free electrons, the
static chi0bar of the response module, the self-consistent reducible response, the
finite-frequency Sternheimer equation solved densely, and the root of a QP equation with a
closed form.  Mutation tests plant mistakes and check that a pin catches them."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import gw
from oracle import headwings as HW
from oracle import response as R
from paper_1501_03141_amd import inputs

TINY = inputs.WORKLOADS["tiny"]


@pytest.fixture(scope="module")
def tiny():
    V = inputs.vloc(TINY)
    m = R.make_model(TINY.L, TINY.n, TINY.ecut, V)
    gs = R.ground_state(m, TINY.n_v, full=True)
    M, Bm = R.chi0bar_matrix(m, gs)
    lam, vec = np.linalg.eigh(0.5 * (M + M.T))
    return m, gs, M, Bm, vec


def _pole_model(rng, k, n_states, n_occ, n_poles):
    """Energies, pair coefficients and a screened interaction made of poles:
    Lambda(w) = sum_s 2 O_s Z_s Z_s^T / (w^2 - O_s^2), Xi(w) = sum_s 2 O_s x_s / (w^2 - O_s^2)."""
    eps = np.sort(rng.uniform(-1.0, 0.6, n_states))
    eps[n_occ:] += 0.3                                  # a gap above the occupied states
    b = rng.standard_normal((n_states, k)) + 1j * rng.standard_normal((n_states, k))
    Om = rng.uniform(2.5, 4.0, n_poles)                 # above every residue frequency used
    Z = rng.standard_normal((n_poles, k))
    x = rng.uniform(0.1, 0.5, n_poles)

    def screen(w, real, eta):
        den = (w * w - Om * Om) if real else -(w * w + Om * Om)
        c = 2.0 * Om / den
        return np.einsum("s,si,sj->ij", c, Z, Z), float(np.sum(c * x))
    return eps, b, Om, Z, x, screen


def _pole_closed_form(E, n, eps, b, Om, Z, x, e_fermi, volume):
    """GW with W_p(w) = sum_s R_s 2 O_s / (w^2 - O_s^2): the real-axis integral closed in the
    upper half plane gives sum_m sum_s R_s^m / (E - e_m + O_s) for occupied m and
    / (E - e_m - O_s) for empty m (R_s^m = x_s delta_mn + |b_m . Z_s|^2 / Omega)."""
    tot = 0.0
    for mm, em in enumerate(eps):
        Rm = np.abs(b[mm] @ Z.T) ** 2 / volume + (x if mm == n else 0.0)
        sgn = 1.0 if em < e_fermi else -1.0
        tot += float(np.sum(Rm / (E - em + sgn * Om)))
    return tot


@pytest.mark.parametrize("seed", [1, 2])
def test_contour_deformation_equals_pole_sum(seed):
    """The imaginary-axis integral plus the residues of Eq. contourdeformationfinal equal
    the closed-form GW self-energy of a pole model, at E equal to a state's energy, between
    occupied states (residues of occupied states, f = -1), and above the Fermi level past
    an empty state (f = +1)."""
    rng = np.random.default_rng(seed)
    volume = 50.0
    eps, b, Om, Z, x, screen = _pole_model(rng, 4, 7, 4, 3)
    ef = 0.5 * (eps[3] + eps[4])
    n = 2
    for E in [eps[n], eps[n] - 0.05, eps[0] + 0.01, eps[3] + 1e-3, ef, eps[4] + 0.02, eps[5] + 0.3]:
        got = gw.sigma_c(E, n, eps, ef, b, screen, volume)
        want = _pole_closed_form(E, n, eps, b, Om, Z, x, ef, volume)
        assert abs(got.imag) <= 1e-14
        assert abs(got.real - want) <= 1e-10 * max(1.0, abs(want)), (E, got, want)


def test_mutation_residue_sign_caught():
    """A residue of the wrong sign (W_p at the real frequency negated) breaks the pole pin
    wherever a residue is taken."""
    rng = np.random.default_rng(3)
    volume = 50.0
    eps, b, Om, Z, x, screen = _pole_model(rng, 4, 7, 4, 3)
    ef = 0.5 * (eps[3] + eps[4])

    def bad(w, real, eta):
        lam, xi = screen(w, real, eta)
        return (-lam, -xi) if real else (lam, xi)
    E = eps[0] + 0.01
    want = _pole_closed_form(E, 0, eps, b, Om, Z, x, ef, volume)
    assert abs(gw.sigma_c(E, 0, eps, ef, b, screen, volume).real - want) <= 1e-10 * abs(want)
    assert abs(gw.sigma_c(E, 0, eps, ef, b, bad, volume).real - want) > 1e-3 * abs(want)


def test_pair_coefficients_reproduce_static_chi0bar(tiny):
    """The Adler-Wiser sum over the pair coefficients of every occupied state,
    -(4/Omega) sum_v sum_c Re[conj(b_ci) b_cj] / (e_c - e_v), is the static chi0bar of the
    response module's direct Sternheimer solve in the same basis."""
    m, gs, M, Bm, vec = tiny
    phi = vec[:, :6].T @ Bm
    n_v = TINY.n_v
    B = np.zeros((6, 6))
    for v in range(n_v):
        b = gw.pair_coefficients(m, gs, phi, v)[n_v:]
        d = gs.eps_all[n_v:] - gs.eps_all[v]
        B += np.real(b.conj().T @ (b / d[:, None]))
    B *= -4.0 / m.volume
    want = np.real(phi.conj() @ R.chi0bar_apply(m, gs, phi).T)
    assert np.max(np.abs(B - want)) <= 1e-11 * np.max(np.abs(want))


def _real_in_r(m, c):
    """The coefficient vector times the phase that makes its grid function real."""
    u = m.inv(c)
    k = np.argmax(np.abs(u))
    return c * np.exp(-1j * np.angle(u[k]))


def _scf_pair_errors(tiny):
    m, gs0, M, Bm, vec = tiny
    lam_body = R.chibar_from_chi0bar(0.5 * (M + M.T))
    n = TINY.n_v - 1
    gs = dataclasses.replace(gs0, C_all=gs0.C_all.copy())
    for col in [1, 2, n]:
        gs.C_all[:, col] = _real_in_r(m, gs.C_all[:, col])
    b = gw.pair_coefficients(m, gs, Bm, n)
    errs = []
    for mm in [1, 2, n]:
        got = gw.pair_strengths(b[mm:mm + 1], lam_body, 0.0, 0, m.volume)[0]
        um, un = m.inv(gs.C_all[:, mm]), m.inv(gs.C_all[:, n])
        x = m.coul * m.fwd(um * np.conj(un))[m.nz]
        chix = R.chibar_apply_scf(m, gs, x[None, :], tol=1e-13)[0]
        want = np.vdot(x, chix).real / m.volume
        errs.append(abs(got - want) / abs(want))
    return max(errs)


def test_screened_pair_element_by_the_self_consistent_response(tiny):
    """With the complete basis of S', (1/Omega) b^H Lambda b with the body-only Lambda =
    (1 - chi0bar)^-1 chi0bar is <psi_n psi_m| W_p(0) |psi_m psi_n> = (1/Omega) <x|chibar x>,
    x = sqrt(4 pi)/|G| Fwd(u_m conj(u_n)) on S', with chibar x from the self-consistent
    Hartree loop (a route that shares no step with the pair coefficients)."""
    assert _scf_pair_errors(tiny) <= 1e-9


def test_mutation_pair_volume_factor_caught(tiny, monkeypatch):
    """A pair strength with 1/Omega^2 instead of 1/Omega fails the self-consistent pin."""
    real = gw.pair_strengths
    monkeypatch.setattr(gw, "pair_strengths", lambda b_, lam, xi, n_, vol: real(b_, lam, xi, n_, vol * vol))
    assert _scf_pair_errors(tiny) > 0.5


def test_exchange_free_electrons_closed_form():
    """V = 0 with the plane waves as orbitals: for G = 0 and the six plane waves of the
    first shell occupied, the G = 0 state has Sigma_X = -I_BZ - 6 (4 pi / Omega) / |G_1|^2;
    an empty plane wave G_2 of the second shell has -(4 pi / Omega) sum_m 1/|G_2 - G_m|^2
    over the occupied m (no G = 0 term)."""
    L, n, ecut = (10.0, 10.0, 10.0), (16, 16, 16), 5.0
    m = R.make_model(L, n, ecut, np.zeros(n))
    order = np.argsort(m.kin, kind="stable")
    C_all = np.eye(m.n_pw, dtype=np.complex128)[:, order]
    eps_all = m.kin[order]
    n_v = 7
    gs = R.GroundState(eps_all[:n_v], C_all[:, :n_v].T.copy(), m.inv(C_all[:, :n_v].T), float(eps_all[n_v] - eps_all[6]),
                       eps_all, C_all, None)
    g1 = 2 * math.pi / 10.0
    want0 = -HW.bz_coulomb_integral(L) - 6 * (4 * math.pi / m.volume) / g1 ** 2
    assert abs(gw.sigma_x(m, gs, 0) - want0) <= 1e-12 * abs(want0)
    Gm = m.miller[order][:n_v] * g1
    j = n_v + 2                                   # a plane wave of the |G|^2 = 2 g1^2 shell
    G2 = m.miller[order][j] * g1
    assert abs(np.sum(G2 * G2) - 2 * g1 ** 2) <= 1e-12
    want2 = -(4 * math.pi / m.volume) * float(np.sum(1.0 / np.sum((G2[None, :] - Gm) ** 2, axis=1)))
    assert abs(gw.sigma_x(m, gs, j) - want2) <= 1e-12 * abs(want2)


def test_real_frequency_screening_by_dynamic_sternheimer(tiny):
    """B(w + i eta) at real frequencies, above and below the gap: each transition's
    [1/(D + w - i eta) + 1/(D - w - i eta)] / 2 is applied as two dense solves of the
    finite-frequency Sternheimer equation (A_v -/+ w - i eta) x = w_jv on range(P_c)."""
    m, gs, M, Bm, vec = tiny
    phi = vec[:, :4].T @ Bm
    scr = gw.Screening(m, gs, phi)
    from oracle.lanczos import rhs_vectors
    Wv = rhs_vectors(m, gs, phi)
    H = gs.H
    sigma = float(gs.eps[-1] - gs.eps[0] + 1.0)
    Pv = gs.C.T @ gs.C.conj()
    eta = 2e-3
    for w in [0.03, 0.2]:
        _, _, B = scr.blocks(w, True, eta)
        want = np.zeros((4, 4), dtype=np.complex128)
        for v in range(TINY.n_v):
            A = H - gs.eps[v] * np.eye(H.shape[0]) + sigma * Pv
            Y = Wv[:, v, :].T
            X = 0.5 * (np.linalg.solve(A + (w - 1j * eta) * np.eye(H.shape[0]), Y)
                       + np.linalg.solve(A - (w + 1j * eta) * np.eye(H.shape[0]), Y))
            G = Y.conj().T @ X                       # <w_i| g(A) |w_j>
            want += 0.5 * (G + G.T)
        want *= -4.0 / m.volume
        assert np.max(np.abs(B - want)) <= 1e-10 * np.max(np.abs(want)), w


def test_screening_imaginary_axis_matches_head_wings_module(tiny):
    """The transition table of Screening gives the F, U, B of headwings' sum over states."""
    m, gs, M, Bm, vec = tiny
    phi = vec[:, :3].T @ Bm
    scr = gw.Screening(m, gs, phi)
    F, U, B = HW.head_wings_body_sos(m, gs, phi, [0.0, 0.4])
    for f, u in enumerate([0.0, 0.4]):
        a = scr.blocks(u)
        for x, y in zip(a, (F[f], U[f], B[f])):
            assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(y))


def test_qp_solver_closed_form():
    """sigma(E) = a + c / (E - p): the QP equation is a quadratic, Z = 1/(1 + c/(e - p)^2),
    and the secant iteration from e and the linearised root reaches the nearer root."""
    e, a, c, p, vxc = -0.3, -0.2, 0.01, -0.8, 0.05
    out = gw.qp_solve(lambda E: a + c / (E - p), e, vxc, h=1e-4, tol=1e-13)
    z = 1.0 / (1.0 + c / (e - p) ** 2)
    assert abs(out["z"] - z) <= 1e-7
    assert abs(out["e_lin"] - (e + z * (a + c / (e - p) - vxc))) <= 1e-7
    # (E - e - a + vxc)(E - p) = c
    s = e + a - vxc
    roots = np.roots([1.0, -(s + p), s * p - c])
    want = roots[np.argmin(np.abs(roots - out["e_lin"]))]
    assert abs(out["e_qp"] - want) <= 1e-12
    assert abs(out["residual"]) <= 1e-12


def test_sigma_c_continuous_at_state_energies(tiny):
    """Sigma_C of the finite model is continuous where E crosses an occupied energy (the
    Lorentzian term jumps by S_m(0) and the residue switches on by -S_m(0))."""
    m, gs, M, Bm, vec = tiny
    phi = vec[:, :4].T @ Bm
    scr = gw.Screening(m, gs, phi)
    n = TINY.n_v - 1
    ef = 0.5 * (gs.eps_all[n] + gs.eps_all[n + 1])
    b = gw.pair_coefficients(m, gs, phi, n)
    for em in [gs.eps_all[n], gs.eps_all[n - 1]]:
        lo = gw.sigma_c(em - 1e-7, n, gs.eps_all, ef, b, scr.at, m.volume, eta=1e-3)
        at = gw.sigma_c(em, n, gs.eps_all, ef, b, scr.at, m.volume, eta=1e-3)
        hi = gw.sigma_c(em + 1e-7, n, gs.eps_all, ef, b, scr.at, m.volume, eta=1e-3)
        assert abs(lo.real - at.real) <= 1e-5 and abs(hi.real - at.real) <= 1e-5
