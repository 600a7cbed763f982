"""GPU parity of the reducible polarizability (RPA, Hartree response only) on the tiny
workload: chibar_apply against the oracle's (1 - chi0bar)^-1 chi0bar on the full
chi0bar matrix (Eq. linearalgebrachichi0; the oracle's self-consistent DFPT loop is
pinned equal to it), the free-electron closed form lambda/(1 - lambda), and the PDEP
Davidson run on chibar (Fig. pdepscheme, right panel) against the exact dielectric
eigenvalues.  Bars: FP64 1e-10 per column, BF16x3 1e-8 (error measure of the parity
module)."""
import os

import numpy as np
import pytest

from oracle import response as R
from paper_1501_03141_amd import inputs, pdep
from parity import relerr

pytestmark = pytest.mark.gpu

W = inputs.WORKLOADS["tiny"]


@pytest.fixture(scope="module")
def oracle_tiny():
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, W.n_v, full=True)
    lam, Phi, M = R.pdep_exact(m, gs, W.n_pdep)
    return V, m, gs, lam, M


def _reducible(m, M, phi):
    Bm = R.real_basis(m)
    a = np.real(Bm.conj() @ phi.T)
    return (R.chibar_from_chi0bar(M) @ a).T @ Bm


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_chibar_apply_parity(oracle_tiny, mode):
    """7 perturbations (one of them zero: its response is zero without a pass)."""
    V, m, gs, lam, M = oracle_tiny
    phi = inputs.trial_block(m.miller[m.nz], 7, 401)
    phi[3] = 0.0
    want = _reducible(m, M, phi)
    prec, cg_tol, tol, bar = ((pdep.PDEP_FP64, 1e-13, 2e-12, 1e-10) if mode == "fp64"
                              else (pdep.PDEP_MIXED_BF16X3, 1e-10, 1e-9, 1e-8))
    with pdep.Context(W.L, W.n, W.ecut, V, W.n_v, precision=prec, cg_tol=cg_tol, psi=gs.C, eps=gs.eps) as c:
        got, st = c.chibar_apply(phi, tol=tol, maxit=100)
    print("chibar", mode, st)
    assert np.all(got[3] == 0)
    keep = [0, 1, 2, 4, 5, 6]
    err = relerr(got[keep], want[keep])
    print("relerr", err)
    assert st["n_notconv"] == 0 and st["cg_notconv"] == 0 and st["max_rel_residual"] <= tol
    assert err <= bar
    # chibar is negative definite with eigenvalues in (-1, 0]: <phi, chibar phi> < 0
    assert np.all(np.real(np.sum(phi[keep].conj() * got[keep], axis=1)) < 0)


def test_chibar_free_electron_closed_form():
    """V = 0, one occupied plane wave (the exact orbital): chibar on a cosine wave at G
    is lambda_G / (1 - lambda_G) times it, lambda_G the closed-form values in
    tests/golden (lambda_G = -32 pi / (Omega |G|^4))."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "free_electron_chi0bar.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    golden = [(tuple(int(x) for x in r[:3]), float(r[3])) for r in rows]
    V0 = np.zeros(W.n)
    m = R.make_model(W.L, W.n, W.ecut, V0)
    psi = np.zeros((1, m.miller.shape[0]), dtype=complex)
    psi[0, int(np.where(~np.any(m.miller != 0, axis=1))[0][0])] = 1.0
    with pdep.Context(W.L, W.n, W.ecut, V0, 1, cg_tol=1e-13, psi=psi, eps=np.zeros(1)) as c:
        sp = c.miller()
        sp = sp[np.any(sp != 0, axis=1)]
        index = {tuple(int(x) for x in g): i for i, g in enumerate(sp)}
        seen, phis, mus = set(), [], []
        for g, lam in golden:
            if g in seen:
                continue
            seen.update({g, tuple(-x for x in g)})
            phi = np.zeros(sp.shape[0], dtype=complex)
            phi[index[g]] = phi[index[tuple(-x for x in g)]] = 1.0
            phis.append(phi)
            mus.append(lam / (1.0 - lam))
        phis = np.array(phis)
        got, st = c.chibar_apply(phis, tol=1e-12, maxit=50)
    err = np.max(np.abs(got - np.array(mus)[:, None] * phis)) / np.max(np.abs(mus))
    print("free electron chibar", st, "max rel err", err)
    assert err <= 1e-10


@pytest.mark.timeout(600)
def test_pdep_eigs_on_chibar(oracle_tiny):
    """Davidson on chibar (every application self-consistent) from the library's random
    start gives the same dielectric eigenvalues as the exact diagonalisation of chi0bar,
    eps_i = 1 - lambda_i; eps^-1 = 1/eps_i (Eq. epsilonandchi)."""
    V, m, gs, lam, M = oracle_tiny
    with pdep.Context(W.L, W.n, W.ecut, V, W.n_v, cg_tol=1e-13, psi=gs.C, eps=gs.eps) as c:
        eps, basis, st = c.eigs(4, seed=17, tol=1e-9, maxit=60, n_buffer=4, reducible=True, want_basis=True)
    print("reducible eig stats", st, eps)
    want = np.sort(1.0 - lam[:4])[::-1]
    assert st["scr_passes"] > 0 and st["n_notconv"] == 0
    assert np.max(np.abs(eps - want) / want) <= 1e-9
    assert np.max(np.abs(1.0 / eps - R.eps_inverse_eigenvalues(lam[:4]))) <= 1e-9   # lam ascending
    # the eigenvectors are those of chi0bar as well (same eigenvectors, Eq. linearalgebrachichi0)
    A = R.chi0bar_apply(m, gs, basis)
    res = np.linalg.norm(A - (1.0 - eps)[:, None] * basis, axis=1)
    assert res.max() <= 1e-7
