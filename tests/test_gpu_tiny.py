"""GPU parity on the tiny workload (10^3 bohr, 16^3 grid, 5 Ha, 515 PW, N_v = 4):
the HIP path through the C ABI against the dense CPU FP64 oracle, element by element.

Tolerances: 1e-10 relative per perturbation in FP64 (the stated FP64 bar); mixed
precision is held to 1e-6 on the dielectric eigenvalues and a derived 1e-7 on
chi0bar columns (FP32 inner solves refined to the same FP64 residual tolerance)."""
import numpy as np
import pytest

from oracle import response as R
from paper_1501_03141_amd import inputs
from parity import relerr

pytestmark = pytest.mark.gpu

W = inputs.WORKLOADS["tiny"]


@pytest.fixture(scope="module")
def oracle_tiny():
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, W.n_v, full=True)
    lam, Phi, M = R.pdep_exact(m, gs, W.n_pdep)
    return V, m, gs, lam, Phi


def _ctx(V, gs=None, **kw):
    from paper_1501_03141_amd import pdep
    kw.setdefault("cg_tol", W.cg_tol)
    if gs is not None:
        kw["psi"] = gs.C
        kw["eps"] = gs.eps
    return pdep.Context(W.L, W.n, W.ecut, V, W.n_v, **kw)


_relerr = relerr


def test_miller_list_identical(oracle_tiny):
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, gs) as c:
        assert np.array_equal(c.miller(), m.miller)
        assert c.n_pw == m.n_pw == 515


def test_chi0_apply_fp64_parity(oracle_tiny):
    """9 perturbations = 36 Sternheimer systems: one full 32-row GEMM tile plus a ragged tail."""
    V, m, gs, lam, Phi = oracle_tiny
    phi = inputs.trial_block(m.miller[m.nz], 9, 101)
    want = R.chi0bar_apply(m, gs, phi)
    with _ctx(V, gs) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("stats", st, "relerr", err)
    assert st["n_notconv"] == 0 and st["max_rel_residual"] <= W.cg_tol
    assert err <= 1e-10


@pytest.mark.parametrize("tile", [4, 12])
def test_chi0_apply_tiled_identical(oracle_tiny, tile):
    """Forcing perturbation tiles (1 and 3 perturbations per tile, ragged last tile)
    gives the same result as the oracle."""
    V, m, gs, lam, Phi = oracle_tiny
    phi = inputs.trial_block(m.miller[m.nz], 7, 102)
    want = R.chi0bar_apply(m, gs, phi)
    with _ctx(V, gs, rhs_tile=tile) as c:
        got, st = c.chi0_apply(phi)
    assert _relerr(got, want) <= 1e-10


def test_chi0_apply_raw_parity(oracle_tiny):
    V, m, gs, lam, Phi = oracle_tiny
    dv = inputs.random_grid_potentials(W.n, 3, 103)
    want = np.stack([R.chi0_real(m, gs, dv[i]) for i in range(3)])
    with _ctx(V, gs) as c:
        got, st = c.chi0_apply_raw(dv)
    assert _relerr(got, want) <= 1e-10


def test_uniform_potential_gives_zero_response(oracle_tiny):
    """Degenerate case: b = 0 for every band; the solver returns x = 0 without iterating."""
    V, m, gs, lam, Phi = oracle_tiny
    dv = np.full((2, m.n_grid), 0.7)
    with _ctx(V, gs) as c:
        got, st = c.chi0_apply_raw(dv)
    assert np.max(np.abs(got)) < 1e-13
    assert st["cg_iter_max"] == 0


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_zero_and_ordinary_right_hand_sides_in_one_block(oracle_tiny, mode):
    """Degenerate rows beside ordinary ones: a uniform potential (b = 0 for all its
    bands) between two random ones, so the refinement updates only part of the rows
    from its first step on (x starts from a zero fill instead of being written by the
    first update).  The uniform potential's response is exactly zero and the others
    match the oracle."""
    V, m, gs, lam, Phi = oracle_tiny
    from paper_1501_03141_amd import pdep
    dv = inputs.random_grid_potentials(W.n, 3, 106)
    dv[1] = 0.7
    want = np.stack([R.chi0_real(m, gs, dv[i]) for i in (0, 2)])
    kw = {} if mode == "fp64" else {"precision": pdep.PDEP_MIXED_BF16X3, "cg_tol": 1e-10}
    with _ctx(V, gs, **kw) as c:
        got, st = c.chi0_apply_raw(dv)
    assert st["n_notconv"] == 0
    assert np.max(np.abs(got[1])) < 1e-13
    err = _relerr(got[[0, 2]], want)
    print(mode, "stats", st, "relerr", err)
    assert err <= (1e-10 if mode == "fp64" else 1e-8)


def test_empty_block(oracle_tiny):
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, gs) as c:
        got, st = c.chi0_apply(np.zeros((0, m.n_pw - 1), complex))
    assert got.shape == (0, m.n_pw - 1)


def test_device_pointers_match_host(oracle_tiny):
    import torch
    V, m, gs, lam, Phi = oracle_tiny
    phi = inputs.trial_block(m.miller[m.nz], 3, 104)
    with _ctx(V, gs) as c:
        host, _ = c.chi0_apply(phi)
    with _ctx(V, gs, device_ptrs=True) as c:
        dev, _ = c.chi0_apply(torch.from_numpy(phi).cuda())
        torch.cuda.synchronize()
    assert np.array_equal(dev.cpu().numpy(), host)


@pytest.mark.parametrize("mode", ["mixed_fp32", "bf16x3"])
def test_mixed_precision_parity(oracle_tiny, mode):
    """Both mixed modes refine to the same FP64 residual tolerance, so both meet the
    same bar against the oracle (BF16x3 only changes the inner P_c products)."""
    V, m, gs, lam, Phi = oracle_tiny
    from paper_1501_03141_amd import pdep
    prec = {"mixed_fp32": pdep.PDEP_MIXED_FP32, "bf16x3": pdep.PDEP_MIXED_BF16X3}[mode]
    phi = inputs.trial_block(m.miller[m.nz], 5, 105)
    want = R.chi0bar_apply(m, gs, phi)
    with _ctx(V, gs, precision=prec, cg_tol=1e-10) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("mixed stats", st, "relerr", err)
    assert st["refine_steps"] >= 2
    assert err <= 1e-8


def test_ground_state_matches_dense_eigh(oracle_tiny):
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, None, gs_tol=1e-11) as c:
        eps, psi = c.orbitals()
        assert c.gs_residual <= 1e-11
        assert abs(c.gap - gs.gap) < 1e-10
    assert np.max(np.abs(eps - gs.eps)) < 1e-10
    # same occupied subspace: projector difference
    P1 = psi.T @ psi.conj()
    P2 = gs.C.T @ gs.C.conj()
    assert np.max(np.abs(P1 - P2)) < 1e-9


def test_pdep_eigs_exact(oracle_tiny):
    """Davidson from the library's own random start reaches the exact lowest N_pdep
    eigenvalues of the full chi0bar matrix."""
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, gs) as c:
        eps, basis, st = c.eigs(W.n_pdep, seed=7, tol=1e-10, maxit=100, n_buffer=4, want_basis=True)
    print("eig stats", st)
    want = np.sort(1.0 - lam)[::-1]
    assert np.max(np.abs(eps - want) / want) <= 1e-10
    # eigenvectors: chi0bar phi = lambda phi by the oracle, and orthonormal
    A = R.chi0bar_apply(m, gs, basis)
    res = np.linalg.norm(A - (1.0 - eps)[:, None] * basis, axis=1)
    assert res.max() <= 1e-9
    assert np.allclose(basis.conj() @ basis.T, np.eye(W.n_pdep), atol=1e-10)


def test_pdep_eigs_seeded_block(oracle_tiny):
    """Start from the seeded trial block (the same input both sides see)."""
    V, m, gs, lam, Phi = oracle_tiny
    phi0 = inputs.trial_block(m.miller[m.nz], W.n_pdep, W.seed)
    with _ctx(V, gs) as c:
        eps, _, st = c.eigs(W.n_pdep, phi0=phi0, tol=1e-10, maxit=100)
    want = np.sort(1.0 - lam)[::-1]
    assert np.max(np.abs(eps - want)) <= 1e-10 * want.max()


@pytest.mark.parametrize("n_pdep,n_buffer", [(2, 6), (4, 8)])
def test_pdep_eigs_buffer_wider_than_block(oracle_tiny, n_pdep, n_buffer):
    """More buffer vectors than wanted pairs: after a restart the search space holds the
    n_pdep + n_buffer Ritz vectors and their residuals, and the library sizes it for
    that; the wanted eigenvalues are still the exact lowest ones."""
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, gs) as c:
        eps, _, st = c.eigs(n_pdep, seed=9, tol=1e-10, maxit=100, n_buffer=n_buffer)
        with pytest.raises(Exception) as e:
            c.eigs(n_pdep, seed=9, tol=1e-10, maxit=5, n_buffer=n_buffer,
                   max_subspace=2 * (n_pdep + n_buffer) - 1)
        assert getattr(e.value, "code", None) == -1
    print("eig stats", st)
    want = np.sort(1.0 - lam[:n_pdep])[::-1]
    assert np.max(np.abs(eps - want) / want) <= 1e-10


def test_pdep_eigs_reports_unconverged_solves(oracle_tiny):
    """Sternheimer solves capped below the tolerance make pdep_eigs return
    PDEP_ENOTCONV (outputs and the count of such systems still filled)."""
    V, m, gs, lam, Phi = oracle_tiny
    from paper_1501_03141_amd import pdep
    with _ctx(V, gs, cg_maxit=2, refine_maxit=1) as c:
        with pytest.raises(pdep.PdepError) as e:
            c.eigs(4, seed=7, tol=1e-10, maxit=2)
        assert e.value.code == pdep.PDEP_ENOTCONV
        eps, _, st = c.eigs(4, seed=7, tol=1e-10, maxit=2, allow_notconv=True)
    assert st["n_notconv"] > 0 and np.all(np.isfinite(eps))


@pytest.mark.parametrize("mode", ["mixed_fp32", "bf16x3"])
def test_pdep_eigs_mixed_within_1e6(oracle_tiny, mode):
    V, m, gs, lam, Phi = oracle_tiny
    from paper_1501_03141_amd import pdep
    prec = {"mixed_fp32": pdep.PDEP_MIXED_FP32, "bf16x3": pdep.PDEP_MIXED_BF16X3}[mode]
    with _ctx(V, gs, precision=prec, cg_tol=1e-8) as c:
        eps, _, st = c.eigs(W.n_pdep, seed=7, tol=1e-7, maxit=100, n_buffer=4)
    want = np.sort(1.0 - lam)[::-1]
    assert np.max(np.abs(eps - want)) <= 1e-6


def _mirror_defect(psi):
    """max |c_{-G} - conj c_G| over rows (-G_k is entry npw - 1 - k of the sphere order)."""
    return np.max(np.abs(psi[:, ::-1] - psi.conj()))


def test_orbitals_real_in_r_from_ground_state(oracle_tiny):
    """The library's orbitals are Hermitian-symmetric (real in r) exactly and span the
    oracle's occupied subspace with its eigenvalues."""
    V, m, gs, lam, Phi = oracle_tiny
    with _ctx(V, None, gs_tol=1e-11) as c:
        eps, psi = c.orbitals()
    assert np.array_equal(m.miller[::-1], -m.miller)
    assert _mirror_defect(psi) == 0.0
    assert np.max(np.abs(eps - gs.eps)) < 1e-10
    assert np.max(np.abs(psi.conj() @ psi.T - np.eye(W.n_v))) < 1e-12
    assert np.max(np.abs(psi.T @ psi.conj() - gs.C.T @ gs.C.conj())) < 1e-9


def test_orbitals_real_in_r_from_caller():
    """Caller orbitals with arbitrary complex phases and a unitary mix inside the
    occupied space: the context keeps the subspace and returns real-in-r Ritz vectors
    with the same energies."""
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, W.n_v, full=True)
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((W.n_v, W.n_v)) + 1j * rng.standard_normal((W.n_v, W.n_v)))
    C = Q.T @ gs.C                                  # rows: unitary mixtures of the eigenvectors
    with _ctx(V, None, psi=C, eps=gs.eps) as c:
        eps, psi = c.orbitals()
    assert _mirror_defect(psi) == 0.0
    assert np.max(np.abs(eps - gs.eps)) < 1e-12
    assert np.max(np.abs(psi.T @ psi.conj() - gs.C.T @ gs.C.conj())) < 1e-12
    # each returned row is an eigenvector of the oracle H
    H = R.hamiltonian(m)
    res = np.linalg.norm(psi @ H.T - eps[:, None] * psi, axis=1)
    assert res.max() < 1e-10


def test_caller_orbitals_not_closed_under_conjugation_rejected():
    """One orbital u + i v built from two real-in-r functions: its conjugate u - i v is
    not in its span, so it cannot be the occupied space of a real H."""
    from paper_1501_03141_amd import pdep
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, W.n_v, full=True)
    sym = 0.5 * (gs.C + gs.C[:, ::-1].conj())        # real-in-r parts
    u = sym[0] / np.linalg.norm(sym[0])
    v = sym[1] - (u.conj() @ sym[1]) * u
    v /= np.linalg.norm(v)
    one = ((u + 1j * v) / np.sqrt(2.0))[None, :]
    with pytest.raises(pdep.PdepError):
        pdep.Context(W.L, W.n, W.ecut, V, 1, cg_tol=W.cg_tol, psi=one, eps=gs.eps[:1])


@pytest.mark.parametrize("mode", ["mixed_fp32", "bf16x3"])
def test_odd_row_count_parity(mode):
    """N_v = 1 and 3 perturbations: 3 Sternheimer rows, so the paired transforms of the
    mixed inner solve carry a lone last row."""
    from paper_1501_03141_amd import pdep
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, 1, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 3, 211)
    want = R.chi0bar_apply(m, gs, phi)
    prec = {"mixed_fp32": pdep.PDEP_MIXED_FP32, "bf16x3": pdep.PDEP_MIXED_BF16X3}[mode]
    with pdep.Context(W.L, W.n, W.ecut, V, 1, precision=prec, cg_tol=1e-10, psi=gs.C[:1], eps=gs.eps[:1]) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("odd rows", st, "relerr", err)
    assert st["n_rhs"] == 3 and st["n_notconv"] == 0
    assert err <= 1e-8


@pytest.mark.parametrize("mode", ["bf16x3"])
def test_fine_grid_runtime_radius_parity(mode):
    """The tiny sphere (5 Ha, 10 bohr) on a 48^3 grid: the register slab pass runs with
    a run-time sphere radius (|mx| <= 5 on 48-point lines, not the compiled one)."""
    from paper_1501_03141_amd import pdep
    Wf = inputs.Workload("tiny_fine", (10.0,) * 3, (48,) * 3, 5.0, 4, 4, 8, 1e-10, 1511)
    V = inputs.vloc(Wf)
    m = R.make_model(Wf.L, Wf.n, Wf.ecut, V, naive=False)
    gs = R.ground_state(m, Wf.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 3, 213)
    want = R.chi0bar_apply(m, gs, phi)
    with pdep.Context(Wf.L, Wf.n, Wf.ecut, V, Wf.n_v, precision=pdep.PDEP_MIXED_BF16X3, cg_tol=1e-10,
                      psi=gs.C, eps=gs.eps) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("fine grid", st, "relerr", err)
    assert st["n_notconv"] == 0
    assert err <= 1e-8


@pytest.mark.parametrize("grid,cell,ecut", [((24, 24, 24), (10.0, 10.0, 10.0), 5.0),
                                            ((64, 64, 16), (12.0, 12.0, 3.0), 4.0)])
@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_lane_quad_grids_parity(grid, cell, ecut, mode):
    """The FP64 slab, density and forward passes with lines on lane quads at the line
    lengths the medium tests do not reach: 24 (two slabs per workgroup) and 64 (one slab,
    a 16-point z axis), in the FP64 mode and as the refinement of the BF16x3 mode."""
    from paper_1501_03141_amd import pdep
    Wg = inputs.Workload("quad_grid", cell, grid, ecut, 2, 4, 6, 1e-10, 1513)
    V = inputs.vloc(Wg)
    m = R.make_model(Wg.L, Wg.n, Wg.ecut, V, naive=False)
    gs = R.ground_state(m, Wg.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 5, 217)
    want = R.chi0bar_apply(m, gs, phi)
    prec = pdep.PDEP_FP64 if mode == "fp64" else pdep.PDEP_MIXED_BF16X3
    with pdep.Context(Wg.L, Wg.n, Wg.ecut, V, Wg.n_v, precision=prec, cg_tol=1e-10, psi=gs.C,
                      eps=gs.eps) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print(grid, mode, "npw", m.miller.shape[0], st, "relerr", err)
    assert st["n_notconv"] == 0
    assert err <= (1e-10 if mode == "fp64" else 1e-8)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_odd_band_count_parity(mode):
    """N_v = 5: an odd number of bands, so the paired right-hand-side and density passes
    end every perturbation with a band transformed alone."""
    from paper_1501_03141_amd import pdep
    Wo = inputs.Workload("tiny_odd", W.L, W.n, W.ecut, 4, 5, 8, 1e-10, 1517)
    V = inputs.vloc(Wo)
    m = R.make_model(Wo.L, Wo.n, Wo.ecut, V)
    gs = R.ground_state(m, Wo.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 3, 223)
    want = R.chi0bar_apply(m, gs, phi)
    prec = pdep.PDEP_FP64 if mode == "fp64" else pdep.PDEP_MIXED_BF16X3
    with pdep.Context(Wo.L, Wo.n, Wo.ecut, V, Wo.n_v, precision=prec, cg_tol=1e-10, psi=gs.C, eps=gs.eps,
                      gap_min=1e-6) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("N_v 5", mode, "gap", gs.gap, st, "relerr", err)
    assert st["n_notconv"] == 0
    assert err <= (1e-10 if mode == "fp64" else 1e-8)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_unequal_xy_grid_parity(mode):
    """A 24 x 32 x 16 grid (10 x 13.3 x 6.7 bohr): NX != NY, so every slab pass (H, density,
    right-hand sides) takes the LDS Stockham kernels instead of the register and lane-quad
    ones."""
    from paper_1501_03141_amd import pdep
    Wu = inputs.Workload("xy_unequal", (10.0, 40.0 / 3.0, 20.0 / 3.0), (24, 32, 16), 5.0, 3, 4, 6, 1e-10, 1519)
    V = inputs.vloc(Wu)
    m = R.make_model(Wu.L, Wu.n, Wu.ecut, V, naive=False)
    gs = R.ground_state(m, Wu.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 3, 227)
    want = R.chi0bar_apply(m, gs, phi)
    prec = pdep.PDEP_FP64 if mode == "fp64" else pdep.PDEP_MIXED_BF16X3
    with pdep.Context(Wu.L, Wu.n, Wu.ecut, V, Wu.n_v, precision=prec, cg_tol=1e-10, psi=gs.C, eps=gs.eps,
                      gap_min=1e-6) as c:
        assert np.array_equal(c.miller(), m.miller)
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("24x32x16", mode, "npw", m.miller.shape[0], "gap", gs.gap, st, "relerr", err)
    assert st["n_notconv"] == 0
    assert err <= (1e-10 if mode == "fp64" else 1e-8)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_runtime_sizes_parity(mode):
    """A 36 x 36 x 18 grid: line lengths with no compiled form, so the slab, stick and
    density passes all run their run-time-size kernels."""
    from paper_1501_03141_amd import pdep
    Wr = inputs.Workload("runtime_sizes", (15.0, 15.0, 7.5), (36, 36, 18), 5.0, 3, 4, 6, 1e-10, 1521)
    V = inputs.vloc(Wr)
    m = R.make_model(Wr.L, Wr.n, Wr.ecut, V, naive=False)
    gs = R.ground_state(m, Wr.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 3, 229)
    want = R.chi0bar_apply(m, gs, phi)
    prec = pdep.PDEP_FP64 if mode == "fp64" else pdep.PDEP_MIXED_BF16X3
    with pdep.Context(Wr.L, Wr.n, Wr.ecut, V, Wr.n_v, precision=prec, cg_tol=1e-10, psi=gs.C, eps=gs.eps,
                      gap_min=1e-6) as c:
        got, st = c.chi0_apply(phi)
    err = _relerr(got, want)
    print("36x36x18", mode, "npw", m.miller.shape[0], "gap", gs.gap, st, "relerr", err)
    assert st["n_notconv"] == 0
    assert err <= (1e-10 if mode == "fp64" else 1e-8)


@pytest.mark.parametrize("mode", ["fp64", "bf16x3"])
def test_free_electron_golden(mode):
    """V = 0 with one occupied plane wave: the library's chi0bar on cosine-wave
    perturbations equals the closed-form eigenvalues stored in tests/golden."""
    import os
    from paper_1501_03141_amd import pdep
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "free_electron_chi0bar.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    golden = [(tuple(int(x) for x in r[:3]), float(r[3])) for r in rows]
    V0 = np.zeros(W.n)
    m = R.make_model(W.L, W.n, W.ecut, V0)
    # the exact occupied orbital: the G = 0 plane wave (a computed one would carry its
    # eigensolver residual into the projector)
    psi = np.zeros((1, m.miller.shape[0]), dtype=complex)
    psi[0, int(np.where(~np.any(m.miller != 0, axis=1))[0][0])] = 1.0
    prec = pdep.PDEP_FP64 if mode == "fp64" else pdep.PDEP_MIXED_BF16X3
    with pdep.Context(W.L, W.n, W.ecut, V0, 1, precision=prec, cg_tol=1e-12 if mode == "fp64" else 1e-10,
                      psi=psi, eps=np.zeros(1)) as c:
        sp = c.miller()
        assert np.array_equal(sp, m.miller)
        sp = sp[np.any(sp != 0, axis=1)]
        index = {tuple(int(x) for x in g): i for i, g in enumerate(sp)}
        # one cosine wave per listed +-G pair (each pair once)
        seen, phis, lams = set(), [], []
        for g, lam in golden:
            if g in seen:
                continue
            seen.add(g)
            seen.add(tuple(-x for x in g))
            phi = np.zeros(sp.shape[0], dtype=complex)
            phi[index[g]] = 1.0
            phi[index[tuple(-x for x in g)]] = 1.0
            phis.append(phi)
            lams.append(lam)
        phis = np.array(phis)
        got, st = c.chi0_apply(phis)
    err = np.max(np.abs(got - np.array(lams)[:, None] * phis)) / np.max(np.abs(lams))
    print("free electron", mode, len(lams), "pairs", st, "max rel err", err)
    assert st["n_notconv"] == 0
    assert err <= (1e-10 if mode == "fp64" else 1e-8)
