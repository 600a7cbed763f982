"""GPU parity of the q -> 0 head and wings of chi0bar at imaginary frequencies and of
Eq. Bfinal (Table limitqchi0; Eqs. commu, finalF, finalU1, finalU2, finalB, Bfinal) on the
tiny workload: against the oracle's sums over empty states (dipole elements through
the commutator) and its Lambda, Xi.  Chains as long as the space they explore are
exact: bar 1e-9 relative to the largest element (FP64, dipole solves to 1e-13); 40-step
chains are the method's approximation, bounded at 1e-4."""
import numpy as np
import pytest

from oracle import headwings as HW
from oracle import response as R
from paper_1501_03141_amd import inputs, pdep

pytestmark = pytest.mark.gpu

W = inputs.WORKLOADS["tiny"]
FREQ = np.array([0.0, 0.7, 5.0])


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_head_wings_parity():
    V = inputs.vloc(W)
    m = R.make_model(W.L, W.n, W.ecut, V)
    gs = R.ground_state(m, W.n_v, full=True)
    phi = inputs.trial_block(m.miller[m.nz], 5, 801)
    F, U, B = HW.head_wings_body_sos(m, gs, phi, FREQ)
    with pdep.Context(W.L, W.n, W.ecut, V, W.n_v, cg_tol=1e-13, psi=gs.C, eps=gs.eps) as c:
        full, st = c.head_wings(phi, FREQ, n_lanczos=m.n_pw)
        short, _ = c.head_wings(phi, FREQ, n_lanczos=40)
    print("stats", st)
    errs = {k: _rel(full[k], ref) for k, ref in (("F", F), ("U", U), ("B", B))}
    print("full chains vs sums over states", errs)
    assert max(errs.values()) <= 1e-9
    for f in range(FREQ.size):
        lam, xi, k = HW.lambda_xi(F[f], U[f], B[f], W.L)
        e_l, e_x = _rel(full["Lambda"][f], lam), abs(full["Xi"][f] - xi) / abs(xi)
        print("u", FREQ[f], "Lambda", e_l, "Xi", e_x, "k", k)
        assert e_l <= 1e-9 and e_x <= 1e-9
    e40 = {k: _rel(short[k], ref) for k, ref in (("F", F), ("U", U), ("B", B))}
    print("40-step chains vs exact", e40)
    assert max(e40.values()) <= 1e-4
