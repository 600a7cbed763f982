"""Batched chi0 requests on a resident system (pdep_server_add_system, pdep_submit_chi0):
requests queued together run as one chi0_apply over their concatenated perturbations,
and every request's result equals chi0bar applied to its perturbations alone on a fresh
context of the same system (Sec. 2.3, Eqs. stern, deltani, chiisamatrixinpdep), in FP64
and in the BF16x3 mixed mode.  The two differ only through the rounding of the
transforms that pair rows, so the bar is set by the CG tolerance of the system."""
import numpy as np
import pytest

from paper_1501_03141_amd import inputs, pdep

pytestmark = pytest.mark.gpu

from parity import relerr   # noqa: E402


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name,prec,tol,bar", [("tiny", pdep.PDEP_FP64, 1e-12, 1e-10),
                                                ("tiny", pdep.PDEP_MIXED_BF16X3, 1e-10, 1e-8),
                                                ("small", pdep.PDEP_MIXED_BF16X3, 1e-10, 1e-8)])
def test_batched_requests_match_alone(name, prec, tol, bar):
    w = inputs.WORKLOADS[name]
    V = inputs.vloc(w)
    with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=prec, cg_tol=tol, use_torch=False) as c:
        miller = c.miller()
        nz = np.any(miller != 0, axis=1)
        sizes = [2, 1, 3, 2, 1]
        phis = [inputs.trial_block(miller[nz], k, w.seed + 7 * j) for j, k in enumerate(sizes)]
        alone = [c.chi0_apply(p)[0] for p in phis]
    with pdep.Server(max_running=1) as s:
        sid = s.add_system(w.L, w.n, w.ecut, V, w.n_v, max_batch_pert=0, precision=prec, cg_tol=tol)
        tickets = [s.submit_chi0(sid, p) for p in phis]
        got, recs = [], []
        for t in tickets:
            assert s.wait(t, 120000) == pdep.JOB_DONE
            state, res, out = s.poll_chi0(t)
            assert state == pdep.JOB_DONE and res["status"] == 0, res
            got.append(out)
            recs.append(res)
        s.remove_system(sid)
    # the requests queued behind the first one ran as one batch
    assert max(r["batch_requests"] for r in recs) > 1, recs
    for p, a, g, r in zip(phis, alone, got, recs):
        assert g.shape == p.shape and r["n_pert"] == p.shape[0]
        err = relerr(g, a)
        assert err <= bar, (name, prec, err, r["batch_requests"])
        print(f"{name} prec {prec}: request of {p.shape[0]} in a batch of {r['batch_requests']} requests "
              f"({r['batch_pert']} perturbations): max rel diff vs alone {err:.2e}")


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec,tol", [(pdep.PDEP_FP64, 1e-12), (pdep.PDEP_MIXED_BF16X3, 1e-10)])
def test_pdep_on_resident_system_matches_standalone(prec, tol):
    """pdep_submit_eigs on a resident system (its orbitals reused, queued behind a chi0
    batch) gives the dielectric eigenvalues of pdep_eigs on a fresh context of the same
    system with the same seeded start (Sec. 2.3, Fig. pdepscheme)."""
    w = inputs.WORKLOADS["tiny"]
    V = inputs.vloc(w)
    with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=prec, cg_tol=tol, use_torch=False) as c:
        alone, _, _ = c.eigs(w.n_pdep, seed=w.seed, tol=1e-9, maxit=60)
        miller = c.miller()
    nz = np.any(miller != 0, axis=1)
    phi = inputs.trial_block(miller[nz], 3, w.seed + 1)
    with pdep.Server(max_running=1) as s:
        sid = s.add_system(w.L, w.n, w.ecut, V, w.n_v, precision=prec, cg_tol=tol)
        tc = s.submit_chi0(sid, phi)
        te = s.submit_eigs(sid, w.n_pdep, seed=w.seed, eig_tol=1e-9, eig_maxit=60)
        assert s.wait(tc, 120000) == pdep.JOB_DONE
        assert s.wait(te, 120000) == pdep.JOB_DONE
        state, res, eps = s.poll_eigs(te)
        assert state == pdep.JOB_DONE and res["status"] == 0, res
        s.remove_system(sid)
    err = float(np.max(np.abs(eps - alone) / np.abs(alone)))
    print(f"prec {prec}: resident-system PDEP vs standalone, max rel diff {err:.2e}, "
          f"{res['eig_iterations']} iterations")
    assert err <= 1e-12, (eps, alone)
