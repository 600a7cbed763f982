"""Serving on the GPU: jobs submitted to a running server (several running at once on
their own streams) give the same dielectric eigenvalues as the same job run alone on a
fresh context, in both mixed modes (FP32 and BF16x3 P_c products); latencies are
reported."""
import time

import numpy as np
import pytest

from paper_1501_03141_amd import inputs, pdep

pytestmark = pytest.mark.gpu


def _jobs():
    specs = [(24, 8, 16), (32, 16, 16), (24, 12, 16), (24, 8, 16), (32, 24, 16), (24, 16, 16)]
    out = []
    for k, (g, nv, npd) in enumerate(specs):
        Ledge = g * 20.0 / 48.0
        nw = int(round(64.0 * Ledge ** 3 / 8000.0))
        w = inputs.Workload(f"job{k}", (Ledge,) * 3, (g,) * 3, 12.0, nw, nv, npd, 1e-8, 2000 + k)
        out.append(w)
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [pdep.PDEP_MIXED_FP32, pdep.PDEP_MIXED_BF16X3])
def test_server_results_match_standalone(prec):
    jobs = _jobs()
    alone = []
    for w in jobs:
        V = inputs.vloc(w)
        with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=prec, cg_tol=w.cg_tol,
                          gap_min=1e-4, use_torch=False) as c:
            eps, _, _ = c.eigs(w.n_pdep, seed=w.seed, tol=1e-7, maxit=60)
        alone.append(eps)
    with pdep.Server(max_running=3) as srv:
        tickets = []
        t0 = time.perf_counter()
        for w in jobs:
            tickets.append(srv.submit(w.L, w.n, w.ecut, inputs.vloc(w), w.n_v, w.n_pdep, seed=w.seed,
                                      precision=prec, cg_tol=w.cg_tol, eig_tol=1e-7,
                                      gap_min=1e-4))
            time.sleep(0.05)
        for t in tickets:
            assert srv.wait(t, 300000) == pdep.JOB_DONE, srv.poll(t)
        wall = time.perf_counter() - t0
        st = srv.stats()
        lat = []
        for w, t, ref in zip(jobs, tickets, alone):
            state, res, eps = srv.poll(t)
            lat.append(res["latency_ms"])
            print(w.name, w.n, "N_v", w.n_v, "latency %.0f ms" % res["latency_ms"], "max|d eps|",
                  np.max(np.abs(eps - ref)))
            np.testing.assert_allclose(eps, ref, rtol=0, atol=1e-12)
    print("server stats", st, "wall %.2f s" % wall, "p50 %.0f ms" % np.percentile(lat, 50),
          "p99 %.0f ms" % np.percentile(lat, 99))
    assert st["peak_running"] >= 2
