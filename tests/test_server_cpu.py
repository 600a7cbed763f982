"""Serving loop on the CPU with the fake executor (no GPU work): admission under the
HBM budget, submission-order start, back-pressure, rejection of jobs that can never
fit, failure isolation and thread-safe concurrent submission."""
import threading

import numpy as np
import pytest

from paper_1501_03141_amd import pdep

CELL = dict(L=(10.0, 10.0, 10.0), n=(16, 16, 16), ecut=5.0)


def _submit(srv, seed, n_v=4, n_pdep=8, **kw):
    V = np.zeros(16 ** 3)
    return srv.submit(CELL["L"], CELL["n"], CELL["ecut"], V, n_v, n_pdep, seed=seed, **kw)


def _estimate():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s:
        t = _submit(s, 1)
        s.wait(t)
        return s.poll(t)[1]["hbm_estimate"]


def test_all_jobs_complete_with_results():
    with pdep.Server(max_running=3, fake=True, fake_ms_per_gb=20.0) as s:
        tickets = [_submit(s, k) for k in range(10)]
        for t in tickets:
            assert s.wait(t, 10000) == pdep.JOB_DONE
        for k, t in enumerate(tickets):
            state, res, eps = s.poll(t)
            assert state == pdep.JOB_DONE and res["status"] == 0
            np.testing.assert_allclose(eps, 1.0 + (k % 97 + 1) / np.arange(1, 9))
            assert res["latency_ms"] >= res["run_ms"] >= 0
        st = s.stats()
        assert st["done"] == 10 and st["failed"] == 0 and st["peak_running"] <= 3


def test_admission_respects_budget():
    est = _estimate()
    budget = int(2.5 * est)               # room for two jobs at a time, not three
    with pdep.Server(max_running=6, hbm_budget=budget, fake=True, fake_ms_per_gb=40.0) as s:
        tickets = [_submit(s, k) for k in range(8)]
        for t in tickets:
            s.wait(t, 20000)
        st = s.stats()
    assert st["peak_committed_bytes"] <= budget
    assert st["peak_running"] == 2
    assert st["done"] == 8


def test_submission_order_start():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=5.0) as s:
        tickets = [_submit(s, k) for k in range(6)]
        for t in tickets:
            s.wait(t, 10000)
        starts = [s.poll(t)[1]["queue_ms"] for t in tickets]
    assert starts == sorted(starts)


def test_job_larger_than_budget_is_rejected():
    with pdep.Server(max_running=2, hbm_budget=1 << 20, fake=True) as s:
        with pytest.raises(pdep.PdepError) as e:
            _submit(s, 1)
        assert e.value.code == pdep.PDEP_ENOMEM


def test_queue_capacity_backpressure():
    with pdep.Server(max_running=1, queue_capacity=2, fake=True, fake_ms_per_gb=2000.0) as s:
        _submit(s, 1)
        got_busy = False
        for k in range(6):
            try:
                _submit(s, 10 + k)
            except pdep.PdepError as e:
                assert e.code == pdep.PDEP_EBUSY
                got_busy = True
        assert got_busy


def test_invalid_job_rejected_at_submit():
    with pdep.Server(max_running=1, fake=True) as s:
        V = np.zeros(16 ** 3)
        V[3] = np.nan
        with pytest.raises(pdep.PdepError) as e:
            s.submit(CELL["L"], CELL["n"], CELL["ecut"], V, 4, 8)
        assert e.value.code == pdep.PDEP_EINVAL
        with pytest.raises(pdep.PdepError):
            s.submit(CELL["L"], (16, 16, 7), CELL["ecut"], np.zeros(16 * 16 * 7), 4, 8)


def test_failure_is_isolated():
    """A job that fails (forced via cg_maxit = 1 in the fake executor) does not affect
    the jobs around it."""
    with pdep.Server(max_running=2, fake=True, fake_ms_per_gb=10.0) as s:
        good1 = _submit(s, 3)
        bad = _submit(s, 4, cg_maxit=1)
        good2 = _submit(s, 5)
        for t in (good1, bad, good2):
            s.wait(t, 10000)
        assert s.poll(good1)[0] == pdep.JOB_DONE
        assert s.poll(good2)[0] == pdep.JOB_DONE
        state, res, eps = s.poll(bad)
        assert state == pdep.JOB_FAILED and res["status"] == pdep.PDEP_ENOTCONV and "forced" in res["error"]


def test_unknown_ticket():
    with pdep.Server(max_running=1, fake=True) as s:
        with pytest.raises(pdep.PdepError) as e:
            s.poll(12345)
        assert e.value.code == pdep.PDEP_ENOTFOUND


def test_concurrent_submitters():
    with pdep.Server(max_running=4, fake=True, fake_ms_per_gb=5.0) as s:
        out = []
        lock = threading.Lock()

        def client(base):
            for k in range(10):
                t = _submit(s, base + k)
                with lock:
                    out.append((base + k, t))
        th = [threading.Thread(target=client, args=(100 * i,)) for i in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert len({t for _, t in out}) == 40
        for seed, t in out:
            assert s.wait(t, 20000) == pdep.JOB_DONE
            np.testing.assert_allclose(s.poll(t)[2][0], 1.0 + (seed % 97 + 1))


def test_destroy_with_queued_jobs():
    s = pdep.Server(max_running=1, fake=True, fake_ms_per_gb=500.0)
    for k in range(5):
        _submit(s, k)
    s.close()


def test_subspace_size_rule():
    """The PDEP search space needs room for 2 (n_pdep + n_buffer) columns after a
    restart: a smaller explicit max_subspace is rejected at submission, and the HBM
    estimate grows with the buffer vectors beyond the default 4 n_pdep columns."""
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s:
        with pytest.raises(pdep.PdepError) as e:
            _submit(s, 1, n_pdep=4, n_buffer=8, max_subspace=23)
        assert e.value.code == pdep.PDEP_EINVAL
        est = []
        for kw in (dict(n_buffer=0), dict(n_buffer=8), dict(n_buffer=8, max_subspace=24)):
            t = _submit(s, 2, n_pdep=4, **kw)
            assert s.wait(t, 10000) == pdep.JOB_DONE
            est.append(s.poll(t)[1]["hbm_estimate"])
    # 16 columns by default; 24 = 2 (4 + 8) with the buffer, explicit or not
    assert est[1] > est[0] and est[1] == est[2]


def test_gvectors_needs_an_output():
    lib = pdep.load()
    assert lib.pdep_get_gvectors(None, None, None) == pdep.PDEP_EINVAL
