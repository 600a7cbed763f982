"""Resident systems and batched chi0 requests on the CPU with the fake executor (no GPU
work; a batch sleeps fake_ms_per_gb ms plus 1 ms per perturbation and returns -phi / 2):
requests queued on one system while a batch runs are merged into the next batch, every
request gets its own rows back, batches respect max_batch_pert, removal fails what is
still queued, and bad arguments and budgets are rejected."""
import threading

import numpy as np
import pytest

from paper_1501_03141_amd import pdep

CELL = dict(L=(10.0, 10.0, 10.0), n=(16, 16, 16), ecut=5.0)
NPW = 515   # plane waves of the 16^3, 5 Ha sphere


def _system(srv, max_batch_pert=0):
    return srv.add_system(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3), 4, max_batch_pert=max_batch_pert)


def _phi(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, NPW - 1)) + 1j * rng.standard_normal((n, NPW - 1))


def test_requests_queued_during_a_batch_share_the_next_one():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=60.0) as s:
        sid = _system(s)
        sizes = [2, 1, 3, 2, 1, 2]
        phis = [_phi(n, k) for k, n in enumerate(sizes)]
        tickets = [s.submit_chi0(sid, p) for p in phis]
        for t in tickets:
            assert s.wait(t, 10000) == pdep.JOB_DONE
        recs = []
        for p, t in zip(phis, tickets):
            state, res, out = s.poll_chi0(t)
            assert state == pdep.JOB_DONE and res["status"] == 0
            np.testing.assert_array_equal(out, -0.5 * p)          # its own rows, in order
            assert res["n_pert"] == p.shape[0]
            assert res["batch_pert"] >= res["n_pert"] and res["batch_requests"] >= 1
            assert res["latency_ms"] >= res["run_ms"] >= 0
            recs.append(res)
        # the requests submitted while the first batch ran were merged into one batch
        assert max(r["batch_requests"] for r in recs) > 1


def test_batches_respect_max_batch_pert():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=40.0) as s:
        sid = _system(s, max_batch_pert=3)
        sizes = [1, 2, 2, 1, 5, 1, 1]
        phis = [_phi(n, 10 + k) for k, n in enumerate(sizes)]
        tickets = [s.submit_chi0(sid, p) for p in phis]
        for t in tickets:
            assert s.wait(t, 10000) == pdep.JOB_DONE
        for p, t in zip(phis, tickets):
            _, res, out = s.poll_chi0(t)
            np.testing.assert_array_equal(out, -0.5 * p)
            if res["n_pert"] > 3:
                # a request larger than the limit runs alone
                assert res["batch_requests"] == 1 and res["batch_pert"] == res["n_pert"]
            else:
                assert res["batch_pert"] <= 3


def test_remove_system_fails_queued_requests_only():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=150.0) as s:
        sid = _system(s, max_batch_pert=1)
        tickets = [s.submit_chi0(sid, _phi(1, k)) for k in range(4)]
        # let the first batch start, then remove the system while the rest wait
        for _ in range(200):
            if s.poll_chi0(tickets[0])[0] == pdep.JOB_RUNNING:
                break
            threading.Event().wait(0.005)
        s.remove_system(sid)
        states = [s.poll_chi0(t)[0] for t in tickets]
        assert states[0] == pdep.JOB_DONE
        assert all(st == pdep.JOB_FAILED for st in states[1:])
        _, res, _ = s.poll_chi0(tickets[1])
        assert res["status"] == pdep.PDEP_EINVAL and "removed" in res["error"]
        assert 0 <= res["queue_ms"] <= res["latency_ms"] < 60000 and res["run_ms"] == 0
        with pytest.raises(pdep.PdepError) as e:
            s.submit_chi0(sid, _phi(1, 9))
        assert e.value.code == pdep.PDEP_ENOTFOUND


def test_bad_arguments_and_budget():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s:
        with pytest.raises(pdep.PdepError) as e:
            s.submit_chi0(12345, _phi(1, 0))
        assert e.value.code == pdep.PDEP_ENOTFOUND
        sid = _system(s)
        with pytest.raises(pdep.PdepError) as e:
            s.submit_chi0(sid, np.zeros((0, NPW - 1), dtype=np.complex128))
        assert e.value.code == pdep.PDEP_EINVAL
        bad = _phi(1, 1)
        bad[0, 3] = np.nan
        with pytest.raises(pdep.PdepError) as e:
            s.submit_chi0(sid, bad)
        assert e.value.code == pdep.PDEP_EINVAL
    with pdep.Server(max_running=1, hbm_budget=1 << 20, fake=True, fake_ms_per_gb=0.0) as s:
        with pytest.raises(pdep.PdepError) as e:
            _system(s)
        assert e.value.code == pdep.PDEP_ENOMEM


def test_concurrent_submitters_get_their_own_rows():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=5.0) as s:
        sid = _system(s, max_batch_pert=8)
        out = {}
        lock = threading.Lock()

        def client(k):
            for j in range(5):
                p = _phi(1 + (k + j) % 3, 100 * k + j)
                t = s.submit_chi0(sid, p)
                s.wait(t, 10000)
                _, _, o = s.poll_chi0(t)
                with lock:
                    out[(k, j)] = (p, o)

        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert len(out) == 20
        for p, o in out.values():
            np.testing.assert_array_equal(o, -0.5 * p)


def test_result_is_delivered_once():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s:
        sid = _system(s)
        p = _phi(2, 3)
        t = s.submit_chi0(sid, p)
        assert s.wait(t, 10000) == pdep.JOB_DONE
        state, res, out = s.poll_chi0(t)
        np.testing.assert_array_equal(out, -0.5 * p)
        with pytest.raises(pdep.PdepError) as e:
            s.poll_chi0(t)
        assert e.value.code == pdep.PDEP_EINVAL


def test_pdep_request_runs_alone_between_chi0_batches():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=40.0) as s:
        sid = _system(s)
        t1 = s.submit_chi0(sid, _phi(2, 1))
        te = s.submit_eigs(sid, 6, seed=11)
        t2 = s.submit_chi0(sid, _phi(1, 2))
        t3 = s.submit_chi0(sid, _phi(3, 3))
        for t in (t1, te, t2, t3):
            assert s.wait(t, 10000) == pdep.JOB_DONE
        state, res, eps = s.poll_eigs(te)
        assert state == pdep.JOB_DONE and res["status"] == 0 and res["n_pdep"] == 6
        np.testing.assert_allclose(eps, 1.0 + (11 % 97 + 1) / np.arange(1, 7))
        r1 = s.poll_chi0(t1)[1]
        r2 = s.poll_chi0(t2)[1]
        # the chi0 blocks on either side of the Davidson never share its batch
        assert r1["batch_pert"] == 2 and r2["batch_requests"] == 2 and r2["batch_pert"] == 4
        with pytest.raises(pdep.PdepError) as e:
            s.poll_chi0(te)
        assert e.value.code == pdep.PDEP_ENOTFOUND
        with pytest.raises(pdep.PdepError) as e:
            s.submit_eigs(sid, 4, eig_tol=-1.0)
        assert e.value.code == pdep.PDEP_EINVAL


def test_jobs_are_admitted_within_the_budget_left_by_resident_systems():
    with pdep.Server(max_running=2, fake=True, fake_ms_per_gb=0.0) as s0:
        sid = _system(s0)
        est_sys = s0.stats()["committed_bytes"]
        t = s0.submit(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3), 4, 8, seed=1)
        s0.wait(t, 10000)
        est_job = s0.poll(t)[1]["hbm_estimate"]
    # room for the system and one job beside it, not two
    budget = est_sys + est_job + est_job // 2
    with pdep.Server(max_running=4, hbm_budget=budget, fake=True, fake_ms_per_gb=30.0) as s:
        sid = _system(s)
        tickets = [s.submit(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3), 4, 8, seed=k) for k in range(4)]
        for t in tickets:
            assert s.wait(t, 20000) == pdep.JOB_DONE
        st = s.stats()
        assert st["peak_running"] == 1 and st["peak_committed_bytes"] <= budget
        s.remove_system(sid)
        assert s.stats()["committed_bytes"] == 0


def test_a_job_waiting_for_memory_starts_when_a_system_is_removed():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s0:
        _system(s0)
        est_sys = s0.stats()["committed_bytes"]
        t = s0.submit(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3), 4, 8, seed=1)
        s0.wait(t, 10000)
        est_job = s0.poll(t)[1]["hbm_estimate"]
    # the job does not fit beside the resident system, and nothing else happens on the
    # server after the removal: the removal itself has to start it
    with pdep.Server(max_running=1, hbm_budget=est_sys + est_job // 2, fake=True, fake_ms_per_gb=0.0) as s:
        sid = _system(s)
        t = s.submit(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3), 4, 8, seed=2)
        assert s.wait(t, 200) == pdep.JOB_QUEUED
        s.remove_system(sid)
        assert s.wait(t, 10000) == pdep.JOB_DONE


def test_system_info_and_shape_checks():
    with pdep.Server(max_running=1, fake=True, fake_ms_per_gb=0.0) as s:
        sid = _system(s)
        info = s.system_info(sid)
        assert info["n_pw"] == NPW and info["n_v"] == 4 and info["n_grid"] == 16 ** 3
        assert abs(info["volume"] - 1000.0) < 1e-12
        # rows of the wrong length or a potential of the wrong size never reach the library
        with pytest.raises(ValueError):
            s.submit_chi0(sid, _phi(1, 0)[:, :-1])
        with pytest.raises(ValueError):
            s.add_system(CELL["L"], CELL["n"], CELL["ecut"], np.zeros(16 ** 3 - 1), 4)
        with pytest.raises(pdep.PdepError) as e:
            s.system_info(sid + 100)
        assert e.value.code == pdep.PDEP_ENOTFOUND
