"""The entry point that allocates no device memory (chi0_apply_noalloc), through the C
ABI, against chi0_apply on the same context and inputs: two calls in a row, the second
with fewer perturbations, in FP64 (bar 1e-10 per perturbation, the FP64 parity bar) and
in the BF16x3 mode (1e-8), on the tiny workload (one pass) and the small one (several
passes through the fixed work space); and the rejection of a workload whose single
perturbation does not fit that space."""
import numpy as np
import pytest

from oracle import response as R
from paper_1501_03141_amd import inputs, pdep
from parity import relerr

pytestmark = pytest.mark.gpu


def _oracle(name):
    w = inputs.WORKLOADS[name]
    V = inputs.vloc(w)
    m = R.make_model(w.L, w.n, w.ecut, V, naive=None if name == "tiny" else False)
    gs = R.ground_state(m, w.n_v, full=False)
    return w, V, m, gs


@pytest.fixture(scope="module")
def tiny():
    return _oracle("tiny")


@pytest.mark.parametrize("mode,bar", [(pdep.PDEP_FP64, 1e-10), (pdep.PDEP_MIXED_BF16X3, 1e-8)])
def test_noalloc_matches_chi0_apply_tiny(tiny, mode, bar):
    w, V, m, gs = tiny
    phi = inputs.trial_block(m.miller[m.nz], 9, 301)
    tol = 1e-11 if mode == pdep.PDEP_FP64 else 1e-10
    want = R.chi0bar_apply(m, gs, phi)
    with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=mode, cg_tol=tol, psi=gs.C, eps=gs.eps) as c:
        for n in (9, 3):                  # the second call is smaller
            got, st = c.chi0_apply_noalloc(phi[:n])
            ref, st_ref = c.chi0_apply(phi[:n])
            err, err_o = relerr(got, ref), relerr(got, want[:n])
            print("tiny", mode, n, "relerr vs chi0_apply", err, "vs oracle", err_o, st)
            assert st["n_rhs"] == n * w.n_v and st["n_notconv"] == 0
            assert err <= bar and err_o <= bar


def test_noalloc_device_pointers_several_passes():
    """Small workload (N_v = 32, 5041 plane waves): 14 perturbations need more than one
    pass through the fixed work space; device pointers; then a call with 2."""
    import torch
    w, V, m, gs = _oracle("small")
    phi = inputs.trial_block(m.miller[m.nz], 14, 302)
    with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, cg_tol=1e-11, psi=gs.C, eps=gs.eps, device_ptrs=True) as c:
        for n in (14, 2):
            x = torch.from_numpy(phi[:n]).cuda()
            got, st = c.chi0_apply_noalloc(x)
            ref, _ = c.chi0_apply(x)
            torch.cuda.synchronize()
            err = relerr(got.cpu().numpy(), ref.cpu().numpy())
            print("small", n, "relerr", err, st)
            assert st["n_rhs"] == n * w.n_v and st["n_notconv"] == 0
            assert err <= 1e-10


def test_noalloc_rejects_a_perturbation_beyond_the_scratch():
    """Medium workload (N_v = 128, 15895 plane waves): one perturbation's work space
    exceeds the fixed 256 MiB; the call fails with PDEP_ENOMEM and a message, and the
    context stays usable."""
    w = inputs.WORKLOADS["medium"]
    V = inputs.vloc(w)
    with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=pdep.PDEP_MIXED_BF16X3, cg_tol=1e-8) as c:
        mil = c.miller()
        phi = inputs.trial_block(mil[np.any(mil != 0, axis=1)], 1, 303)
        with pytest.raises(pdep.PdepError) as e:
            c.chi0_apply_noalloc(phi)
        assert e.value.code == pdep.PDEP_ENOMEM and "no-allocation scratch" in str(e.value)
        out, st = c.chi0_apply(phi)
        assert st["n_notconv"] == 0 and np.all(np.isfinite(out))
