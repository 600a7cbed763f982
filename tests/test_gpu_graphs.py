"""HIP-graph replay of the batched inner CG (PDEP_CG_GRAPHS): every block of iterations
between two reads of the active-row count is captured once per live-row count and
replayed, with the eager compaction, refinement and synchronisation in between.  The
kernels and their order are those of eager mode, so every result must be bit-identical
to it; each replay is thereby checked against the eager result of the same solve."""
import numpy as np
import pytest

from oracle import response as R
from paper_1501_03141_amd import inputs, pdep

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,mode,npert", [("small", pdep.PDEP_MIXED_BF16X3, 12), ("small", pdep.PDEP_FP64, 6),
                                             ("tiny", pdep.PDEP_MIXED_FP32, 9)])
def test_graph_replay_bit_identical(name, mode, npert):
    w = inputs.WORKLOADS[name]
    V = inputs.vloc(w)
    m = R.make_model(w.L, w.n, w.ecut, V, naive=None if name == "tiny" else False)
    gs = R.ground_state(m, w.n_v, full=False)
    phi = inputs.trial_block(m.miller[m.nz], npert, 501)
    tol = 1e-10 if mode != pdep.PDEP_FP64 else w.cg_tol
    out = {}
    for graphs in (False, True):
        with pdep.Context(w.L, w.n, w.ecut, V, w.n_v, precision=mode, cg_tol=tol, psi=gs.C, eps=gs.eps,
                          cg_graphs=graphs) as c:
            got, st = c.chi0_apply(phi)
            got2, st2 = c.chi0_apply(phi[:npert // 2])   # a second call with fewer perturbations
        print(name, mode, "graphs" if graphs else "eager", st)
        out[graphs] = (got, got2, st, st2)
    e, g = out[False], out[True]
    assert e[2]["graph_launches"] == 0
    assert g[2]["graph_launches"] > 0 and g[2]["graph_captures"] > 0 and g[3]["graph_launches"] > 0
    assert g[2]["cg_iter_total"] == e[2]["cg_iter_total"] and g[2]["op_applications"] == e[2]["op_applications"]
    assert np.array_equal(g[0], e[0]) and np.array_equal(g[1], e[1])
