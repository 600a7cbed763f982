"""Error measure shared by the GPU parity tests.

For each row (one perturbation, or one grid) the error of `got` against `want` is the
larger of the 2-norm relative error and the largest element error relative to the
row's largest element; the measure is the maximum over rows.  The second term keeps an
error confined to a few components from hiding inside a small 2-norm."""
import numpy as np


def relerr(got, want):
    got = np.atleast_2d(np.asarray(got))
    want = np.atleast_2d(np.asarray(want))
    assert got.shape == want.shape, (got.shape, want.shape)
    d = got - want
    norm = np.linalg.norm(d, axis=1) / np.linalg.norm(want, axis=1)
    elem = np.max(np.abs(d), axis=1) / np.max(np.abs(want), axis=1)
    return float(max(np.max(norm), np.max(elem)))
