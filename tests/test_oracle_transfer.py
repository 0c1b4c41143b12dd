"""Pins for the transfer operators: nested interpolation reproduces affine
fields exactly, R is the transpose of I, P I = Id, rows of I sum to one, and
the restricted box keeps every prolongated correction feasible."""
import numpy as np
import pytest

from oracle import fem, transfer

RNG = np.random.default_rng(3)


@pytest.mark.parametrize("d,Nc", [(2, 2), (2, 5), (3, 2), (3, 3)])
def test_prolongation_reproduces_affine_fields(d, Nc):
    nc = d + 1
    gc, gf = fem.Grid(d, Nc), fem.Grid(d, 2 * Nc)
    I = transfer.prolongation(d, Nc, nc)
    A = RNG.standard_normal((nc, d))
    b = RNG.standard_normal(nc)
    xc = (gc.node_coords() @ A.T + b).reshape(-1)
    xf = (gf.node_coords() @ A.T + b).reshape(-1)
    assert np.allclose(I @ xc, xf, rtol=0, atol=1e-14)


@pytest.mark.parametrize("d,Nc", [(2, 3), (3, 2)])
def test_restriction_is_transpose_and_injection_inverts(d, Nc):
    nc = d + 1
    I = transfer.prolongation(d, Nc, nc)
    R = transfer.restriction(d, Nc, nc)
    P = transfer.injection(d, Nc, nc)
    assert (abs(R - I.T)).max() == 0.0
    PI = (P @ I).toarray()
    assert np.array_equal(PI, np.eye(PI.shape[0]))
    assert np.allclose(np.asarray(I.sum(axis=1)).reshape(-1), 1.0, atol=0)
    # weights are 1, 1/2, 1/4, 1/8 only
    assert set(np.unique(I.data).tolist()) <= {1.0, 0.5, 0.25, 0.125}


@pytest.mark.parametrize("d,Nc", [(2, 3), (3, 2)])
def test_box_restriction_keeps_prolongated_corrections_feasible(d, Nc):
    nc = d + 1
    I = transfer.prolongation(d, Nc, nc)
    nf = I.shape[0]
    lo = -RNG.uniform(0.0, 1.0, nf)
    hi = RNG.uniform(0.0, 1.0, nf)
    lo[::7] = 0.0
    hi[::5] = 0.0
    loH, hiH = transfer.box_restrict(I, lo, hi)
    assert np.all(loH <= 0.0) and np.all(hiH >= 0.0)
    for _ in range(50):
        u = RNG.uniform(0.0, 1.0, I.shape[1])
        sH = loH + u * (hiH - loH)
        sH[::3] = np.where(RNG.uniform(size=sH[::3].shape) < 0.5, loH[::3], hiH[::3])
        s = I @ sH
        assert np.all(s >= lo - 1e-15) and np.all(s <= hi + 1e-15)
    # brute force: loH[j] is the max of lo over the fine dofs j feeds
    Id = I.toarray()
    for j in range(0, I.shape[1], 5):
        rows = np.nonzero(Id[:, j] > 0)[0]
        assert loH[j] == lo[rows].max() and hiH[j] == hi[rows].min()
