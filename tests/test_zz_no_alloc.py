"""rmtr_energy_noalloc (the entry point for callers that cannot allocate)
against rmtr_energy through the C-ABI, on two calls in a row, the second on
a smaller grid; the first library call of the process is the no-alloc one,
so the per-device scratch lookup happens here."""
import numpy as np
import pytest

from oracle import fem
from _util import material, rand_state, ctx_for, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("d,N,L", [(3, 32, 3), (2, 64, 3)])
def test_energy_noalloc_matches_energy(d, N, L):
    import torch
    print(f"case d={d} N={N} L={L}", flush=True)
    mat = material(N)
    ctx = ctx_for(d, N, L, mat)
    for level in (L, 1):                    # the second call is the smaller grid
        Nl = N >> (L - level)
        g, x, p = rand_state(d, Nl, seed=10 * level + d)
        xd, pd = dev(x), dev(p)
        out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        ctx.energy_noalloc(level, xd, pd, out)
        got = float(host(out)[0])
        want = float(host(ctx.energy(level, xd, pd))[0])
        assert got == want                  # same kernels, same reduction order
        assert got == pytest.approx(fem.energy(g, x, p, mat), rel=1e-12)
