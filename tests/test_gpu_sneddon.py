"""Sneddon's pressurised crack under refinement, on the GPU.

A straight crack of half-length a = 0.1 at the centre of the unit square
(the C1 crack: a band of width 2h), uniform pressure p = 1e-3, E = 1,
nu = 0.3, l_s = 2h, u = 0 on the boundary, one load step to 1e-8.  For a
line crack in an infinite plane-strain body the opening is
  w(x) = 4 p a / E' sqrt(1 - (x - 1/2)^2 / a^2),   E' = E / (1 - nu^2)
(Sneddon and Lowengrub).  The GPU's opening is measured two ways: the jump
of u_y across the crack band at +-2 l_s, and the phase-field opening
w(x) = -int u_y dc/dy dy along each grid column.  On 128^2, 256^2 and
512^2 cells both errors against w, the largest over |x - 1/2| <= 0.8 a
relative to w(1/2), decrease monotonically (the regularised crack converges
to the sharp one as l_s -> 0; the bounded domain and the clamped boundary
keep a small offset)."""
import numpy as np
import pytest

import workloads as W
from _util import host

pytestmark = pytest.mark.gpu

E, NU, GC, P0, A = 1.0, 0.3, 1e-3, 1e-3, 0.1


def _opening(N):
    import torch
    import paper_2007_12908_amd as P
    L = int(np.log2(N // 16)) + 1
    lam = E * NU / ((1 + NU) * (1 - 2 * NU))
    mu = E / (2 * (1 + NU))
    ctx = P.Context(2, N, L, lam, mu, GC, 2.0 / N, 1e-6)
    c0, p = ctx.init_fields(L, W.fractures.c1_crack(N, P0), band=1.0 / N, p_mode=0, p_value=P0)
    x = torch.zeros(3 * (N + 1) ** 2, dtype=torch.float64, device="cuda")
    x.view(-1, 3)[:, 2] = c0
    st = ctx.solve_loadstep(x, p, c0, P.default_params(max_vcycles=1000))
    print(f"N={N} L={L} vcycles={st['vcycles']} chi/chi0={st['chi'] / st['chi0']:.2e}", flush=True)
    assert st["code"] == 0
    xs = host(x)
    uy = xs[1::3].reshape(N + 1, N + 1)
    c = xs[2::3].reshape(N + 1, N + 1)
    xc = np.arange(N + 1) / N
    sned = 4 * P0 * A * (1 - NU * NU) / E * np.sqrt(np.clip(1 - ((xc - 0.5) / A) ** 2, 0, None))
    inside = np.abs(xc - 0.5) <= 0.8 * A
    jump = uy[N // 2 + 4, :] - uy[N // 2 - 4, :]
    dcdy = np.gradient(c, 1.0 / N, axis=0)
    pf = -np.trapezoid(uy * dcdy, dx=1.0 / N, axis=0)
    e_jump = np.abs(jump - sned)[inside].max() / sned.max()
    e_pf = np.abs(pf - sned)[inside].max() / sned.max()
    print(f"  centre opening: jump {jump[N // 2]:.4e}  phase-field {pf[N // 2]:.4e}  Sneddon {sned[N // 2]:.4e}"
          f"  errors {e_jump:.4f} {e_pf:.4f}", flush=True)
    assert np.allclose(jump, jump[::-1], rtol=1e-6, atol=1e-12)
    return e_jump, e_pf


def test_opening_converges_to_sneddon():
    errs = [_opening(N) for N in (128, 256, 512)]
    for k in range(2):
        e = [er[k] for er in errs]
        assert e[0] > e[1] > e[2]
