"""Hand-worked pins for oracle parts that the finite-difference and
closed-form tests elsewhere do not reach: the stopping measure chi, the
per-fracture pressure field, the trust-region ratio and radius control of
Alg. 3 (with the round-off and step-based readings) and Adam's bias
correction beyond the first step.  Every expected value below was worked out
by hand from the definitions cited in each test, not by calling the oracle
or retyping its formulas."""
import math

import numpy as np
import pytest

from oracle import cnn, fem, fields, rmtr


# ------------------------------------------------------------------ chi
# Stopping measure (Sec. 3, the projected-gradient criterion of the
# load-step loop): chi = || P_F(x - g) - x ||_2 over the free dofs, with F
# the box c_lower <= c <= 1 on the phase field and no bound on u.
#
# 2D, 2 x 2 cells: nodes n = i + 3 j; only node 4 has free displacements
# under the default Dirichlet set.  Per node: (c, c_lower, dE/dc) and the
# hand-worked residual P(c - g) - c.
_CHI_NODES = [
    # c,    c_lower, g_c,   residual
    (1.0,  0.0,  -0.5,   0.0),     # at the upper bound, pushed out: 0
    (0.2,  0.2,   0.3,   0.0),     # at its lower bound c_lower = 0.2, pushed out: 0
    (0.5,  0.0,   0.25, -0.25),    # interior: -g
    (0.9,  0.1,  -0.3,   0.1),     # clipped at 1
    (0.3,  0.3,  -0.2,   0.2),     # at the lower bound, pushed inwards: -g
    (0.6,  0.5,   0.4,  -0.1),     # clipped at c_lower = 0.5 (not at 0)
    (1.0,  0.0,   0.5,  -0.5),     # at the upper bound, pushed inwards
    (0.0,  0.0,   0.0,   0.0),
    (0.75, 0.0,   0.125, -0.125),
]
# sum of squared c residuals: 0.0625 + 0.01 + 0.04 + 0.01 + 0.25 + 0.015625
_CHI_C_SQ = 0.388125


def _chi_case():
    g = fem.Grid(2, 2)
    x = np.zeros(g.n_dofs)
    gv = np.zeros(g.n_dofs)
    cl = np.zeros(g.n_nodes)
    for n, (c, lo, gc, _) in enumerate(_CHI_NODES):
        x[3 * n + 2] = c
        cl[n] = lo
        gv[3 * n + 2] = gc
        # displacement values and gradients everywhere; the boundary ones are
        # Dirichlet dofs and must not count
        x[3 * n:3 * n + 2] = (0.01 * n, -0.02 * n)
        gv[3 * n:3 * n + 2] = (7.0, 7.0)
    gv[3 * 4:3 * 4 + 2] = (0.3, -0.4)   # node 4, free: residual (-0.3, 0.4)
    return g, x, gv, cl


def test_chi_hand_worked_bounds_and_dirichlet():
    g, x, gv, cl = _chi_case()
    # free u of node 4 contributes 0.09 + 0.16
    assert fem.chi(g, x, gv, cl) == pytest.approx(math.sqrt(_CHI_C_SQ + 0.25), rel=1e-14)


def test_chi_hand_worked_custom_dirichlet_mask():
    g, x, gv, cl = _chi_case()
    dirm = g.default_dirichlet()
    dirm[3 * 6 + 2] = True          # fix the phase field of node 6: drops 0.25
    dirm[0:2] = False               # free both displacements of node 0: adds 49 + 49
    expect = math.sqrt(_CHI_C_SQ - 0.25 + 0.25 + 98.0)
    assert fem.chi(g, x, gv, cl, dirm) == pytest.approx(expect, rel=1e-14)


# ------------------------------------------------- per-fracture pressure
# Sec. 5 (nodal inclusion) and the per-fracture pressure reading: p at a
# node is the largest p_f over the discs within distance p_band of it.
# Disc D1: centre (0.5, 0.5, 0.25), normal e_z, radius 1/8, p = 1e-3.
# Disc D2: centre (0.5, 0.5, 0.75), normal (0, 0.6, 0.8), radius 1/4,
# p = 2e-3.  p_band = 0.3, grid 8^3 cells (nodes at multiples of 1/8).
_TABLE = np.array([
    [0.5, 0.5, 0.25, 0.0, 0.0, 1.0, 0.125, 1e-3],
    [0.5, 0.5, 0.75, 0.0, 0.6, 0.8, 0.25, 2e-3],
])
_P_NODES = [
    # point,             p     (distances to D1, D2 worked by hand)
    ((0.5, 0.5, 0.5),    2e-3),  # D1 0.25, D2 0.2 (in-plane 0.15 < r): both, max
    ((0.5, 0.5, 0.0),    1e-3),  # D1 0.25; D2: normal 0.6, in-plane 0.45 -> sqrt(0.40)
    ((0.875, 0.5, 0.25), 1e-3),  # D1 rim distance 0.375 - 0.125 = 0.25; D2 ~0.46
    ((1.0, 0.5, 0.25),   0.0),   # D1 0.375 > 0.3; D2 ~0.52
    ((0.5, 0.625, 0.875), 2e-3), # D2: normal 0.175, in-plane 0.025 < r
    ((0.5, 0.5, 1.0),    2e-3),  # D2 0.2; D1 0.75
]


def _node_index(g, pt):
    i = [int(round(v * g.N)) for v in pt]
    return i[0] + g.nside * (i[1] + g.nside * i[2])


def test_per_fracture_pressure_two_discs():
    g = fem.Grid(3, 8)
    c0, p = fields.initial_fields(g, _TABLE, p_uniform=None, p_band=0.3)
    for pt, want in _P_NODES:
        assert p[_node_index(g, pt)] == want, pt
    # every other node: p is one of the two pressures or zero
    assert set(np.unique(p)) <= {0.0, 1e-3, 2e-3}


def test_inclusion_band_is_inclusive_and_uniform_pressure_overrides():
    g = fem.Grid(3, 8)
    c0, p = fields.initial_fields(g, _TABLE, p_uniform=5e-4)
    assert c0[_node_index(g, (0.5, 0.5, 0.25))] == 1.0      # on D1
    assert c0[_node_index(g, (0.5, 0.5, 0.375))] == 1.0     # exactly h from D1 (inclusive)
    assert c0[_node_index(g, (0.5, 0.5, 0.5))] == 0.0       # 0.25 from D1, 0.2 from D2
    assert np.all(p == 5e-4)


# ------------------------------------------------ Alg. 3 ratio / control
def _solver(**kw):
    g = fem.Grid(2, 4)                      # 16 elements: sqrt = 4
    mat = fem.material_from_E_nu(1.0, 0.3, 1e-3, 0.5)
    s = rmtr.RMTR(2, 4, 1, mat, np.zeros(g.n_nodes), rmtr.Params(**kw))
    s.f_ref = -4.0                           # round-off level 1e-14 * 4 / 4 = 1e-14
    return s, s.levels[1]


@pytest.mark.parametrize("ared,pred,rho", [
    (0.5, 1.0, 0.5),
    (-0.2, 1.0, -0.2),
    (1.0, 0.0, 1.0),                  # |pred| <= tol, ared >= -tol: counts as rho = 1
    (-0.5e-14, 5e-15, 1.0),           # both below the round-off level
    (-2e-14, 5e-15, -math.inf),       # measurably uphill below the round-off level
    (0.3, -1.0, -math.inf),           # the model predicts an increase
    (math.nan, 1.0, -math.inf),
    (1.0, math.inf, -math.inf),
])
def test_ratio_table(ared, pred, rho):
    s, lev = _solver()
    assert s.ratio(ared, pred, lev) == rho


@pytest.mark.parametrize("rho,delta,snorm,accept,new", [
    (0.5, 1.0, 0.3, True, 1.0),               # [eta1, eta2]: keep
    (0.1, 1.0, 0.3, False, 1.0),              # rho = eta1 exactly: reject, keep (reading 11)
    (0.10000000000000002, 1.0, 0.3, True, 1.0),
    (0.75, 1.0, 0.3, True, 1.0),              # rho = eta2: keep
    (0.76, 1.0, 0.3, True, 2.0),              # gamma2 delta
    (0.9, 6.0, 0.3, True, 10.0),              # capped at delta_max
    (0.05, 1.0, 0.3, False, 0.5),             # gamma1 delta
    (-math.inf, 0.25, 0.3, False, 0.125),
])
def test_control_table(rho, delta, snorm, accept, new):
    s, _ = _solver()
    step = np.array([0.0, -snorm, 0.1])
    assert s.control(rho, delta, step) == (accept, new)


@pytest.mark.parametrize("rho,delta,snorm,accept,new", [
    (0.05, 1.0, 0.2, False, 0.1),             # gamma1 min(delta, |s|_inf)
    (0.05, 1.0, 3.0, False, 0.5),
    (0.1, 1.0, 0.2, False, 1.0),              # rho = eta1: no shrink
    (0.8, 1.0, 0.2, True, 2.0),               # growth ignores the step length
])
def test_control_table_step_based(rho, delta, snorm, accept, new):
    s, _ = _solver(shrink_to_step=True)
    step = np.array([snorm, -0.01])
    assert s.control(rho, delta, step) == (accept, new)


# ---------------------------------------------------------- Adam, t > 1
# Kingma and Ba: with a constant gradient a, m_t = (1 - b1^t) a and
# v_t = (1 - b2^t) a^2, so the bias-corrected moments are a and a^2 at every
# t and each step moves lr * a / (|a| + eps).
@pytest.mark.parametrize("t_end", [3, 10])
def test_adam_constant_gradient_closed_form(t_end):
    a = np.array([0.5, -2.0, 1e-3])
    p = np.array([1.0, 1.0, 1.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr = 0.01
    for t in range(1, t_end + 1):
        p, m, v = cnn.adam_step(p, a, m, v, t, lr)
    want = 1.0 - t_end * lr * a / (np.abs(a) + 1e-8)
    assert np.allclose(p, want, rtol=0, atol=1e-13)


def test_adam_late_gradient_bias_correction():
    """Gradients 0, 0, a: m_3 = 0.1 a and v_3 = 0.001 a^2; corrected by
    1 - 0.9^3 = 0.271 and 1 - 0.999^3 = 0.002997001 the third step is
    lr (0.1 / 0.271) / sqrt(0.001 / 0.002997001) sign(a) (eps negligible)."""
    a = np.array([3.0, -0.25])
    p = np.zeros(2)
    m = np.zeros(2)
    v = np.zeros(2)
    lr = 0.1
    for t, gr in enumerate([np.zeros(2), np.zeros(2), a], start=1):
        p, m, v = cnn.adam_step(p, gr, m, v, t, lr)
    step = lr * (0.1 / 0.271) / math.sqrt(0.001 / 0.002997001)
    assert np.allclose(p, -step * np.sign(a), rtol=1e-7, atol=0)
