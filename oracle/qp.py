"""Oracle: solvers for the box-constrained trust-region subproblem.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The TR subproblem (eq. (model_qp)) with the infinity-norm ball folded into
the bounds is      min_s  g^T s + 1/2 s^T H s,   lo <= s <= hi.

pgs    symmetric projected Gauss-Seidel (Sec. 3.2.1: PGS on all levels but
       the coarsest, symmetric = forward then backward substitution).  Order:
       the 2^d node colours (i%2 + 2 (j%2) + 4 (k%2)) ascending, components
       ascending inside a colour; the backward sweep reverses both.  Nodes of
       one colour share no element, so updating all of them at once equals
       any sequential order.  Per dof: r = g_j + (H s)_j,
       s_j <- clamp(s_j - r / H_jj, lo_j, hi_j).  When H_jj <= 1e-300 the dof
       moves to whichever bound has the lower 1D model value (ties: lo).
mprgp  MPRGP (Dostal), the coarsest-level solver of Sec. 3.2.1, for a box;
       on non-positive curvature it stops and falls back to PGS sweeps.
"""
import numpy as np
import scipy.sparse as sp

TINY_CURV = 1e-300


def colour_blocks(nodes_colour, nc, n_colours):
    """Dof index arrays per (colour, component), in sweep order."""
    blocks = []
    for col in range(n_colours):
        nodes = np.nonzero(nodes_colour == col)[0]
        for comp in range(nc):
            blocks.append(nodes * nc + comp)
    return blocks


def _update_block(HJ, Hd, g, s, lo, hi, J):
    if J.size == 0:
        return
    r = g[J] + HJ @ s
    dj = Hd[J]
    pos = dj > TINY_CURV
    new = np.empty(J.size)
    new[pos] = np.clip(s[J][pos] - r[pos] / dj[pos], lo[J][pos], hi[J][pos])
    neg = ~pos
    if np.any(neg):
        sj = s[J][neg]
        tlo, thi = lo[J][neg] - sj, hi[J][neg] - sj
        mlo = r[neg] * tlo + 0.5 * dj[neg] * tlo * tlo
        mhi = r[neg] * thi + 0.5 * dj[neg] * thi * thi
        new[neg] = np.where(mhi < mlo, hi[J][neg], lo[J][neg])
    s[J] = new


def pgs(H, g, lo, hi, s, blocks, sweeps, free=None):
    """`sweeps` symmetric PGS sweeps on s (modified in place and returned)."""
    H = H.tocsr()
    Hd = H.diagonal()
    if free is None:
        free = np.ones(g.shape[0], dtype=bool)
    blocks = [J[free[J]] for J in blocks]
    rows = [H[J, :] for J in blocks]
    for _ in range(sweeps):
        for J, HJ in zip(blocks, rows):
            _update_block(HJ, Hd, g, s, lo, hi, J)
        for J, HJ in zip(reversed(blocks), reversed(rows)):
            _update_block(HJ, Hd, g, s, lo, hi, J)
    return s


def model_value(H, g, s):
    return float(g @ s + 0.5 * s @ (H @ s))


def mprgp(H, g, lo, hi, s0=None, rtol=1e-10, max_it=500, gamma=1.0,
          fallback=None):
    """Box-constrained QP  min 1/2 s^T A s - b^T s,  A = H, b = -g,  by MPRGP.

    Step length alpha_bar = 1.9 / ||A||, with ||A|| bounded by the largest
    Gershgorin row sum.  Returns (s, iterations, status) where status is
    'converged', 'max_it' or 'negative_curvature' (then `fallback(s)` is
    applied when given).
    """
    A = H.tocsr()
    b = -g
    n = b.shape[0]
    s = np.zeros(n) if s0 is None else np.clip(s0.copy(), lo, hi)
    absA = abs(A)
    normA = float(np.max(np.asarray(absA.sum(axis=1)).reshape(-1))) if n else 0.0
    if normA <= 0.0:
        return s, 0, "converged"
    abar = 1.9 / normA

    def free_grad(x, gr):
        f = (x > lo) & (x < hi)
        return np.where(f, gr, 0.0)

    def chopped(x, gr):
        atlo = (x <= lo) & (lo < hi)
        athi = (x >= hi) & (lo < hi)
        return np.where(atlo, np.minimum(gr, 0.0), 0.0) + np.where(athi, np.maximum(gr, 0.0), 0.0)

    def reduced_free(x, phi):
        return np.where(phi > 0.0, np.minimum((x - lo) / abar, phi),
                        np.maximum((x - hi) / abar, phi))

    gr = A @ s - b
    phi = free_grad(s, gr)
    beta = chopped(s, gr)
    bnorm = float(np.linalg.norm(b))
    tol = rtol * max(bnorm, 1e-300)
    p = phi.copy()
    it = 0
    status = "max_it"
    while it < max_it:
        if np.linalg.norm(phi + beta) <= tol:
            status = "converged"
            break
        it += 1
        phit = reduced_free(s, phi)
        if beta @ beta <= gamma * gamma * (phit @ phi):
            Ap = A @ p
            pAp = float(p @ Ap)
            if pAp <= 0.0:
                status = "negative_curvature"
                break
            acg = float(gr @ p) / pAp
            # largest feasible step along -p
            with np.errstate(divide="ignore", invalid="ignore"):
                af_lo = np.where(p > 0.0, (s - lo) / p, np.inf)
                af_hi = np.where(p < 0.0, (s - hi) / p, np.inf)
            af = float(min(np.min(af_lo), np.min(af_hi))) if n else np.inf
            if acg <= af:
                s = s - acg * p
                gr = gr - acg * Ap
                phi = free_grad(s, gr)
                bet = float(phi @ Ap) / pAp
                p = phi - bet * p
            else:
                s = s - af * p
                gr = gr - af * Ap
                phi = free_grad(s, gr)
                s = np.clip(s - abar * phi, lo, hi)
                gr = A @ s - b
                phi = free_grad(s, gr)
                p = phi.copy()
        else:
            d = beta
            Ad = A @ d
            dAd = float(d @ Ad)
            if dAd <= 0.0:
                status = "negative_curvature"
                break
            a = float(gr @ d) / dAd
            # stay inside the box along -d (a chopped component can only
            # move a variable off its active bound, towards the other one)
            with np.errstate(divide="ignore", invalid="ignore"):
                af_lo = np.where(d > 0.0, (s - lo) / d, np.inf)
                af_hi = np.where(d < 0.0, (s - hi) / d, np.inf)
            a = min(a, float(min(np.min(af_lo), np.min(af_hi))))
            s = np.clip(s - a * d, lo, hi)
            gr = gr - a * Ad
            phi = free_grad(s, gr)
            p = phi.copy()
        beta = chopped(s, gr)
    if status == "negative_curvature" and fallback is not None:
        s = fallback(s)
    return s, it, status
