"""One projected-Newton step with a feasibility-aware backtracking line search.

The paper returns the solution of H dx = g and leaves the step to the caller
("Solution Extraction"); the step below is the standard one on the fixed
stencil set:

* p = -H^-1 g by block-Jacobi PCG (``pcg.py``);
* alpha_0 = min(1, 0.4 min_s sqrt(d_s) / max_v |p_v|) over the contact
  stencils (1 when there are none);
* halve alpha (at most 40 times) until every stencil has d > 0, every PT/EE
  stencil keeps the sign of its plane/line side, and the Armijo condition
  E(x + alpha p) <= E(x) + 1e-4 alpha g.p holds.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import pcg as pcgmod


def solve_direction(orc, x, rtol=1e-8, max_iter=20000, hess=0, shift=0.0):
    """p = -(H + shift M)^-1 g by block-Jacobi PCG (shift: Levenberg-Marquardt
    damping with the lumped masses M; 0 for plain Newton)."""
    ev = orc.eval(x, hess)
    asm = orc.assemble(ev)
    H = orc.csr(asm)
    D = orc.diag_blocks(asm)
    if shift:
        m3 = np.repeat(shift * np.asarray(orc.mass), 3)
        H = (H + sp.diags(m3)).tocsr()
        D = D + (shift * np.asarray(orc.mass))[:, None, None] * np.eye(3)[None]
    Minv = pcgmod.block_inverse(D)
    g = asm["grad"].ravel()
    p, it, rel, status = pcgmod.pcg(lambda v: H @ v, -g, Minv, rtol, max_iter)
    return ev, asm, H, p.reshape(-1, 3), it, rel, status


def initial_step(orc, x, p):
    pmax = float(np.sqrt((p * p).sum(1)).max()) if p.size else 0.0
    if orc.cidx.shape[0] == 0 or pmax == 0.0:
        return 1.0
    dmin = float(orc.distances(x).min())
    return min(1.0, 0.4 * np.sqrt(dmin) / pmax)


def line_search(orc, x, p, E0, g, max_halvings=40, tie_rtol=0.0):
    """tie_rtol > 0: a trial whose energy differs from E0 by at most
    tie_rtol |E0| also counts as sufficient decrease (solves driven to the
    rounding floor of E, where Armijo can no longer decide); tie_rtol = 0 is
    plain Armijo."""
    alpha = initial_step(orc, x, p)
    gp = float(g.ravel() @ p.ravel())
    if gp >= 0.0 and np.abs(p).max() > 0.0:
        return 0.0, x, E0, 0  # not a descent direction (exact Hessian away from a minimum)
    s0 = np.sign(orc.sides(x))
    trials = 0
    for _ in range(max_halvings + 1):
        xt = x + alpha * p
        trials += 1
        ok = True
        if orc.cidx.shape[0]:
            d = orc.distances(xt)
            st = np.sign(orc.sides(xt))
            ok = bool((d > 0).all()) and bool((st == s0).all())
        if ok:
            E1 = orc.energy(xt)
            if E1 <= E0 + 1e-4 * alpha * gp or (tie_rtol > 0 and abs(E1 - E0) <= tie_rtol * abs(E0)):
                return alpha, xt, E1, trials
        alpha *= 0.5
    return 0.0, x, E0, trials


def newton_step(orc, x, rtol=1e-8, max_iter=20000, tie_rtol=0.0, hess=0, shift=0.0):
    """hess=1 (EXACT) solves with the unprojected Hessian; the caller checks
    ``cg_status`` ('breakdown' when that matrix is not positive definite).
    shift: Levenberg-Marquardt damping (H + shift M) of the solve only."""
    x = np.asarray(x, np.float64).reshape(orc.n, 3)
    ev, asm, H, p, it, rel, status = solve_direction(orc, x, rtol, max_iter, hess, shift)
    if status == "breakdown":
        return x, dict(E0=ev["E"], E1=ev["E"], alpha=0.0, cg_iters=it, cg_rel=rel, cg_status=status,
                       ls_trials=0, p=p, grad=asm["grad"])
    alpha, x1, E1, trials = line_search(orc, x, p, ev["E"], asm["grad"], tie_rtol=tie_rtol)
    return x1, dict(E0=ev["E"], E1=E1, alpha=alpha, cg_iters=it, cg_rel=rel,
                    cg_status=status, ls_trials=trials, p=p, grad=asm["grad"])
