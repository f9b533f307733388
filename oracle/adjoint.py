"""Adjoint of the static-equilibrium solve with respect to per-tet Young's moduli.

Static problem (no inertia): E(x; theta) = sum_t theta_t psi_t(x) + sum_s kappa b(d_s)
- sum_v m_v g . x_v, where psi_t is the Neo-Hookean energy of tet t with unit
Young's modulus (Psi is linear in E at fixed Poisson ratio, since alpha depends
only on mu / lambda).  x*(theta) minimises E; the loss is L = |x* - x_tgt|^2.

Implicit differentiation of grad_x E(x*(theta); theta) = 0:
    H(x*) dx*/dtheta_t = - d(grad_x E)/dtheta_t = - grad_x psi_t(x*)
so with H lambda = dL/dx* = 2 (x* - x_tgt) (H the exact, unprojected Hessian),
    dL/dtheta_t = - lambda . grad_x psi_t(x*)   (free vertices only).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla
import torch

from . import assemble as oasm
from . import local
from . import newton as onewton


def set_theta(orc, theta):
    """Per-tet Lame parameters theta_t * (mu_1, lambda_1) (unit-modulus values)."""
    p = orc.p
    orc.mu = torch.as_tensor(np.asarray(theta) * p["mu1"], dtype=torch.float64)
    orc.lam = torch.as_tensor(np.asarray(theta) * p["lam1"], dtype=torch.float64)


def converged(orc, x, p_dir=None, gtol=1e-9):
    """Stop rule: max_v |grad_v E| <= gtol * max_v m_v |g| (and, when a step is
    given, max_v |p_v| / h < 1e-2)."""
    g = orc.assemble(orc.eval(x))["grad"]
    scale = np.max(orc.mass) * np.linalg.norm(orc.gravity)
    gmax = float(np.sqrt((g * g).sum(1)).max())
    ok = gmax <= gtol * scale
    if p_dir is not None:
        ok = ok and np.sqrt((p_dir ** 2).sum(1)).max() / float(orc.p["h"]) < 1e-2
    return ok, gmax


TIE_RTOL = 1e-14  # energy changes this small (relative) are below what E resolves
def shift_scale(orc, x):
    """1 % of the median ratio of the Hessian's diagonal (trace / 3 per vertex)
    to the vertex mass: the first Levenberg-Marquardt shift."""
    asm = orc.assemble(orc.eval(x, oasm.EXACT))
    tr = np.abs(np.trace(orc.diag_blocks(asm), axis1=1, axis2=2)) / 3.0
    return 1e-2 * float(np.median(tr / np.asarray(orc.mass)))


def solve_equilibrium(orc, x0, max_newton=60, gtol=1e-9):
    """Damped exact Newton to the stop rule: each step solves
    (H_exact + mu M) p = -g (Levenberg-Marquardt with the lumped masses) and
    line-searches E; a step whose PCG breaks down, whose direction is not one
    of descent or whose line search fails is retried with a larger mu (x
    unchanged), and mu shrinks by 4 after full steps (to 0 once below 1e-6 of
    its first value), so the iteration becomes plain exact Newton near the
    minimum, where the exact Hessian (the adjoint solve's matrix) is positive
    definite.  Projected Newton alone converges only linearly wherever the
    projection clamps modes of indefinite element and contact Hessians.  Near
    the minimum the energy change of a step falls below the rounding of E, so
    trials that change E by at most TIE_RTOL |E| count as a decrease
    (feasibility is still enforced)."""
    x = np.array(x0, dtype=np.float64)
    gmax = np.inf
    mu, mu0 = 0.0, None
    for k in range(max_newton):
        x1, info = onewton.newton_step(orc, x, rtol=1e-12, max_iter=50000, tie_rtol=TIE_RTOL, hess=1, shift=mu)
        if info["cg_status"] != "ok" or info["alpha"] == 0.0:
            if mu0 is None:
                mu0 = shift_scale(orc, x)
            mu = mu0 if mu == 0.0 else 4.0 * mu
            continue
        ok, gmax = converged(orc, x1, info["p"], gtol)
        x = x1
        if ok:
            return x, k + 1
        if info["alpha"] == 1.0 and mu > 0.0:
            mu = 0.0 if mu / 4.0 < 1e-6 * mu0 else mu / 4.0
    raise RuntimeError(f"equilibrium not reached (|g|_inf = {gmax:.3e})")


def unit_gradients(orc, x):
    """grad_x psi_t(x*) for every tet with unit modulus: (n_t, 4, 3), fixed vertices zeroed."""
    p = orc.p
    nt = orc.tet_idx.shape[0]
    mu1 = torch.full((nt,), float(p["mu1"]))
    lam1 = torch.full((nt,), float(p["lam1"]))
    _, g, _ = orc.tets(x, oasm.EXACT, mu=mu1, lam=lam1)
    return g.numpy()


def theta_gradient(orc, x_star, x_tgt):
    """dL/dtheta for L = |x* - x_tgt|^2 (exact Hessian, sparse direct solve)."""
    ev = orc.eval(x_star, oasm.EXACT)
    asm = orc.assemble(ev)
    H = orc.csr(asm).tocsc()
    rhs = 2.0 * (np.asarray(x_star) - np.asarray(x_tgt)).ravel()
    lam = spla.spsolve(H, rhs).reshape(-1, 3)
    gu = unit_gradients(orc, x_star)
    idx = orc.tet_idx
    n = orc.n
    lam_t = np.where((idx >= 0)[..., None] & (idx < n)[..., None], lam[np.clip(idx, 0, n - 1)], 0.0)
    return -(lam_t * gu).sum(axis=(1, 2)), lam
