"""Differentiable static equilibrium: x*(theta) for per-tet Young's moduli theta.

Forward: damped exact Newton steps of the library on the static problem
E(x; theta) = sum_t Psi_t(x; theta_t) + sum_s kappa b(d_s) - sum_v m_v g . x_v
until max_v |grad_v E| <= gtol * max_v m_v |g|: each step solves
(H_exact + mu M) p = -g (Levenberg-Marquardt with the lumped masses) and
line-searches E; mu grows when a step fails (indefinite H_exact away from the
minimum) and vanishes near it, where the iteration is plain exact Newton
(quadratic).  Projected Newton alone converges only linearly wherever the
projection clamps modes of indefinite local Hessians, and on the 48x48x29
static block it stalls.

Backward (implicit differentiation of grad_x E(x*; theta) = 0): with the
upstream gradient dL/dx*, solve H(x*) lambda = dL/dx* by the library's PCG on
the exact (unprojected) Hessian, then dL/dtheta_t = -lambda . d/dx Psi_t /
theta_t (Psi is linear in the modulus at fixed Poisson ratio), computed per tet
by ``yasps_theta_adjoint``.  Every step runs in the library's kernels.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

from .yasps import E_BREAKDOWN, E_LINESEARCH, EXACT, PROJECTED, Yasps, YaspsError


class StaticEquilibrium:
    """Binds a static problem (``synth.c5_static``-shaped dict: ``mu1``, ``lam1``
    unit-modulus Lame parameters, per-tet ``mu_t``/``lam_t``) to a library
    context whose per-tet parameters are rewritten in place for each theta."""

    TIE_RTOL = 1e-14

    def __init__(self, prob, device="cuda", gtol=1e-10, max_newton=60, rtol=1e-12, verbose=False):
        if "mu_t" not in prob:
            raise ValueError("the problem needs per-tet Lame parameters")
        self.prob = prob
        self.lib = Yasps(prob, device=device)
        self.mu1 = float(prob["mu1"])
        self.lam1 = float(prob["lam1"])
        self.gtol = gtol
        self.max_newton = max_newton
        self.rtol = rtol
        m = np.asarray(prob["mass"])
        self.gscale = float(m.max() * np.linalg.norm(prob["gravity"]))
        self.newton_iters = 0
        self.exact_steps = 0
        self.cg_iters = 0  # PCG iterations of the accepted steps of the last solve
        self.adjoint_info = None  # PCG info of the last adjoint solve
        self.verbose = verbose

    def set_theta(self, theta):
        ml = self.lib._ml  # [2][n_t] device array read by every evaluation
        ml[0].copy_(theta * self.mu1)
        ml[1].copy_(theta * self.lam1)

    def _step(self, x, hessian, shift=0.0):
        # an exact-Hessian attempt away from the minimum may never converge: bound it
        cap = 20000 if hessian == EXACT else 100000
        return self.lib.newton_step(x, rtol=self.rtol, max_iter=cap, tie_rtol=self.TIE_RTOL, hessian=hessian,
                                    shift=shift)

    def _shift_scale(self):
        """A Levenberg-Marquardt shift of 1 % of the median diagonal of the last
        assembled Hessian, in units of the mass (the shift multiplies m_v)."""
        return self.lib.lm_shift(1e-2)

    def solve(self, x0):
        """Damped exact Newton: each step solves (H_exact + mu M) p = -g and
        takes the line search on E.  mu starts at 0; a step whose PCG breaks
        down, whose direction is not one of descent, or whose line search fails
        is retried with a larger mu (x unchanged), and mu shrinks after full
        steps, so the iteration becomes plain exact Newton near the minimum."""
        x = x0.detach().clone().contiguous()
        xk = torch.empty_like(x)
        self.exact_steps = 0
        self.cg_iters = 0
        mu, mu0 = 0.0, None
        info = {"grad_max": float("inf")}
        for k in range(self.max_newton):
            xk.copy_(x)
            ok = True
            try:
                info = self._step(x, EXACT, mu)
                ok = info["alpha"] > 0.0
            except YaspsError as e:
                if e.status not in (E_BREAKDOWN, E_LINESEARCH):
                    raise
                ok = False
            self.newton_iters = k + 1
            if not ok:
                x.copy_(xk)
                if mu0 is None:
                    mu0 = self._shift_scale()
                mu = mu0 if mu == 0.0 else 4.0 * mu
                if self.verbose:
                    print(f"[equilibrium] step {k}: rejected, shift -> {mu:.3e}", file=sys.stderr, flush=True)
                continue
            self.exact_steps += 1
            self.cg_iters += info["cg_iters"]
            if self.verbose:
                print(f"[equilibrium] step {k}: shift {mu:.3e}, max|g| {info['grad_max']:.3e}, "
                      f"alpha {info['alpha']:.3g}, {info['cg_iters']} PCG iterations", file=sys.stderr, flush=True)
            # grad_max is the gradient at the start of the step
            if info["grad_max"] <= self.gtol * self.gscale:
                return x
            if info["alpha"] == 1.0 and mu > 0.0:
                mu = 0.0 if mu0 is not None and mu / 4.0 < 1e-6 * mu0 else mu / 4.0
        raise YaspsError(-5, f"static equilibrium not reached in {self.max_newton} Newton steps "
                             f"(max |g| = {info['grad_max']:.3e})")

    def adjoint(self, x_star, theta, dl_dx, rtol=1e-12):
        self.set_theta(theta)
        self.lib.eval(x_star, exact=True)
        self.lib.view()  # assemble the exact Hessian
        lam, info = self.lib.pcg(dl_dx.contiguous(), rtol=rtol, max_iter=100000, allow=())
        self.adjoint_info = info
        return self.lib.theta_adjoint(x_star, lam, theta.contiguous()), lam


class YaspsEquilibrium(torch.autograd.Function):
    """x* = YaspsEquilibrium.apply(theta, solver, x0)."""

    @staticmethod
    def forward(ctx, theta, solver, x0):
        solver.set_theta(theta)
        x = solver.solve(x0)
        ctx.solver = solver
        ctx.save_for_backward(theta, x)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        theta, x = ctx.saved_tensors
        g_theta, _ = ctx.solver.adjoint(x, theta, grad_x)
        return g_theta, None, None
