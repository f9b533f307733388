"""Differentiable static equilibrium: x*(theta) for per-tet Young's moduli theta.

Forward: Newton steps of the library on the static problem
E(x; theta) = sum_t Psi_t(x; theta_t) + sum_s kappa b(d_s) - sum_v m_v g . x_v
until max_v |grad_v E| <= gtol * max_v m_v |g|: projected steps first, then,
once the gradient is below ``EXACT_SWITCH`` of that scale, steps with the exact
Hessian (projected Newton converges only linearly where the projection still
clamps modes of indefinite local Hessians; the exact Hessian must be positive
definite at x* for the adjoint solve anyway).  An exact step whose PCG breaks
down or whose line search fails is replaced by a projected step.

Backward (implicit differentiation of grad_x E(x*; theta) = 0): with the
upstream gradient dL/dx*, solve H(x*) lambda = dL/dx* by the library's PCG on
the exact (unprojected) Hessian, then dL/dtheta_t = -lambda . d/dx Psi_t /
theta_t (Psi is linear in the modulus at fixed Poisson ratio), computed per tet
by ``yasps_theta_adjoint``.  Every step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from .yasps import E_BREAKDOWN, E_LINESEARCH, EXACT, PROJECTED, Yasps, YaspsError


class StaticEquilibrium:
    """Binds a static problem (``synth.c5_static``-shaped dict: ``mu1``, ``lam1``
    unit-modulus Lame parameters, per-tet ``mu_t``/``lam_t``) to a library
    context whose per-tet parameters are rewritten in place for each theta."""

    TIE_RTOL = 1e-14
    EXACT_SWITCH = 1e-3

    def __init__(self, prob, device="cuda", gtol=1e-10, max_newton=60, rtol=1e-12):
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

    def set_theta(self, theta):
        ml = self.lib._ml  # [2][n_t] device array read by every evaluation
        ml[0].copy_(theta * self.mu1)
        ml[1].copy_(theta * self.lam1)

    def _step(self, x, hessian):
        return self.lib.newton_step(x, rtol=self.rtol, max_iter=100000, tie_rtol=self.TIE_RTOL, hessian=hessian)

    def solve(self, x0):
        x = x0.detach().clone().contiguous()
        gmax = np.inf
        for k in range(self.max_newton):
            info = None
            if gmax <= self.EXACT_SWITCH * self.gscale:
                xk = x.clone()
                try:
                    info = self._step(x, EXACT)
                    if info["alpha"] == 0.0:
                        info = None
                except YaspsError as e:
                    if e.status not in (E_BREAKDOWN, E_LINESEARCH):
                        raise
                if info is None:
                    x.copy_(xk)
            if info is None:
                info = self._step(x, PROJECTED)
            self.newton_iters = k + 1
            # grad_max is the gradient at the start of the step
            if info["grad_max"] <= self.gtol * self.gscale:
                return x
            gmax = info["grad_max"]
        raise YaspsError(-5, f"static equilibrium not reached in {self.max_newton} Newton steps "
                             f"(max |g| = {info['grad_max']:.3e})")

    def adjoint(self, x_star, theta, dl_dx, rtol=1e-12):
        self.set_theta(theta)
        self.lib.eval(x_star, exact=True)
        self.lib.view()  # assemble the exact Hessian
        lam, info = self.lib.pcg(dl_dx.contiguous(), rtol=rtol, max_iter=100000, allow=())
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
