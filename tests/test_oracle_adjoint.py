"""Pins for the oracle's adjoint of the static-equilibrium solve: central finite
differences of L(theta) = |x*(theta) - x_tgt|^2 on seeded tets, and the special
case x_tgt = x* where the adjoint vector and the gradient vanish exactly."""
import numpy as np
import pytest

from oracle import adjoint
from oracle import assemble as oasm
from paper_2605_23088_amd import synth

GTOL = 5e-11


@pytest.fixture(scope="module")
def static_case():
    p = synth.c5_static(seed=21, nx=4, ny=3, nz=3, a=0.05, n_pt=40, kappa=1e4, pin="corners")
    o = oasm.Oracle(p)
    adjoint.set_theta(o, p["theta"])
    xs, _ = adjoint.solve_equilibrium(o, p["x0"], gtol=GTOL)
    return p, o, xs


def test_adjoint_matches_central_differences(static_case):
    p, o, xs = static_case
    g, _ = adjoint.theta_gradient(o, xs, p["x_tgt"])
    L = lambda x: float(((x - p["x_tgt"]) ** 2).sum())
    rng = np.random.default_rng(20265)
    gmax = np.abs(g).max()
    for t in rng.choice(len(g), 6, replace=False):
        th = p["theta"].copy()
        eps = 1e-4 * th[t]
        th[t] += eps
        adjoint.set_theta(o, th)
        xp, _ = adjoint.solve_equilibrium(o, xs, gtol=GTOL)
        th[t] -= 2 * eps
        adjoint.set_theta(o, th)
        xm, _ = adjoint.solve_equilibrium(o, xs, gtol=GTOL)
        fd = (L(xp) - L(xm)) / (2 * eps)
        assert abs(g[t] - fd) <= 1e-3 * abs(fd) + 1e-8 * gmax, (t, g[t], fd)
    adjoint.set_theta(o, p["theta"])


def test_adjoint_vanishes_at_the_target(static_case):
    p, o, xs = static_case
    g, lam = adjoint.theta_gradient(o, xs, xs)
    assert np.abs(lam).max() == 0.0 and np.abs(g).max() == 0.0


def test_equilibrium_is_stationary(static_case):
    p, o, xs = static_case
    ok, gmax = adjoint.converged(o, xs, gtol=GTOL)
    assert ok
