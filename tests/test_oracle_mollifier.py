"""Pins of the oracle's edge-edge mollifier (IPC's near-parallel treatment):
m(c) = -c^2/eps^2 + 2c/eps below eps, 1 above, on c = |e_a x e_b|^2.

Against closed forms: the mollifier's values and its C^1 join at eps, the
cross norm of two edges at a known angle, and the whole mollified barrier of
two crossing edges at a known separation and angle; the parallel limit; the
line-search energy path against the evaluation path; central differences of
the mollified stencil's gradient and Hessian.
"""
import math

import numpy as np
import pytest
import torch

from oracle import energy as en
from oracle import local

KAPPA, DHAT = 1e4, 1e-3


def crossing_edges(la, lb, theta, h):
    """Edge a along x through the origin, edge b at angle theta in the plane
    z = -h, both centred over the origin: line distance h, c = la^2 lb^2 sin^2."""
    a0 = torch.tensor([-la / 2, 0.0, 0.0])
    a1 = torch.tensor([la / 2, 0.0, 0.0])
    u = torch.tensor([math.cos(theta), math.sin(theta), 0.0])
    b0 = torch.tensor([0.0, 0.0, -h]) - lb / 2 * u
    b1 = torch.tensor([0.0, 0.0, -h]) + lb / 2 * u
    return torch.stack([a0, a1, b0, b1])


def test_mollifier_values_and_c1_join():
    eps = torch.tensor(2.5e-3, dtype=torch.float64)
    m = lambda c: en.ee_mollifier(torch.as_tensor(c, dtype=torch.float64), eps)
    assert float(m(0.0)) == 0.0
    assert float(m(float(eps))) == 1.0
    assert float(m(0.5 * float(eps))) == pytest.approx(0.75, rel=1e-15)
    assert float(m(3.0 * float(eps))) == 1.0
    # increasing on [0, eps), slope 2/eps at 0, slope 0 at eps from below
    cs = torch.linspace(0.0, float(eps) * (1 - 1e-12), 101, dtype=torch.float64)
    assert bool((torch.diff(m(cs)) > 0).all())
    g = torch.func.grad(lambda c: en.ee_mollifier(c, eps))
    assert float(g(torch.tensor(0.0, dtype=torch.float64))) == pytest.approx(2.0 / float(eps), rel=1e-14)
    assert abs(float(g(torch.tensor(float(eps) * (1 - 1e-9), dtype=torch.float64)))) < 1e-6 / float(eps)
    # eps <= 0: no mollifier
    assert float(en.ee_mollifier(torch.tensor(0.0, dtype=torch.float64), torch.tensor(0.0, dtype=torch.float64))) == 1.0


@pytest.mark.parametrize("theta", [0.3, 1.2, 0.01])
def test_cross_norm_closed_form(theta):
    la, lb = 0.25, 0.25 * math.sqrt(2.0)
    x = crossing_edges(la, lb, theta, 0.02)
    c = float(en.ee_cross_norm(x))
    assert c == pytest.approx(la ** 2 * lb ** 2 * math.sin(theta) ** 2, rel=1e-13)


@pytest.mark.parametrize("theta,mollified", [(0.01, True), (0.025, True), (0.2, False)])
def test_mollified_barrier_closed_form(theta, mollified):
    la, lb, h = 0.25, 0.25, 0.02
    x = crossing_edges(la, lb, theta, h)
    eps = 1e-3 * la ** 2 * lb ** 2
    c = la ** 2 * lb ** 2 * math.sin(theta) ** 2
    assert (c < eps) == mollified
    m = -(c / eps) ** 2 + 2 * c / eps if c < eps else 1.0
    d = h * h
    b = (d - DHAT) ** 2 * math.log(d / DHAT) ** 2
    free = torch.ones(1, 4, dtype=torch.bool)
    E, g, H, dd = local.contact_local(x[None], torch.tensor([1]), free, KAPPA, DHAT, local.EXACT,
                                      eps=np.array([eps]))
    assert float(dd[0]) == pytest.approx(d, rel=1e-13)
    assert float(E[0]) == pytest.approx(KAPPA * m * b, rel=1e-12)
    # without thresholds the plain barrier
    E0, _, _, _ = local.contact_local(x[None], torch.tensor([1]), free, KAPPA, DHAT, local.EXACT)
    assert float(E0[0]) == pytest.approx(KAPPA * b, rel=1e-12)
    if not mollified:
        assert float(E[0]) == float(E0[0])


def test_parallel_limit():
    """At a fixed line distance the mollified energy and its gradient vanish as
    the edges turn parallel (the unmollified gradient grows like 1/theta)."""
    la = lb = 0.25
    eps = 1e-3 * la ** 2 * lb ** 2
    free = torch.ones(1, 4, dtype=torch.bool)
    last_e, last_g = None, None
    for theta in [1e-2, 1e-3, 1e-4]:
        x = crossing_edges(la, lb, theta, 0.02)
        # move b sideways within its plane (the line distance stays h)
        x[2:, 1] += 0.3 * lb
        E, g, _, _ = local.contact_local(x[None], torch.tensor([1]), free, KAPPA, DHAT, eps=np.array([eps]))
        gn = float(g.norm())
        if last_e is not None:
            assert float(E[0]) < 0.02 * last_e and gn < 0.2 * last_g
        last_e, last_g = float(E[0]), gn


def test_fd_gradient_and_hessian_of_the_mollified_stencil():
    la, lb = 0.25, 0.3
    x = crossing_edges(la, lb, 0.015, 0.02).clone()
    x += 1e-3 * torch.tensor(np.random.default_rng(3).normal(size=(4, 3)))
    eps = 1e-3 * la ** 2 * lb ** 2
    c = float(en.ee_cross_norm(x))
    assert c < eps
    free = torch.ones(1, 4, dtype=torch.bool)

    def energy(y):
        return float(local.contact_local(y[None], torch.tensor([1]), free, KAPPA, DHAT, local.EXACT,
                                         eps=np.array([eps]))[0][0])

    E, g, H, _ = local.contact_local(x[None], torch.tensor([1]), free, KAPPA, DHAT, local.EXACT,
                                     eps=np.array([eps]))
    step = 1e-6
    gf = np.zeros(12)
    for k in range(12):
        e = torch.zeros(12)
        e[k] = step
        gf[k] = (energy(x + e.view(4, 3)) - energy(x - e.view(4, 3))) / (2 * step)
    assert np.abs(gf - g[0].reshape(-1).numpy()).max() <= 1e-5 * np.abs(gf).max()

    def grad_at(y):
        return local.contact_local(y[None], torch.tensor([1]), free, KAPPA, DHAT, local.EXACT,
                                   eps=np.array([eps]))[1][0].reshape(-1).numpy()

    Hf = np.zeros((12, 12))
    for k in range(12):
        e = torch.zeros(12)
        e[k] = step
        Hf[:, k] = (grad_at(x + e.view(4, 3)) - grad_at(x - e.view(4, 3))) / (2 * step)
    assert np.abs(Hf - H[0].numpy()).max() <= 1e-4 * np.abs(Hf).max()


def test_line_search_energy_includes_the_mollifier():
    from oracle import assemble as oasm
    from paper_2605_23088_amd import synth
    p = synth.block_problem(4, 3, 2, 0.25, 20, 60, 11, ee_angle=(0.005, 0.06))
    o = oasm.Oracle(p)
    m = o.mollifiers(p["x0"]).numpy()
    assert (m < 1.0).sum() >= 10 and (m[p["ctype"] == 0] == 1.0).all()
    ev = o.eval(p["x0"])
    assert o.energy(p["x0"]) == pytest.approx(ev["E"], rel=1e-14)
    assert np.abs(o.energy_parts(p["x0"])["contact_terms"] - ev["E_c"]).max() <= 1e-14 * np.abs(ev["E_c"]).max()
