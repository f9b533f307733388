"""Pins for the oracle's step-length rule and side test on hand-built scenes
whose distances and step sizes are known in closed form:

* initial_step: alpha_0 = min(1, 0.4 sqrt(min_s d_s) / max_v |p_v|) over every
  contact stencil (active or not), 1 without contacts or with p = 0;
* signed_side: (p - t0) . ((t1 - t0) x (t2 - t0)) for point-triangle and
  (a0 - b0) . ((a1 - a0) x (b1 - b0)) for edge-edge stencils, 1 otherwise.
"""
import numpy as np
import pytest
import torch

from oracle import assemble, newton
from oracle import energy as en

PT, EE, PE, PP = 0, 1, 2, 3


def scene(contacts, x_fixed):
    """Three free vertices (a unit right triangle in z = 0), no tets, the given
    contact stencils (type, ids) against the given fixed vertices."""
    x0 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    ct = np.array([c[0] for c in contacts], np.int32)
    ci = np.array([c[1] for c in contacts], np.int32).reshape(-1, 4)
    return dict(n_free=3, x0=x0, x_fixed=np.asarray(x_fixed, np.float64).reshape(-1, 3), mass=np.ones(3),
                x_tilde=x0.copy(), tet_idx=np.zeros((0, 4), np.int32), dm_inv=np.zeros((0, 3, 3)),
                vol=np.zeros(0), ctype=ct, cidx=ci, mu=1.0, lam=1.0, h=0.01, kappa=1.0, dhat=1e-3,
                gravity=np.array([0.0, 0.0, -9.81]), static=False)


# PT: fixed point 0.03 below the triangle (d = 9e-4); PP: fixed point 0.01 above
# vertex 1 (d = 1e-4); PP: fixed point 0.05 from vertex 2 (d = 2.5e-3, inactive)
FIXED = [[0.2, 0.2, -0.03], [1.0, 0.0, 0.01], [0.0, 1.05, 0.0]]
CONTACTS = [(PT, [3, 0, 1, 2]), (PP, [1, 4, -1, -1]), (PP, [2, 5, -1, -1])]
P_DIR = np.array([[0.0, 0.0, 0.05], [0.03, 0.04, 0.0], [0.06, 0.08, 0.0]])  # max |p_v| = 0.1


def test_distances_of_the_hand_built_scene():
    o = assemble.Oracle(scene(CONTACTS, FIXED))
    d = o.distances(o.p["x0"])
    assert d == pytest.approx([9e-4, 1e-4, 2.5e-3], rel=1e-12)


def test_initial_step_closed_form():
    o = assemble.Oracle(scene(CONTACTS, FIXED))
    x = o.p["x0"]
    # 0.4 sqrt(1e-4) / 0.1 = 0.04
    assert newton.initial_step(o, x, P_DIR) == pytest.approx(0.04, rel=1e-13)
    # a short direction is not bounded: 0.4 * 0.01 / 0.001 = 4 -> 1
    assert newton.initial_step(o, x, 0.01 * P_DIR) == 1.0
    # the bound scales inversely with max |p_v| (here 0.2 -> 0.02)
    assert newton.initial_step(o, x, 2.0 * P_DIR) == pytest.approx(0.02, rel=1e-13)
    assert newton.initial_step(o, x, np.zeros_like(P_DIR)) == 1.0


def test_initial_step_counts_inactive_stencils_and_needs_contacts():
    # only the inactive stencil (d = 2.5e-3 >= dhat): 0.4 * 0.05 / 0.1 = 0.2
    o = assemble.Oracle(scene([CONTACTS[2]], FIXED))
    assert newton.initial_step(o, o.p["x0"], P_DIR) == pytest.approx(0.2, rel=1e-13)
    o = assemble.Oracle(scene([], np.zeros((0, 3))))
    assert newton.initial_step(o, o.p["x0"], P_DIR) == 1.0


def test_signed_side_closed_forms():
    x = torch.zeros(4, 4, 3, dtype=torch.float64)
    # PT, point above a triangle in z = 0 (normal +z, |n| = 2): 0.5 * 2
    x[0] = torch.tensor([[0.2, 0.2, 0.5], [0, 0, 0], [2, 0, 0], [0, 1, 0]], dtype=torch.float64)
    # PT, the same point below: -1
    x[1] = x[0]
    x[1, 0, 2] = -0.5
    # EE, a0 - b0 = (-0.5, 0.5, -0.3), n = (1,0,0) x (0,1,0) = +z: -0.3
    x[2] = torch.tensor([[0, 0, 0], [1, 0, 0], [0.5, -0.5, 0.3], [0.5, 0.5, 0.3]], dtype=torch.float64)
    # EE with the second edge reversed: the normal flips, +0.3
    x[3] = x[2][[0, 1, 3, 2]]
    s = en.signed_side(x, torch.tensor([PT, PT, EE, EE]))
    assert s.tolist() == pytest.approx([1.0, -1.0, -0.3, 0.3], rel=1e-15)
    # point-edge and point-point stencils carry no side
    assert en.signed_side(x[:2], torch.tensor([PE, PP])).tolist() == [1.0, 1.0]


def test_line_search_armijo_halvings_closed_form():
    """Inertia only: E(x) = 1/2 sum m |x - x_tilde|^2 and the direction
    p = -4 (x - x_tilde) give E(x + alpha p) = (1 - 4 alpha)^2 E(x) and
    g . p = -8 E(x).  Armijo (c = 1e-4) rejects alpha = 1 (9 E) and 0.5 (E) and
    accepts alpha = 0.25 (0): three trials, E1 = 0 up to rounding."""
    p = scene([], np.zeros((0, 3)))
    p["x_tilde"] = p["x0"] + np.array([[0.1, 0.0, 0.0], [0.0, -0.2, 0.0], [0.0, 0.0, 0.3]])
    o = assemble.Oracle(p)
    x = p["x0"]
    ev = o.eval(x)
    E0 = ev["E"]
    assert E0 == pytest.approx(0.5 * (0.01 + 0.04 + 0.09), rel=1e-14)
    g = o.assemble(ev)["grad"]
    d = -4.0 * (x - p["x_tilde"])
    assert float(g.ravel() @ d.ravel()) == pytest.approx(-8.0 * E0, rel=1e-14)
    alpha, x1, E1, trials = newton.line_search(o, x, d, E0, g)
    assert alpha == 0.25 and trials == 3
    assert abs(E1) <= 1e-15 * E0
    assert np.abs(x1 - p["x_tilde"]).max() <= 1e-15
