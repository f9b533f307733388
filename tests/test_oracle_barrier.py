"""Pins for the oracle's contact stencils: barrier closed forms, distance
definitions against brute-force minimisation, finite differences, cutoff,
fixed-vertex handling and PSD projection."""
import numpy as np
import pytest
import torch
from scipy.optimize import minimize

from oracle import energy as en
from oracle import local

torch.set_default_dtype(torch.float64)
DHAT, KAPPA = 1e-3, 1e4


def b_closed(d):
    """b, b', b'' of (d - dhat)^2 log(d/dhat)^2 derived by hand."""
    u, L = d - DHAT, np.log(d / DHAT)
    return (u * u * L * L, 2 * u * L * L + 2 * u * u * L / d,
            2 * L * L + 8 * u * L / d + 2 * u * u * (1 - L) / (d * d))


def test_barrier_vanishes_to_second_order_at_dhat():
    for v in b_closed(DHAT):
        assert v == 0.0
    d = torch.tensor(DHAT, requires_grad=True)
    b = en.barrier(d, DHAT, 1.0)
    (g,) = torch.autograd.grad(b, d, create_graph=True)
    (h,) = torch.autograd.grad(g, d)
    assert float(b) == 0.0 and float(g) == 0.0 and float(h) == 0.0


def test_barrier_derivatives_match_hand_derivation_and_decrease():
    ds = np.geomspace(1e-6, 0.999 * DHAT, 40)
    for dv in ds:
        d = torch.tensor(dv, requires_grad=True)
        b = en.barrier(d, DHAT, 1.0)
        (g,) = torch.autograd.grad(b, d, create_graph=True)
        (h,) = torch.autograd.grad(g, d)
        b0, b1, b2 = b_closed(dv)
        assert abs(float(b) - b0) <= 1e-13 * abs(b0) + 1e-300
        assert abs(float(g) - b1) <= 1e-12 * abs(b1)
        assert abs(float(h) - b2) <= 1e-12 * abs(b2)
        assert b1 < 0  # monotone decreasing on (0, dhat)


def _seg_pts(a, b, t):
    return a[None] + t[:, None] * (b - a)[None]


def brute_pt(p, t0, t1, t2):
    f = lambda uv: np.sum((t0 + uv[0] * (t1 - t0) + uv[1] * (t2 - t0) - p) ** 2)
    r = minimize(f, [1 / 3, 1 / 3], method="SLSQP", bounds=[(0, 1), (0, 1)],
                 constraints=[{"type": "ineq", "fun": lambda uv: 1 - uv[0] - uv[1]}],
                 options=dict(ftol=1e-20, maxiter=500))
    return r.fun, r.x


def brute_ee(a0, a1, b0, b1):
    f = lambda st: np.sum((a0 + st[0] * (a1 - a0) - b0 - st[1] * (b1 - b0)) ** 2)
    r = minimize(f, [0.5, 0.5], method="L-BFGS-B", bounds=[(0, 1), (0, 1)],
                 options=dict(ftol=1e-20, gtol=1e-14, maxiter=500))
    return r.fun, r.x


def brute_pe(p, e0, e1):
    t = np.linspace(0, 1, 20001)
    q = _seg_pts(e0, e1, t)
    k = np.argmin(((q - p) ** 2).sum(1))
    f = lambda s: np.sum((e0 + s[0] * (e1 - e0) - p) ** 2)
    r = minimize(f, [t[k]], method="L-BFGS-B", bounds=[(0, 1)], options=dict(ftol=1e-22, gtol=1e-15))
    return r.fun, r.x


def test_interior_distances_equal_true_minimum():
    rng = np.random.default_rng(3)
    n_ok = 0
    for _ in range(60):
        t0, t1, t2 = rng.normal(size=(3, 3))
        p = (t0 + t1 + t2) / 3 + 0.3 * rng.normal(size=3)
        dmin, uv = brute_pt(p, t0, t1, t2)
        if min(uv[0], uv[1], 1 - uv.sum()) > 1e-3:  # interior closest point
            x = torch.tensor(np.stack([p, t0, t1, t2]))
            assert abs(float(en.dist_pt(x)) - dmin) <= 1e-8 * dmin
            n_ok += 1
        a0, a1, b0, b1 = rng.normal(size=(4, 3))
        dmin, st = brute_ee(a0, a1, b0, b1)
        if min(st.min(), 1 - st.max()) > 1e-3:
            x = torch.tensor(np.stack([a0, a1, b0, b1]))
            assert abs(float(en.dist_ee(x)) - dmin) <= 1e-8 * dmin
            n_ok += 1
        e0, e1 = rng.normal(size=(2, 3))
        dmin, s = brute_pe(p, e0, e1)
        if 1e-3 < s[0] < 1 - 1e-3:
            x = torch.tensor(np.stack([p, e0, e1, np.zeros(3)]))
            assert abs(float(en.dist_pe(x)) - dmin) <= 1e-8 * dmin
            n_ok += 1
    assert n_ok > 60


def rand_stencils(n, t, seed, scale=0.02):
    """Stencils of type t with squared distance well inside (0, dhat)."""
    g = torch.Generator().manual_seed(seed)
    base = torch.tensor([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]) * 0.05
    if t == 0:
        base = torch.tensor([[0.3, 0.3, 0.02], [0, 0, 0], [1, 0, 0], [0, 1, 0]]) * 1.0 * 0.05 * torch.tensor([1, 1, 1.0])
        base[0, 2] = 0.02
    elif t == 1:
        base = torch.tensor([[0.0, 0.5, 0.0], [1.0, 0.5, 0.0], [0.5, 0.0, 0.4], [0.5, 1.0, 0.4]]) * 0.05
    elif t == 2:
        base = torch.tensor([[0.5, 0.3, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0]]) * 0.05
    else:
        base = torch.tensor([[0.0, 0.0, 0.0], [0.015, 0.01, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    x = base.unsqueeze(0) + 0.002 * torch.randn(n, 4, 3, generator=g)
    nv = en.N_VERTS[t]
    x[:, nv:] = 0.0
    return x


@pytest.mark.parametrize("t", [0, 1, 2, 3])
def test_finite_differences_contact(t):
    n = 24
    x = rand_stencils(n, t, 10 + t)
    ct = torch.full((n,), t)
    nv = en.N_VERTS[t]
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :nv] = True
    E, g, H, d = local.contact_local(x, ct, free, KAPPA, DHAT, local.EXACT)
    assert bool((d > 0).all()) and bool((d < DHAT).all())
    eps = 1e-7
    m = 3 * nv
    for k in range(m):
        dx = torch.zeros(n, 12)
        dx[:, k] = eps
        Ep, gp, _, _ = local.contact_local(x + dx.view(n, 4, 3), ct, free, KAPPA, DHAT, local.EXACT)
        Em, gm, _, _ = local.contact_local(x - dx.view(n, 4, 3), ct, free, KAPPA, DHAT, local.EXACT)
        gfd = (Ep - Em) / (2 * eps)
        Hfd = (gp - gm).reshape(n, 12) / (2 * eps)
        gs = g.reshape(n, 12).abs().amax(1)
        Hs = H.abs().amax((1, 2))
        assert float(((gfd - g.reshape(n, 12)[:, k]).abs() / gs).max()) < 1e-5
        assert float(((Hfd - H[:, :, k]).abs() / Hs[:, None]).max()) < 1e-5


def test_pp_gradient_closed_form():
    n = 30
    x = rand_stencils(n, 3, 4)
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :2] = True
    E, g, H, d = local.contact_local(x, torch.full((n,), 3), free, KAPPA, DHAT)
    for i in range(n):
        dv = float(d[i])
        b1 = b_closed(dv)[1]
        ref = KAPPA * b1 * 2 * (x[i, 1] - x[i, 0]).numpy()
        assert np.allclose(g[i, 1].numpy(), ref, rtol=1e-12, atol=0)
        assert np.allclose(g[i, 0].numpy(), -ref, rtol=1e-12, atol=0)


def test_cutoff_is_exactly_zero():
    n = 10
    x = rand_stencils(n, 3, 5)
    x[:, 1] = x[:, 0] + torch.tensor([0.0316227766016838 + 1e-4, 0.0, 0.0])  # d just above dhat
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :2] = True
    E, g, H, d = local.contact_local(x, torch.full((n,), 3), free, KAPPA, DHAT)
    assert bool((d >= DHAT).all())
    assert float(E.abs().max()) == 0 and float(g.abs().max()) == 0 and float(H.abs().max()) == 0


def test_nonpositive_distance_raises():
    x = torch.zeros(1, 4, 3)
    free = torch.ones(1, 4, dtype=torch.bool)
    with pytest.raises(ValueError):
        local.contact_local(x, torch.tensor([3]), free, KAPPA, DHAT)


@pytest.mark.parametrize("t", [0, 1, 2, 3])
def test_projected_contact_hessian_psd_and_fixed_vertices(t):
    n = 64
    x = rand_stencils(n, t, 20 + t)
    nv = en.N_VERTS[t]
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :nv] = True
    free[::2, 0] = False  # half of them have a fixed first vertex
    E, g, H, d = local.contact_local(x, torch.full((n,), t), free, KAPPA, DHAT)
    _, _, He, _ = local.contact_local(x, torch.full((n,), t), free, KAPPA, DHAT, local.EXACT)
    w = torch.linalg.eigvalsh(H)
    assert float((w.min(1).values / w.abs().max(1).values.clamp(min=1e-300)).min()) > -1e-12
    assert float(H[::2, :3].abs().max()) == 0 and float(H[::2, :, :3].abs().max()) == 0
    assert float(g[::2, 0].abs().max()) == 0
    # projection only adds a PSD correction to the free principal submatrix
    wd = torch.linalg.eigvalsh(H - He)
    assert float((wd.min(1).values / He.abs().amax((1, 2))).min()) > -1e-12


def test_rigid_motion_invariance_of_distances():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    sh = rng.normal(size=3)
    for t in range(4):
        x = rand_stencils(5, t, 30 + t)
        y = x @ torch.tensor(Q).T + torch.tensor(sh)
        for i in range(5):
            a, b = float(en.DIST[t](x[i])), float(en.DIST[t](y[i]))
            assert abs(a - b) <= 1e-11 * a


# ---------------------------------------------------------------- classic IPC barrier
# The alternative reading of the printed barrier (section "Eigendecomposition:
# Automatic Optimization"): b(d) = -(d - dhat)^2 log(d / dhat), d squared.


def b_classic_closed(d):
    """b, b', b'' of -(d - dhat)^2 log(d/dhat) derived by hand: with u = d - dhat
    and L = log(d/dhat), b' = -2uL - u^2/d and b'' = -2L - 4u/d + u^2/d^2."""
    u, L = d - DHAT, np.log(d / DHAT)
    return -u * u * L, -2 * u * L - u * u / d, -2 * L - 4 * u / d + u * u / (d * d)


def _derivs(fun, dv):
    d = torch.tensor(dv, requires_grad=True)
    b = fun(d, DHAT, 1.0)
    (g,) = torch.autograd.grad(b, d, create_graph=True)
    (h,) = torch.autograd.grad(g, d)
    return float(b.detach()), float(g.detach()), float(h)


def test_classic_barrier_vanishes_to_second_order_at_dhat():
    assert b_classic_closed(DHAT) == (0.0, 0.0, 0.0)
    assert _derivs(en.barrier_ipc_classic, DHAT) == (0.0, 0.0, 0.0)
    # near dhat it vanishes like (d - dhat)^3: b / u^3 -> -1 / dhat
    for u in (1e-7, -1e-7, 1e-8):
        b = float(en.barrier_ipc_classic(torch.tensor(DHAT + u), DHAT, 1.0))
        assert abs(b / u ** 3 + 1.0 / DHAT) <= 1e-3 / DHAT


def test_classic_barrier_closed_forms_monotone_convex():
    for dv in np.geomspace(1e-7, 0.999 * DHAT, 40):
        b, g, h = _derivs(en.barrier_ipc_classic, dv)
        b0, b1, b2 = b_classic_closed(dv)
        assert abs(b - b0) <= 1e-13 * abs(b0)
        assert abs(g - b1) <= 1e-12 * abs(b1)
        assert abs(h - b2) <= 1e-12 * abs(b2)
        assert b0 > 0 and b1 < 0 and b2 > 0  # positive, decreasing and convex on (0, dhat)


def test_classic_barrier_special_value_and_kappa_scaling():
    # at d = dhat / e the log is -1 and b = (dhat (1 - 1/e))^2
    d = DHAT / np.e
    b = float(en.barrier_ipc_classic(torch.tensor(d), DHAT, 1.0))
    assert abs(b - (DHAT * (1 - 1 / np.e)) ** 2) <= 1e-15 * b
    assert float(en.barrier_ipc_classic(torch.tensor(d), DHAT, KAPPA)) == pytest.approx(KAPPA * b, rel=1e-15)


def test_classic_barrier_finite_differences():
    for dv in (2e-5, 3e-4, 9e-4):
        eps = 1e-6 * dv
        f = lambda t: float(en.barrier_ipc_classic(torch.tensor(t), DHAT, 1.0))
        _, b1, b2 = b_classic_closed(dv)
        assert abs((f(dv + eps) - f(dv - eps)) / (2 * eps) - b1) <= 1e-7 * abs(b1)
        g = lambda t: b_classic_closed(t)[1]
        assert abs((g(dv + eps) - g(dv - eps)) / (2 * eps) - b2) <= 1e-7 * abs(b2)


def test_classic_pp_gradient_closed_form_and_cutoff():
    n = 30
    x = rand_stencils(n, 3, 41)
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :2] = True
    E, g, H, d = local.contact_local(x, torch.full((n,), 3), free, KAPPA, DHAT, classic=True)
    for i in range(n):
        dv = float(d[i])
        b0, b1, _ = b_classic_closed(dv)
        assert float(E[i]) == pytest.approx(KAPPA * b0, rel=1e-12)
        ref = KAPPA * b1 * 2 * (x[i, 1] - x[i, 0]).numpy()
        assert np.allclose(g[i, 1].numpy(), ref, rtol=1e-12, atol=0)
        assert np.allclose(g[i, 0].numpy(), -ref, rtol=1e-12, atol=0)
    x[:, 1] = x[:, 0] + torch.tensor([0.0316227766016838 + 1e-4, 0.0, 0.0])
    E, g, H, d = local.contact_local(x, torch.full((n,), 3), free, KAPPA, DHAT, classic=True)
    assert bool((d >= DHAT).all())
    assert float(E.abs().max()) == 0 and float(g.abs().max()) == 0 and float(H.abs().max()) == 0


@pytest.mark.parametrize("t", [0, 1, 2, 3])
def test_classic_finite_differences_contact(t):
    n = 12
    x = rand_stencils(n, t, 50 + t)
    ct = torch.full((n,), t)
    nv = en.N_VERTS[t]
    free = torch.zeros(n, 4, dtype=torch.bool)
    free[:, :nv] = True
    E, g, H, d = local.contact_local(x, ct, free, KAPPA, DHAT, local.EXACT, classic=True)
    eps = 1e-7
    for k in range(3 * nv):
        dx = torch.zeros(n, 12)
        dx[:, k] = eps
        Ep, gp, _, _ = local.contact_local(x + dx.view(n, 4, 3), ct, free, KAPPA, DHAT, local.EXACT, classic=True)
        Em, gm, _, _ = local.contact_local(x - dx.view(n, 4, 3), ct, free, KAPPA, DHAT, local.EXACT, classic=True)
        gs = g.reshape(n, 12).abs().amax(1)
        Hs = H.abs().amax((1, 2))
        assert float((((Ep - Em) / (2 * eps) - g.reshape(n, 12)[:, k]).abs() / gs).max()) < 1e-5
        assert float((((gp - gm).reshape(n, 12) / (2 * eps) - H[:, :, k]).abs() / Hs[:, None]).max()) < 1e-5
