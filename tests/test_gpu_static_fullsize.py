"""Differentiation form on the full-size static block (48x48x29 cells, 400,896
tets with per-tet moduli, 300k PT stencils, bottom rim fixed), solved as
bench.py times it: the library's equilibrium x* is checked on the oracle's
gradient rows of sampled vertices (the stop rule holds there), the adjoint
lambda on the oracle's exact Hessian rows (H(x*) lambda = dL/dx* there), the
per-tet theta gradient on the oracle's unit-modulus tet gradients of sampled
tets, and the whole theta gradient against central finite differences of the
GPU forward solve along seeded directions (every tet perturbed at once)."""
import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import assemble as oasm
from paper_2605_23088_amd import synth
from parity_util import TOL, restrict, scales

pytestmark = pytest.mark.gpu
GTOL = 1e-9


@pytest.fixture(scope="module")
def solved():
    from paper_2605_23088_amd.adjoint import StaticEquilibrium
    p = synth.c5_static()
    s = StaticEquilibrium(p, gtol=GTOL)
    theta = torch.as_tensor(p["theta"], dtype=torch.float64, device="cuda")
    x0 = torch.as_tensor(p["x0"], dtype=torch.float64, device="cuda").contiguous()
    xt = torch.as_tensor(p["x_tgt"], dtype=torch.float64, device="cuda")
    s.set_theta(theta)
    xs = s.solve(x0)
    g, lam = s.adjoint(xs, theta, 2.0 * (xs - xt))
    print(f"static block: equilibrium in {s.newton_iters} Newton steps", flush=True)
    return p, s, theta, xs, xt, g.cpu().numpy(), lam.cpu().numpy()


def test_equilibrium_and_adjoint_rows(solved):
    p, _, _, xs, _, _, lam = solved
    x = xs.cpu().numpy()
    n = p["n_free"]
    rng = np.random.default_rng(20265)
    cverts = np.unique(p["cidx"][:, 1:])
    cverts = cverts[cverts < n]
    S = np.unique(np.concatenate([rng.choice(n, 32, replace=False), rng.choice(cverts, 32, replace=False)]))
    o = oasm.Oracle(restrict(p, S))
    ev = o.eval(x, oasm.EXACT)
    asm = o.assemble(ev)
    _, _, gs, _ = scales(o, ev, x)
    # the stop rule max_v |g_v| <= GTOL m_max |gravity| on the sampled rows, up to rounding
    gscale = float(np.max(p["mass"]) * np.linalg.norm(p["gravity"]))
    gn = np.sqrt((asm["grad"][S] ** 2).sum(1))
    assert np.all(gn <= GTOL * gscale + TOL * np.sqrt((gs[S] ** 2).sum(1))), gn.max() / gscale
    # adjoint: the rows of H(x*) lambda - 2 (x* - x_tgt) are within the PCG stop
    # (1e-12 of |b|) plus the rounding of the two sides' exact Hessians
    H = o.csr(asm)
    rows = (3 * S[:, None] + np.arange(3)).ravel()
    b = 2.0 * (x - p["x_tgt"]).ravel()
    lv = lam.ravel()
    r = H[rows] @ lv - b[rows]
    mag = abs(H[rows]) @ np.abs(lv)
    assert np.all(np.abs(r) <= 1e-12 * np.linalg.norm(b) + 2 * TOL * mag), np.abs(r).max()


def test_theta_gradient_sampled_tets(solved):
    p, _, _, xs, _, g, lam = solved
    x = xs.cpu().numpy()
    rng = np.random.default_rng(20266)
    T = np.sort(rng.choice(len(p["tet_idx"]), 64, replace=False))
    q = dict(p)
    for key in ("tet_idx", "dm_inv", "vol", "mu_t", "lam_t"):
        q[key] = p[key][T]
    q["ctype"], q["cidx"] = p["ctype"][:0], p["cidx"][:0]
    gu = oadj.unit_gradients(oasm.Oracle(q), x)  # (64, 4, 3), fixed vertices zeroed
    idx = q["tet_idx"]
    n = p["n_free"]
    lam_t = np.where((idx < n)[..., None], lam[np.clip(idx, 0, n - 1)], 0.0)
    ref = -(lam_t * gu).sum(axis=(1, 2))
    # rounding scale: |lambda| times the unit-modulus stress scale of the tet
    dm = q["dm_inv"]
    st = q["vol"] * (p["mu1"] + p["lam1"]) * np.sqrt((dm * dm).sum(axis=(1, 2))) * 4.0
    mag = (np.abs(lam_t) * np.maximum(np.abs(gu), st[:, None, None])).sum(axis=(1, 2))
    assert np.all(np.abs(g[T] - ref) <= TOL * mag), np.abs(g[T] - ref).max()


def test_theta_gradient_finite_differences(solved):
    p, s, theta, xs, xt, g, _ = solved
    rng = np.random.default_rng(20267)
    eps = 1e-6
    gtol = s.gtol
    # perturbed solves well below the change they measure, and above the
    # rounding floor of max|g| (about 2e-11 of the weight scale here)
    s.gtol = 1e-10
    try:
        for _ in range(3):
            d = rng.standard_normal(len(g)) * p["theta"]
            dt = torch.as_tensor(d, dtype=torch.float64, device="cuda")
            L = []
            for sgn in (1.0, -1.0):
                s.set_theta(theta + sgn * eps * dt)
                L.append(float(((s.solve(xs) - xt) ** 2).sum()))
            fd = (L[0] - L[1]) / (2 * eps)
            an = float(g @ d)
            print(f"directional derivative: adjoint {an:.9e}, central difference {fd:.9e}", flush=True)
            assert abs(fd - an) <= 1e-4 * np.abs(g * d).sum()
    finally:
        s.gtol = gtol
        s.set_theta(theta)
