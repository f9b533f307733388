"""Per-stencil energy, gradient and PSD-projected local Hessian (float64, CPU).

Derivatives are exact derivatives of the definitions in ``energy.py`` taken by
``torch.func`` automatic differentiation; projection is ``torch.linalg.eigh``
followed by clamping negative eigenvalues to zero (section "Eigendecomposition
(EVD) and PSD Projection").
"""
from __future__ import annotations

import numpy as np
import torch
from torch.func import grad, hessian, jacrev, vmap

from . import energy as en

F_SPACE, X_SPACE = 0, 1
PROJECTED, EXACT = 0, 1

torch.set_default_dtype(torch.float64)


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.asarray(a), dtype=dtype)


def sym(A):
    """(A + A^T) / 2: local Hessians are stored exactly symmetric, so the
    assembled diagonal blocks (stored in full) are exactly symmetric too."""
    return 0.5 * (A + A.transpose(-1, -2))


def psd_project(A):
    """Proj(A) = Q max(Lambda, 0) Q^T (the Frobenius-nearest PSD matrix), batched."""
    A = 0.5 * (A + A.transpose(-1, -2))
    lam, Q = torch.linalg.eigh(A)
    P = (Q * lam.clamp(min=0.0).unsqueeze(-2)) @ Q.transpose(-1, -2)
    return 0.5 * (P + P.transpose(-1, -2))


def project_principal(H, mask):
    """Project the principal submatrix of each H (n, m, m) selected by the boolean
    mask (n, m) and return it embedded back (zeros outside the mask)."""
    out = torch.zeros_like(H)
    if H.shape[0] == 0:
        return out
    keys = mask.to(torch.int64) @ (2 ** torch.arange(mask.shape[1], dtype=torch.int64))
    for key in torch.unique(keys).tolist():
        rows = torch.nonzero(keys == key).flatten()
        idx = torch.nonzero(mask[rows[0]]).flatten()
        if idx.numel() == 0:
            continue
        sub = H[rows][:, idx][:, :, idx]
        P = psd_project(sub)
        blk = out[rows]
        blk[:, idx.unsqueeze(1), idx.unsqueeze(0)] = P
        out[rows] = blk
    return out


def _mask12(free):
    """(n, 4) vertex mask -> (n, 12) DoF mask."""
    return free.repeat_interleave(3, dim=1)


def snh_local(xt, dm_inv, mu, lam, vol, h, free, proj=F_SPACE, hess=PROJECTED):
    """Neo-Hookean tets.  xt (n, 4, 3), dm_inv (n, 3, 3), mu/lam/vol (n,),
    free (n, 4) bool.  Returns h^2 Psi (n,), h^2 dPsi/dx (n, 4, 3) with fixed
    vertices zeroed, and the 12x12 local Hessian over the free vertices:

    * F_SPACE: h^2 J_F^T Proj(d2Psi/dF2) J_F, the reduced-coordinate projection
      of the section "Eigendecomposition: Manual Optimization" (valid because
      F is linear in x);
    * X_SPACE: Proj(h^2 d2Psi/dx2) on the free principal submatrix;
    * hess=EXACT: the unprojected h^2 d2Psi/dx2.
    """
    n = xt.shape[0]
    h2 = h * h
    E = h2 * vmap(en.snh_tet_energy)(xt, dm_inv, mu, lam, vol)
    g = h2 * vmap(grad(en.snh_tet_energy))(xt, dm_inv, mu, lam, vol)
    g = g * free.unsqueeze(-1)
    m12 = _mask12(free)
    mm = (m12.unsqueeze(2) & m12.unsqueeze(1)).to(xt.dtype)
    if hess == EXACT or proj == X_SPACE:
        Hx = h2 * vmap(hessian(en.snh_tet_energy))(xt, dm_inv, mu, lam, vol).reshape(n, 12, 12)
        if hess == EXACT:
            return E, g, sym(Hx * mm)
        return E, g, sym(project_principal(Hx, m12))
    F = vmap(en.deformation_gradient)(xt, dm_inv)
    HF = vmap(hessian(en.snh_psi))(F, mu, lam, vol).reshape(n, 9, 9)
    JF = vmap(jacrev(en.deformation_gradient))(xt, dm_inv).reshape(n, 9, 12)
    H = h2 * (JF.transpose(1, 2) @ psd_project(HF) @ JF)
    return E, g, sym(H * mm)


def membrane_local(xf, dm_inv2, area, thickness, mu, lam, h, free, hess=PROJECTED):
    """StVK membrane triangles.  xf (n, 3, 3), dm_inv2 (n, 2, 2), area (n,).
    Energy h^2 Psi, gradient, and h^2 J_F^T Proj(d2Psi/dF2) J_F (6x6 F-space
    projection) over the free vertices, padded to (n, 12, 12) / (n, 4, 3)."""
    n = xf.shape[0]
    h2 = h * h
    t = torch.full((n,), float(thickness))
    m = torch.full((n,), float(mu))
    l = torch.full((n,), float(lam))

    def psi_x(x, D, A, tt, mm, ll):
        return en.stvk_membrane(x, D, A, tt, mm, ll)

    def psi_F(F, A, tt, mm, ll):
        G = 0.5 * (F.T @ F - torch.eye(2, dtype=F.dtype))
        return A * tt * (mm * (G * G).sum() + 0.5 * ll * torch.trace(G) ** 2)

    E = h2 * vmap(psi_x)(xf, dm_inv2, area, t, m, l)
    g3 = h2 * vmap(grad(psi_x))(xf, dm_inv2, area, t, m, l) * free[:, :3].unsqueeze(-1)
    m9 = free[:, :3].repeat_interleave(3, dim=1)
    mm9 = (m9.unsqueeze(2) & m9.unsqueeze(1)).to(xf.dtype)
    if hess == EXACT:
        H9 = h2 * vmap(hessian(psi_x))(xf, dm_inv2, area, t, m, l).reshape(n, 9, 9) * mm9
    else:
        F = vmap(en.membrane_deformation)(xf, dm_inv2)
        HF = vmap(hessian(psi_F))(F, area, t, m, l).reshape(n, 6, 6)
        JF = vmap(jacrev(en.membrane_deformation))(xf, dm_inv2).reshape(n, 6, 9)
        H9 = h2 * (JF.transpose(1, 2) @ psd_project(HF) @ JF) * mm9
    g = torch.zeros(n, 4, 3)
    g[:, :3] = g3
    H = torch.zeros(n, 12, 12)
    H[:, :9, :9] = sym(H9)
    return E, g, H


def hinge_local(xh, theta_bar, stiffness, h, free, hess=PROJECTED):
    """Dihedral bending hinges.  xh (n, 4, 3); energy h^2 E_b, gradient, and the
    free principal submatrix of h^2 d2E_b/dx2, projected unless hess=EXACT."""
    n = xh.shape[0]
    h2 = h * h
    E = h2 * vmap(en.hinge_energy)(xh, theta_bar, stiffness)
    g = h2 * vmap(grad(en.hinge_energy))(xh, theta_bar, stiffness) * free.unsqueeze(-1)
    H = h2 * vmap(hessian(en.hinge_energy))(xh, theta_bar, stiffness).reshape(n, 12, 12)
    m12 = _mask12(free)
    if hess == EXACT:
        return E, g, sym(H * (m12.unsqueeze(2) & m12.unsqueeze(1)).to(xh.dtype))
    return E, g, sym(project_principal(H, m12))


def contact_local(xc, ctype, free, kappa, dhat, hess=PROJECTED, classic=False, eps=None):
    """Barrier stencils.  xc (n, 4, 3) vertex rows (unused rows arbitrary finite),
    ctype (n,), free (n, 4) bool (False for fixed and unused vertices).

    Returns kappa b(d) (n,), its gradient (n, 4, 3) (fixed vertices zeroed), the
    free-DoF Hessian (n, 12, 12) projected on its free principal submatrix (the
    Hessian with fixed vertices held constant), and d (n,).  Stencils with
    d >= dhat contribute exactly zero; d <= 0 raises ValueError.  eps (n,) or
    None: edge-edge mollifier thresholds; an EE stencil's energy is then
    m(c) kappa b(d) (``energy.ee_mollifier``)."""
    n = xc.shape[0]
    E = torch.zeros(n)
    g = torch.zeros(n, 4, 3)
    H = torch.zeros(n, 12, 12)
    d = torch.zeros(n)
    bfun = en.barrier_ipc_classic if classic else en.barrier
    for t in range(4):
        sel = torch.nonzero(ctype == t).flatten()
        if sel.numel() == 0:
            continue
        x = xc[sel]
        dist = en.DIST[t]
        dt = vmap(dist)(x)
        if bool((dt <= 0).any()):
            raise ValueError("contact stencil with non-positive distance")

        act = (dt < dhat).to(x.dtype)
        d[sel] = dt
        if t == 1 and eps is not None:
            def f(xs, e, dist=dist):
                return en.ee_mollifier(en.ee_cross_norm(xs), e) * bfun(dist(xs), dhat, kappa)

            es = torch.as_tensor(eps, dtype=x.dtype)[sel]
            E[sel] = vmap(f)(x, es) * act
            g[sel] = vmap(grad(f))(x, es) * act.view(-1, 1, 1)
            H[sel] = vmap(hessian(f))(x, es).reshape(-1, 12, 12) * act.view(-1, 1, 1)
        else:
            def f(xs, dist=dist):
                return bfun(dist(xs), dhat, kappa)

            E[sel] = vmap(f)(x) * act
            g[sel] = vmap(grad(f))(x) * act.view(-1, 1, 1)
            H[sel] = vmap(hessian(f))(x).reshape(-1, 12, 12) * act.view(-1, 1, 1)
    g = g * free.unsqueeze(-1)
    m12 = _mask12(free)
    if hess == EXACT:
        mm = (m12.unsqueeze(2) & m12.unsqueeze(1)).to(xc.dtype)
        return E, g, sym(H * mm), d
    return E, g, sym(project_principal(H, m12)), d


def gather_positions(x_free, x_fixed, idx, n_free):
    """Rows of the stencil's vertices: ids < n_free are free, ids >= n_free are
    fixed vertex id - n_free, -1 is unused (returned as zeros).  Returns
    (positions (n, 4, 3), free mask (n, 4))."""
    idx = torch.as_tensor(idx, dtype=torch.int64)
    xall = torch.cat([x_free, x_fixed], 0)
    safe = idx.clamp(min=0)
    pos = xall[safe] * (idx >= 0).unsqueeze(-1)
    free = (idx >= 0) & (idx < n_free)
    return pos, free
