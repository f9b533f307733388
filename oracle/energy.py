"""Energy definitions of the Newton-iteration objective (float64, PyTorch CPU).

Each function maps the positions of one stencil to a scalar, written exactly as
the definition reads; derivatives are taken elsewhere by autograd.  The
functions are vmapped over stencils by ``local.py``.

    E(x) = 1/2 ||x - x_tilde||_M^2 + h^2 sum_t Psi_t(x) + sum_s kappa b(d_s(x))
"""
from __future__ import annotations

import torch

# ---------------------------------------------------------------- elasticity


def deformation_gradient(xt, dm_inv):
    """F = Ds Dm^-1 with Ds = [x1-x0, x2-x0, x3-x0] (columns); xt is (4, 3)."""
    Ds = torch.stack([xt[1] - xt[0], xt[2] - xt[0], xt[3] - xt[0]], dim=1)
    return Ds @ dm_inv


def det3(F):
    """det F as the triple product of its columns, f0 . (f1 x f2).  (Written out
    because batched second derivatives through torch.linalg.det are unreliable.)"""
    return torch.dot(F[:, 0], torch.linalg.cross(F[:, 1], F[:, 2]))


def snh_density(F, mu, lam):
    """Stable Neo-Hookean energy density, Eq. (snh) in the section
    "Eigendecomposition: Manual Optimization":

        mu/2 (I_C - 3) - mu/2 log(I_C + 1) + lam/2 (J - (1 + 3 mu / (4 lam)))^2

    with I_C = tr(F^T F) and J = det F (the printed I_C/F_I definitions are
    garbled; this is the standard reading)."""
    Ic = (F * F).sum()
    J = det3(F)
    alpha = 1.0 + 3.0 * mu / (4.0 * lam)
    return 0.5 * mu * (Ic - 3.0) - 0.5 * mu * torch.log(Ic + 1.0) + 0.5 * lam * (J - alpha) ** 2


def snh_psi(F, mu, lam, vol):
    """Psi = V [density(F) - density(I)]: the rest value is subtracted so the
    energy is zero at rest (derivatives are unchanged by the constant)."""
    eye = torch.eye(3, dtype=F.dtype)
    return vol * (snh_density(F, mu, lam) - snh_density(eye, mu, lam))


def snh_tet_energy(xt, dm_inv, mu, lam, vol):
    """Psi_t as a function of the tet's 4 vertex positions."""
    return snh_psi(deformation_gradient(xt, dm_inv), mu, lam, vol)


# ---------------------------------------------------------------- barrier


def barrier(d, dhat, kappa):
    """kappa (d - dhat)^2 log(d / dhat)^2 with d a squared distance: the point-point
    barrier of the "Energies" code listing and of the section "Eigendecomposition:
    Automatic Optimization", applied here to every stencil type.  Only called for
    0 < d < dhat; for d >= dhat the stencil contributes exactly zero."""
    return kappa * (d - dhat) ** 2 * torch.log(d / dhat) ** 2


def barrier_ipc_classic(d, dhat, kappa):
    """The classic IPC barrier -kappa (d - dhat)^2 log(d / dhat) (alternative reading)."""
    return -kappa * (d - dhat) ** 2 * torch.log(d / dhat)


# ---------------------------------------------------------------- distances
# Squared distances of a stencil given its 4 vertex rows x (4, 3).  The stencil
# type fixes the formula (the generator assigns the type from the closest-feature
# region); unused trailing rows are ignored.


def _cross(a, b):
    return torch.linalg.cross(a, b)


def dist_pt(x):
    """Point-triangle (interior type): squared distance from p to the plane of
    (t0, t1, t2).  x = [p, t0, t1, t2]."""
    p, t0, t1, t2 = x[0], x[1], x[2], x[3]
    n = _cross(t1 - t0, t2 - t0)
    return torch.dot(p - t0, n) ** 2 / torch.dot(n, n)


def dist_ee(x):
    """Edge-edge (interior type): squared distance between the lines through
    (a0, a1) and (b0, b1).  x = [a0, a1, b0, b1]."""
    a0, a1, b0, b1 = x[0], x[1], x[2], x[3]
    n = _cross(a1 - a0, b1 - b0)
    return torch.dot(a0 - b0, n) ** 2 / torch.dot(n, n)


def dist_pe(x):
    """Point-edge (interior type): squared distance from p to the line (e0, e1).
    x = [p, e0, e1, unused]."""
    p, e0, e1 = x[0], x[1], x[2]
    c = _cross(e0 - p, e1 - p)
    e = e1 - e0
    return torch.dot(c, c) / torch.dot(e, e)


def dist_pp(x):
    """Point-point: ||p - q||^2.  x = [p, q, unused, unused]."""
    d = x[1] - x[0]
    return torch.dot(d, d)


def ee_cross_norm(x):
    """c = ||(a1 - a0) x (b1 - b0)||^2 of an edge-edge stencil x = [a0, a1, b0, b1]
    (zero for parallel edges)."""
    n = _cross(x[1] - x[0], x[3] - x[2])
    return torch.dot(n, n)


def ee_mollifier(c, eps):
    """The edge-edge mollifier of Incremental Potential Contact (Li et al.
    2020): m(c) = -c^2 / eps^2 + 2 c / eps for c < eps, else 1, with the
    threshold eps = 1e-3 ||a1 - a0||^2 ||b1 - b0||^2 taken at rest.  eps <= 0
    means no mollifier (m = 1)."""
    on = (eps > 0) & (c < eps)
    e = torch.where(eps > 0, eps, torch.ones_like(eps))
    return torch.where(on, -(c * c) / (e * e) + 2.0 * c / e, torch.ones_like(c))


DIST = (dist_pt, dist_ee, dist_pe, dist_pp)
N_VERTS = (4, 4, 3, 2)


def signed_side(x, ctype):
    """Sign-carrying quantity used by the line search for PT and EE stencils:
    (p - t0) . n (PT) or (a0 - b0) . n (EE).  x is (n, 4, 3), ctype (n,)."""
    p, q1, q2, q3 = x[:, 0], x[:, 1], x[:, 2], x[:, 3]
    n_pt = torch.linalg.cross(q2 - q1, q3 - q1, dim=1)
    s_pt = ((p - q1) * n_pt).sum(1)
    n_ee = torch.linalg.cross(q1 - p, q3 - q2, dim=1)
    s_ee = ((p - q2) * n_ee).sum(1)
    return torch.where(ctype == 0, s_pt, torch.where(ctype == 1, s_ee, torch.ones_like(s_pt)))


# ---------------------------------------------------------------- cloth


def membrane_deformation(xf, dm_inv2):
    """3x2 deformation gradient [x1 - x0, x2 - x0] Dm^-1 of a triangle (rest shape
    Dm in a 2-D orthonormal frame of the rest triangle)."""
    Ds = torch.stack([xf[1] - xf[0], xf[2] - xf[0]], dim=1)
    return Ds @ dm_inv2


def stvk_membrane(xf, dm_inv2, area, thickness, mu, lam):
    """StVK membrane: A t [mu tr(G^2) + lam/2 (tr G)^2] with G = (F^T F - I) / 2."""
    F = membrane_deformation(xf, dm_inv2)
    G = 0.5 * (F.T @ F - torch.eye(2, dtype=F.dtype))
    return area * thickness * (mu * (G * G).sum() + 0.5 * lam * torch.trace(G) ** 2)


def hinge_angle(x):
    """Dihedral angle of the hinge (x0, x1 shared edge; x2, x3 the opposite
    vertices of the two triangles): atan2((n1 x n2) . e_hat, n1 . n2) with the
    unnormalised normals n1 = (x1 - x0) x (x2 - x0), n2 = (x3 - x0) x (x1 - x0)
    (both triangles oriented consistently; zero for a flat hinge)."""
    e = x[1] - x[0]
    n1 = torch.linalg.cross(e, x[2] - x[0])
    n2 = torch.linalg.cross(x[3] - x[0], e)
    return torch.atan2(torch.dot(torch.linalg.cross(n1, n2), e) / torch.sqrt(torch.dot(e, e)), torch.dot(n1, n2))


def hinge_energy(x, theta_bar, stiffness):
    """Discrete-shells bending k_b 3|e_bar|^2/(A1 + A2) (theta - theta_bar)^2;
    `stiffness` is the precomputed rest factor k_b 3|e_bar|^2/(A1 + A2)."""
    return stiffness * (hinge_angle(x) - theta_bar) ** 2
