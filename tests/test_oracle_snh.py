"""Pins for the oracle's stable Neo-Hookean term (Eq. snh).

Each check is fixed by mathematics, not by re-running the oracle's own code:
closed-form values and spectra at rest and under uniform stretch, rotation
invariance, and central finite differences of energy -> gradient -> Hessian."""
import numpy as np
import pytest
import torch
from torch.func import grad, hessian, vmap

from oracle import energy as en
from oracle import local

torch.set_default_dtype(torch.float64)
MU, LAM = 35714.28571428571, 142857.14285714287


def rand_tets(n, seed, spread=0.25):
    g = torch.Generator().manual_seed(seed)
    X = torch.tensor([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]) * 0.3
    x = X.unsqueeze(0) + spread * 0.3 * torch.randn(n, 4, 3, generator=g)
    Ds = torch.stack([X[1] - X[0], X[2] - X[0], X[3] - X[0]], 1)
    dm = torch.linalg.inv(Ds).expand(n, 3, 3).clone()
    vol = torch.full((n,), float(torch.det(Ds)) / 6)
    return x, dm, vol


def test_rest_energy_and_gradient_are_zero():
    F = torch.eye(3)
    assert float(en.snh_psi(F, MU, LAM, 1.0)) == 0.0
    P = grad(en.snh_psi)(F, torch.tensor(MU), torch.tensor(LAM), torch.tensor(1.0))
    # alpha = 1 + 3mu/(4 lam) makes dPsi/dF(I) = mu(1 - 1/4) I + lam(1 - alpha) I = 0
    assert float(P.abs().max()) < 1e-9 * MU


def test_rest_spectrum_closed_form():
    # d2Psi/dF2(I) = 3mu/4 (I9 + T) + (lam - 5mu/8) vec(I) vec(I)^T with T the
    # transpose permutation: eigenvalues 0 (x3, skew), 3mu/2 (x5, symmetric
    # traceless), 3 lam - 3mu/8 (x1, trace direction).
    H = hessian(en.snh_psi)(torch.eye(3), torch.tensor(MU), torch.tensor(LAM), torch.tensor(1.0))
    w = np.sort(np.linalg.eigvalsh(H.reshape(9, 9).numpy()))
    ref = np.sort([0.0] * 3 + [1.5 * MU] * 5 + [3 * LAM - 3 * MU / 8])
    assert np.allclose(w, ref, rtol=1e-12, atol=1e-9 * LAM)


def test_x_space_rest_hessian_has_six_rigid_modes_and_projection_is_identity():
    x, dm, vol = rand_tets(1, 0, spread=0.0)
    free = torch.ones(1, 4, dtype=torch.bool)
    mu, lam = torch.full((1,), MU), torch.full((1,), LAM)
    _, g, Hp = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.PROJECTED)
    _, _, He = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.EXACT)
    w = np.linalg.eigvalsh(He[0].numpy())
    scale = np.abs(w).max()
    assert (np.abs(w) < 1e-10 * scale).sum() == 6
    assert (w > -1e-10 * scale).all()
    assert float((Hp - He).abs().max()) < 1e-10 * scale
    assert float(g.abs().max()) < 1e-10 * scale


def test_uniform_stretch_closed_form():
    alpha = 1 + 3 * MU / (4 * LAM)
    for s in (0.7, 0.93, 1.0, 1.25, 1.4):
        F = s * torch.eye(3)
        ref = (MU / 2 * (3 * s * s - 3) - MU / 2 * np.log(3 * s * s + 1) + LAM / 2 * (s ** 3 - alpha) ** 2) \
            - (-MU / 2 * np.log(4) + 9 * MU * MU / (32 * LAM))
        val = float(en.snh_psi(F, MU, LAM, 1.0))
        assert abs(val - ref) <= 1e-12 * (abs(ref) + MU)


def _rot(seed):
    g = torch.Generator().manual_seed(seed)
    q = torch.randn(4, generator=g)
    q = q / q.norm()
    w, x, y, z = q
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)]),
        torch.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)]),
        torch.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)])])


@pytest.mark.parametrize("proj", [local.F_SPACE, local.X_SPACE])
def test_rigid_rotation_equivariance(proj):
    n = 64
    x, dm, vol = rand_tets(n, 1)
    R = _rot(3)
    free = torch.ones(n, 4, dtype=torch.bool)
    mu, lam = torch.full((n,), MU), torch.full((n,), LAM)
    E0, g0, H0 = local.snh_local(x, dm, mu, lam, vol, 0.01, free, proj)
    E1, g1, H1 = local.snh_local(x @ R.T, dm, mu, lam, vol, 0.01, free, proj)
    RR = torch.block_diag(R, R, R, R)
    sc = H0.abs().amax((1, 2), keepdim=True)
    assert torch.allclose(E1, E0, rtol=1e-11, atol=1e-14)
    assert float(((g1.reshape(n, 12) - (RR @ g0.reshape(n, 12, 1)).squeeze(-1)).abs() / sc[:, 0]).max()) < 1e-11
    assert float(((H1 - RR @ H0 @ RR.T).abs() / sc).max()) < 1e-10


def test_finite_differences_gradient_and_hessian():
    n = 40
    x, dm, vol = rand_tets(n, 5)
    mu, lam = torch.full((n,), MU), torch.full((n,), LAM)
    free = torch.ones(n, 4, dtype=torch.bool)
    E, g, H = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.EXACT)
    eps = 1e-6 * 0.3
    gfd = torch.zeros(n, 12)
    Hfd = torch.zeros(n, 12, 12)
    for k in range(12):
        dx = torch.zeros(n, 12)
        dx[:, k] = eps
        Ep, gp, _ = local.snh_local(x + dx.view(n, 4, 3), dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.EXACT)
        Em, gm, _ = local.snh_local(x - dx.view(n, 4, 3), dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.EXACT)
        gfd[:, k] = (Ep - Em) / (2 * eps)
        Hfd[:, :, k] = (gp - gm).reshape(n, 12) / (2 * eps)
    gs = g.reshape(n, 12).abs().amax(1, keepdim=True)
    Hs = H.abs().amax((1, 2), keepdim=True)
    assert float(((gfd - g.reshape(n, 12)).abs() / gs).max()) < 1e-6
    assert float(((Hfd - H).abs() / Hs).max()) < 1e-6


def test_batched_matches_single():
    # guards against batching bugs in the autodiff stack
    n = 16
    x, dm, vol = rand_tets(n, 9)
    mu, lam = torch.full((n,), MU), torch.full((n,), LAM)
    free = torch.ones(n, 4, dtype=torch.bool)
    _, _, Hb = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE)
    for i in range(n):
        _, _, Hi = local.snh_local(x[i:i + 1], dm[i:i + 1], mu[i:i + 1], lam[i:i + 1], vol[i:i + 1],
                                   1.0, free[i:i + 1], local.F_SPACE)
        assert torch.allclose(Hi[0], Hb[i], rtol=1e-12, atol=1e-12 * float(Hb[i].abs().max()))


@pytest.mark.parametrize("proj", [local.F_SPACE, local.X_SPACE])
def test_projected_hessian_is_psd_and_fixed_rows_vanish(proj):
    n = 200
    x, dm, vol = rand_tets(n, 11, spread=0.4)
    mu, lam = torch.full((n,), MU), torch.full((n,), LAM)
    free = torch.ones(n, 4, dtype=torch.bool)
    free[::3, 0] = False
    _, g, H = local.snh_local(x, dm, mu, lam, vol, 0.01, free, proj)
    w = torch.linalg.eigvalsh(H)
    assert float((w.min(1).values / w.abs().max(1).values).min()) > -1e-12
    assert float(H[::3, :3, :].abs().max()) == 0.0 and float(g[::3, 0].abs().max()) == 0.0


def test_projection_only_adds_the_negative_part():
    # Proj(A) - A = Q max(-Lambda, 0) Q^T is PSD, and so is J^T (Proj(A) - A) J
    n = 100
    x, dm, vol = rand_tets(n, 4, spread=0.3)
    mu, lam = torch.full((n,), MU), torch.full((n,), LAM)
    free = torch.ones(n, 4, dtype=torch.bool)
    _, _, Hp = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE)
    _, _, He = local.snh_local(x, dm, mu, lam, vol, 1.0, free, local.F_SPACE, local.EXACT)
    w = np.linalg.eigvalsh((Hp - He).numpy())
    sc = np.abs(np.linalg.eigvalsh(He.numpy())).max(1)
    assert (w.min(1) / sc).min() > -1e-12
    assert (np.abs(w).max(1) > 1e-8 * sc).any()  # some tets really were indefinite
