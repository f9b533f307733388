"""Pins for the PSD projection Proj(A) = Q max(Lambda, 0) Q^T (section
"Eigendecomposition (EVD) and PSD Projection"): PSD output, idempotence,
identity on PSD input, the nearest-PSD property in the Frobenius norm, and
||Proj(A) - A||_F = ||Lambda_-||_2 checked through the trace identity."""
import numpy as np
import torch

from oracle.local import project_principal, psd_project

torch.set_default_dtype(torch.float64)


def rand_sym(n, m, seed):
    g = torch.Generator().manual_seed(seed)
    A = torch.randn(n, m, m, generator=g)
    return 0.5 * (A + A.transpose(1, 2))


def test_psd_idempotent_identity_on_psd():
    for m in (2, 6, 9, 12):
        A = rand_sym(50, m, m)
        P = psd_project(A)
        # PSD: Cholesky of P + tiny shift succeeds
        torch.linalg.cholesky(P + 1e-12 * torch.eye(m))
        assert torch.allclose(psd_project(P), P, atol=1e-12)
        B = A @ A.transpose(1, 2)
        assert torch.allclose(psd_project(B), B, atol=1e-12 * float(B.abs().max()))


def test_nearest_psd_and_negative_part_norm():
    A = rand_sym(40, 9, 1)
    P = psd_project(A)
    g = torch.Generator().manual_seed(2)
    for _ in range(20):
        C = torch.randn(40, 9, 9, generator=g)
        B = P + 0.1 * C @ C.transpose(1, 2)  # another PSD matrix
        assert bool(((A - P).norm(dim=(1, 2)) <= (A - B).norm(dim=(1, 2)) + 1e-12).all())
    # ||P - A||_F^2 = sum of squared negative eigenvalues = (||A||_F^2 - ||P||_F^2)
    # since P - A and P are orthogonal in the trace inner product (P (P - A) = 0)
    lhs = (P - A).norm(dim=(1, 2)) ** 2
    rhs = A.norm(dim=(1, 2)) ** 2 - P.norm(dim=(1, 2)) ** 2
    assert torch.allclose(lhs, rhs, rtol=1e-10, atol=1e-12)
    assert float((P @ (P - A)).abs().max()) < 1e-10


def test_principal_projection_embeds_with_zeros():
    A = rand_sym(8, 12, 3)
    mask = torch.zeros(8, 12, dtype=torch.bool)
    mask[:, 3:] = True
    mask[4:, 3:6] = False
    P = project_principal(A, mask)
    for i in range(8):
        idx = torch.nonzero(mask[i]).flatten()
        sub = A[i][idx][:, idx]
        assert torch.allclose(P[i][idx][:, idx], psd_project(sub[None])[0])
        assert float(P[i][~mask[i]].abs().max()) == 0.0
