"""The GPU kernels' closed-form Neo-Hookean F-space projection (snh_math.h,
compiled for the host) against the oracle's eigh-based projection of the
autodiff Hessian, over stretched, compressed, inverted, degenerate and random
deformation gradients; and the SVD it rests on."""
import ctypes as C

import numpy as np
import pytest
import torch
from torch.func import hessian

import native_build
from oracle import energy as en
from oracle.local import psd_project

torch.set_default_dtype(torch.float64)
MU, LAM = 35714.28571428571, 142857.14285714287


@pytest.fixture(scope="module")
def L():
    lib = native_build.load("snh_host")
    lib.snh_proj_host.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double] + [C.c_void_p] * 4
    lib.snh_proj_host_f32.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_void_p]
    return lib


def rot(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def cases():
    rng = np.random.default_rng(7)
    out = [np.eye(3), 1.3 * np.eye(3), 0.6 * np.eye(3), np.diag([1.2, 1.2, 0.8]), np.diag([1.0, 1.0, -0.3]),
           np.diag([1e-9, 1.0, 1.0]), 1e-6 * np.eye(3)]
    for _ in range(60):
        s = rng.uniform(0.5, 1.6, 3)
        if rng.random() < 0.2:
            s[2] *= -1  # inverted
        if rng.random() < 0.2:
            s[1] = s[0] * (1 + 1e-10 * rng.standard_normal())  # near-degenerate
        out.append(rot(rng) @ np.diag(s) @ rot(rng).T)
    out.append(rng.standard_normal((3, 3)))
    return out


def oracle_proj(F, vol=0.7):
    H = hessian(en.snh_psi)(torch.tensor(F), torch.tensor(MU), torch.tensor(LAM), torch.tensor(vol)).reshape(9, 9)
    P = psd_project(H[None])[0].numpy()
    # oracle vec is row-major (3i + j); the kernels' is column-major (i + 3j)
    perm = np.array([3 * (k % 3) + k // 3 for k in range(9)])
    return P[np.ix_(perm, perm)], H.numpy()[np.ix_(perm, perm)]


def test_closed_form_projection_matches_oracle(L):
    for F in cases():
        P_ref, H = oracle_proj(F)
        P = np.zeros(81)
        U, s, V = np.zeros(9), np.zeros(3), np.zeros(9)
        Fc = np.ascontiguousarray(F, np.float64)
        L.snh_proj_host(Fc.ctypes.data, MU, LAM, 0.7, P.ctypes.data, U.ctypes.data, s.ctypes.data, V.ctypes.data)
        P = P.reshape(9, 9)
        scale = np.abs(H).max()
        assert np.abs(P - P_ref).max() <= 1e-10 * scale, (F, np.abs(P - P_ref).max(), scale)
        U, V = U.reshape(3, 3), V.reshape(3, 3)
        if True:
            assert np.allclose(U @ np.diag(s) @ V.T, F, atol=1e-12 * np.abs(F).max())
            assert np.allclose(U @ U.T, np.eye(3), atol=1e-12) and np.allclose(V @ V.T, np.eye(3), atol=1e-12)
            assert np.linalg.det(U) > 0 and np.linalg.det(V) > 0


def test_float32_closed_form_projection(L):
    for F in cases()[7:]:
        P_ref, H = oracle_proj(F)
        P = np.zeros(81)
        Fc = np.ascontiguousarray(F, np.float64)
        L.snh_proj_host_f32(Fc.ctypes.data, MU, LAM, 0.7, P.ctypes.data)
        assert np.abs(P.reshape(9, 9) - P_ref).max() <= 2e-5 * np.abs(H).max()
