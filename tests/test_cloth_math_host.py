"""The GPU kernels' per-stencil cloth arithmetic (cloth_math.h, compiled for
the host by hipcc) against the oracle, on the CPU: StVK membranes under
stretch and compression with fixed vertices, and hinges at every number of
free vertices, projected and exact Hessians."""
import ctypes as C
import itertools

import numpy as np
import pytest
import torch

import native_build
from oracle import assemble, local

torch.set_default_dtype(torch.float64)
MU, LAM, THICK, H2 = 3.8e4, 3.3e4, 1e-3, 1e-4


@pytest.fixture(scope="module")
def harness():
    L = native_build.load("cloth_host")
    L.hinge_host.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.membrane_host.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    return L


def membrane_cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        P = rng.uniform(-1, 1, (3, 2)) * 0.004
        D = np.stack([P[1] - P[0], P[2] - P[0]], 1)
        if np.linalg.det(D) < 0:
            P[[1, 2]] = P[[2, 1]]
            D = np.stack([P[1] - P[0], P[2] - P[0]], 1)
        s = [0.6, 0.95, 1.0, 1.3][k % 4]
        x = np.concatenate([P * s, np.zeros((3, 1))], 1) + 2e-4 * rng.standard_normal((3, 3))
        out.append((x, np.linalg.inv(D), 0.5 * abs(np.linalg.det(D))))
    return out


@pytest.mark.parametrize("exact", [False, True])
def test_membrane_math_matches_oracle(harness, exact):
    hess = assemble.EXACT if exact else assemble.PROJECTED
    for (x, Dinv, A), free in itertools.product(membrane_cases(3, 8), [(1, 1, 1), (1, 0, 1), (0, 1, 0)]):
        fr = np.array(free, np.int32)
        e = C.c_double()
        g = np.zeros(9)
        H = np.zeros(81)
        xs = np.ascontiguousarray(x)
        Ds = np.ascontiguousarray(Dinv)
        assert harness.membrane_host(int(exact), xs.ctypes.data, Ds.ctypes.data, A, THICK, MU, LAM, H2,
                                     fr.ctypes.data, C.byref(e), g.ctypes.data, H.ctypes.data) == 0
        m4 = torch.tensor(list(free) + [0], dtype=torch.bool)[None]
        Eo, go, Ho = local.membrane_local(torch.tensor(x)[None], torch.tensor(Dinv)[None], torch.tensor([A]),
                                          THICK, MU, LAM, np.sqrt(H2), m4, hess)
        Ho = Ho[0, :9, :9].numpy()
        scale = np.abs(Ho).max() + 1e-300
        assert abs(e.value - float(Eo[0])) <= 1e-12 * abs(float(Eo[0])) + 1e-30
        assert np.abs(g - go[0, :3].numpy().ravel()).max() <= 1e-10 * (np.abs(g).max() + 1e-300)
        assert np.abs(H.reshape(9, 9) - Ho).max() <= 1e-10 * scale


def hinge_cases(seed, n):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        phi = rng.uniform(-2.5, 2.5)
        x = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.4, 0.9, 0], [0.6, -np.cos(phi), -np.sin(phi)]]) * 0.004
        x = x + 3e-4 * rng.standard_normal((4, 3))
        out.append((x, rng.uniform(-0.3, 0.3), rng.uniform(0.01, 0.2)))
    return out


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("nfree", [1, 2, 3, 4])
def test_hinge_math_matches_oracle(harness, exact, nfree):
    hess = assemble.EXACT if exact else assemble.PROJECTED
    for (x, tb, k), fl in itertools.product(hinge_cases(10 + nfree, 6),
                                            [c for c in itertools.combinations(range(4), nfree)][:3]):
        fl4 = np.array(list(fl) + [0] * (4 - nfree), np.int32)
        e, th = C.c_double(), C.c_double()
        g = np.zeros(12)
        H = np.zeros(144)
        xs = np.ascontiguousarray(x)
        assert harness.hinge_host(nfree, int(exact), xs.ctypes.data, fl4.ctypes.data, tb, k, H2, C.byref(e),
                                  C.byref(th), g.ctypes.data, H.ctypes.data) == 0
        free = torch.zeros(1, 4, dtype=torch.bool)
        free[0, list(fl)] = True
        Eo, go, Ho = local.hinge_local(torch.tensor(x)[None], torch.tensor([tb]), torch.tensor([k]), np.sqrt(H2),
                                       free, hess)
        Ho = Ho[0].numpy()
        scale = np.abs(Ho).max() + 1e-300
        assert abs(e.value - float(Eo[0])) <= 1e-12 * abs(float(Eo[0])) + 1e-300
        assert np.abs(g - go[0].numpy().ravel()).max() <= 1e-10 * (np.abs(go.numpy()).max() + 1e-300)
        assert np.abs(H.reshape(12, 12) - Ho).max() <= 1e-9 * scale, (nfree, fl, exact)
