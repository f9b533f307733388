"""The GPU kernels' per-stencil contact arithmetic (contact_math.h, compiled
for the host by hipcc) against the oracle, on the CPU: every type, every number
of free vertices, projected and exact Hessians."""
import ctypes as C
import itertools

import numpy as np
import pytest
import torch

import native_build
from oracle import energy as en
from oracle import local

torch.set_default_dtype(torch.float64)
KAPPA, DHAT = 1e4, 1e-3
NV = (4, 4, 3, 2)


@pytest.fixture(scope="module")
def harness():
    L = native_build.load("contact_host")
    L.contact_host.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_double, C.c_double,
                               C.c_int, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.contact_host.restype = C.c_int
    return L


def stencils(t, n, seed):
    rng = np.random.default_rng(seed)
    if t == 0:
        base = np.array([[0.3, 0.3, 0.4], [0, 0, 0], [1, 0, 0], [0, 1, 0]]) * 0.05
    elif t == 1:
        base = np.array([[0.0, 0.5, 0.0], [1.0, 0.5, 0.0], [0.5, 0.0, 0.4], [0.5, 1.0, 0.4]]) * 0.05
    elif t == 2:
        base = np.array([[0.5, 0.3, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0, 0, 0]]) * 0.05
    else:
        base = np.array([[0.0, 0.0, 0.0], [0.015, 0.01, 0.0], [0, 0, 0], [0, 0, 0]])
    x = base[None] + 0.002 * rng.standard_normal((n, 4, 3))
    x[:, NV[t]:] = 0.0
    return x


def run_host(L, t, K, exact, x, fl, classic=0, eps=0.0):
    e, d = C.c_double(), C.c_double()
    g = np.zeros(12)
    H = np.zeros(144)
    xs = np.ascontiguousarray(x, np.float64)
    f = np.ascontiguousarray(fl, np.int32)
    rc = L.contact_host(t, K, int(exact), xs.ctypes.data, f.ctypes.data, KAPPA, DHAT, classic, eps, C.byref(e),
                        C.byref(d), g.ctypes.data, H.ctypes.data)
    assert rc == 0
    return e.value, d.value, g.reshape(4, 3), H.reshape(12, 12)


@pytest.mark.parametrize("t", [0, 1, 2, 3])
@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("classic", [0, 1])
def test_contact_math_matches_oracle(harness, t, exact, classic):
    n = 6
    x = stencils(t, n, 100 + t)
    for K in range(1, NV[t] + 1):
        for freeset in itertools.combinations(range(NV[t]), K):
            fl = list(freeset) + [0] * (4 - K)
            free = torch.zeros(n, 4, dtype=torch.bool)
            free[:, list(freeset)] = True
            Eo, go, Ho, do = local.contact_local(torch.tensor(x), torch.full((n,), t), free, KAPPA, DHAT,
                                                 local.EXACT if exact else local.PROJECTED,
                                                 classic=bool(classic))
            for s in range(n):
                e, d, g, H = run_host(harness, t, K, exact, x[s], fl, classic)
                sc = np.abs(Ho[s].numpy()).max() + 1e-300
                assert abs(d - float(do[s])) <= 1e-12 * float(do[s])
                assert abs(e - float(Eo[s])) <= 1e-10 * abs(float(Eo[s])) + 1e-300
                assert np.abs(g - go[s].numpy()).max() <= 1e-10 * np.abs(go[s].numpy()).max()
                err = np.abs(H - Ho[s].numpy()).max()
                assert err <= 1e-10 * sc, (t, K, freeset, exact, s, err, sc)


@pytest.mark.parametrize("t", [0, 1, 2, 3])
@pytest.mark.parametrize("classic", [0, 1])
def test_contact_math_inactive_beyond_dhat(harness, t, classic):
    """Stencils at d >= dhat (the stencils above scaled by 3, and one placed
    exactly at dhat): energy, gradient and Hessian exactly zero for every free
    set, projected or not, and the distance still reported (the stencil keeps
    its slots; its staged blocks are zeros)."""
    n = 6
    x = 3.0 * stencils(t, n, 200 + t)
    xs = [x[s] for s in range(n)]
    if t == 3:  # at the cutoff: the smallest separation whose square rounds to >= dhat
        s = np.sqrt(DHAT)
        while s * s < DHAT:
            s = np.nextafter(s, np.inf)
        xe = np.zeros((4, 3))
        xe[1, 0] = s
        xs.append(xe)
    for xv in xs:
        for K in range(1, NV[t] + 1):
            for freeset in itertools.combinations(range(NV[t]), K):
                fl = list(freeset) + [0] * (4 - K)
                for exact in (False, True):
                    e, d, g, H = run_host(harness, t, K, exact, xv, fl, classic)
                    d_o = float(en.DIST[t](torch.tensor(xv)))
                    assert d >= DHAT and abs(d - d_o) <= 1e-12 * d_o
                    assert e == 0.0 and not g.any() and not H.any(), (t, K, freeset, exact, d)


@pytest.mark.parametrize("exact", [False, True])
@pytest.mark.parametrize("classic", [0, 1])
def test_ee_mollifier_matches_oracle(harness, exact, classic):
    """Near-parallel edge-edge stencils under the mollifier (eps_x above c for
    most of them, below for some): every free set against the oracle's m(c) b(d)."""
    n = 8
    rng = np.random.default_rng(300 + classic)
    la, lb = 0.05, 0.05
    x = np.zeros((n, 4, 3))
    th = rng.uniform(0.004, 0.05, size=n)
    for s in range(n):
        x[s, 0] = [-la / 2, 0.0, 0.0]
        x[s, 1] = [la / 2, 0.0, 0.0]
        u = np.array([np.cos(th[s]), np.sin(th[s]), 0.0])
        c0 = np.array([0.0, 0.0, -0.02])
        x[s, 2] = c0 - lb / 2 * u
        x[s, 3] = c0 + lb / 2 * u
    x += 1e-4 * rng.standard_normal(x.shape)
    eps = np.full(n, 1e-3 * la ** 2 * lb ** 2)
    c = np.array([float(en.ee_cross_norm(torch.tensor(x[s]))) for s in range(n)])
    assert (c < eps).sum() >= 3 and (c >= eps).sum() >= 1
    for K in range(1, 5):
        for freeset in itertools.combinations(range(4), K):
            fl = list(freeset) + [0] * (4 - K)
            free = torch.zeros(n, 4, dtype=torch.bool)
            free[:, list(freeset)] = True
            Eo, go, Ho, do = local.contact_local(torch.tensor(x), torch.full((n,), 1), free, KAPPA, DHAT,
                                                 local.EXACT if exact else local.PROJECTED,
                                                 classic=bool(classic), eps=eps)
            for s in range(n):
                e, d, g, H = run_host(harness, 1, K, exact, x[s], fl, classic, eps[s])
                sc = np.abs(Ho[s].numpy()).max() + 1e-300
                assert abs(e - float(Eo[s])) <= 1e-10 * abs(float(Eo[s])) + 1e-300, (K, freeset, s)
                assert np.abs(g - go[s].numpy()).max() <= 1e-10 * np.abs(go[s].numpy()).max()
                err = np.abs(H - Ho[s].numpy()).max()
                assert err <= 1e-10 * sc, (K, freeset, exact, s, err, sc)


def random_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def oriented_stencils(t, n, seed):
    """Stencils of type t in random orientations and shapes, all active
    (0 < d < dhat): triangles, edges and points placed at a random distance
    below sqrt(dhat) from the other primitive, then rotated and translated."""
    rng = np.random.default_rng(seed)
    h_max = np.sqrt(DHAT)
    x = np.zeros((n, 4, 3))
    for s in range(n):
        h = rng.uniform(0.15, 0.95) * h_max
        L = rng.uniform(0.02, 0.2)
        if t == 0:  # triangle in z = 0, point above an arbitrary spot of its plane
            tri = np.c_[L * rng.uniform(-1, 1, (3, 2)), np.zeros(3)]
            p = np.r_[L * rng.uniform(-1.2, 1.2, 2), h * rng.choice([-1, 1])]
            pts = np.vstack([p, tri])
        elif t == 1:  # two edges in the planes z = 0 and z = h, at an angle
            th = rng.uniform(0.2, np.pi - 0.2)
            a0 = np.r_[L * rng.uniform(-1, 0), 0.0, 0.0]
            a1 = np.r_[L * rng.uniform(0.2, 1), 0.0, 0.0]
            u = np.array([np.cos(th), np.sin(th), 0.0])
            c = np.r_[L * rng.uniform(-0.5, 0.5, 2), h]
            b0 = c - L * rng.uniform(0.2, 1) * u
            b1 = c + L * rng.uniform(0.2, 1) * u
            pts = np.vstack([a0, a1, b0, b1])
        else:  # edge along x, point at distance h from its line
            e0 = np.r_[L * rng.uniform(-1, 0), 0.0, 0.0]
            e1 = np.r_[L * rng.uniform(0.2, 1), 0.0, 0.0]
            ph = rng.uniform(0, 2 * np.pi)
            p = np.r_[L * rng.uniform(-1.5, 1.5), h * np.cos(ph), h * np.sin(ph)]
            pts = np.vstack([p, e0, e1, np.zeros(3)])
        R = random_rotation(rng)
        off = rng.uniform(-1, 1, 3)
        x[s, :NV[t]] = pts[:NV[t]] @ R.T + off
    return x


@pytest.mark.parametrize("t", [0, 1, 2])
@pytest.mark.parametrize("classic", [0, 1])
def test_structured_projection_random_orientations(harness, t, classic):
    """The in-frame projections (plane split for point-triangle and edge-edge,
    line split for point-edge, closed forms for the 2 x 2 pieces) against the
    oracle's dense eigendecomposition of the free Hessian, on stencils in
    random orientations, shapes and distances, for every free set."""
    n = 24
    x = oriented_stencils(t, n, 400 + 10 * t + classic)
    for K in range(1, NV[t] + 1):
        for freeset in itertools.combinations(range(NV[t]), K):
            fl = list(freeset) + [0] * (4 - K)
            free = torch.zeros(n, 4, dtype=torch.bool)
            free[:, list(freeset)] = True
            Eo, go, Ho, do = local.contact_local(torch.tensor(x), torch.full((n,), t), free, KAPPA, DHAT,
                                                 local.PROJECTED, classic=bool(classic))
            assert (do > 0).all() and (do < DHAT).all()
            for s in range(n):
                e, d, g, H = run_host(harness, t, K, False, x[s], fl, classic)
                sc = np.abs(Ho[s].numpy()).max() + 1e-300
                err = np.abs(H - Ho[s].numpy()).max()
                assert err <= 1e-10 * sc, (t, K, freeset, s, err, sc)
                assert np.linalg.eigvalsh(H).min() >= -1e-12 * sc
