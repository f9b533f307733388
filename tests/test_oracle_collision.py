"""Pins of the oracle's proximity search, additive CCD and time stepping.

Against independent constructions: closest points by brute force (the
triangle's plane projection, its three clamped edge projections and its
vertices; a dense parameter grid with local refinement for two segments), the
type-fixed stencil distances of the energy module, an exhaustive pair search
without the candidate boxes, the exact time of impact of a point falling onto
a triangle, sampled distances along random trajectories, and the closed-form
free fall of implicit Euler.
"""
import math

import numpy as np
import pytest
import torch

from oracle import collision as col
from oracle import energy as en
from oracle import timestep as ts
from paper_2605_23088_amd import synth


def brute_point_triangle(p, a, b, c):
    """Closest distance^2 and feature ('F', 'E', 'V') by explicit candidates."""
    p, a, b, c = (np.asarray(v, np.float64) for v in (p, a, b, c))
    cands = []
    n = np.cross(b - a, c - a)
    q = p - np.dot(p - a, n) / np.dot(n, n) * n
    # barycentric coordinates of the projection
    T = np.stack([b - a, c - a], 1)
    uv = np.linalg.lstsq(T, q - a, rcond=None)[0]
    if uv[0] > 0 and uv[1] > 0 and uv.sum() < 1:
        cands.append((np.sum((p - q) ** 2), "F"))
    for u, w in ((a, b), (a, c), (b, c)):
        t = np.dot(p - u, w - u) / np.dot(w - u, w - u)
        if 0 < t < 1:
            cands.append((np.sum((p - (u + t * (w - u))) ** 2), "E"))
    for v in (a, b, c):
        cands.append((np.sum((p - v) ** 2), "V"))
    return min(cands, key=lambda z: z[0])


def test_point_triangle_against_brute_force():
    rng = np.random.default_rng(1)
    kinds = set()
    for _ in range(400):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 1.5
        kind, loc, d2 = col.point_triangle(tuple(p), tuple(a), tuple(b), tuple(c))
        d2b, kb = brute_point_triangle(p, a, b, c)
        assert d2 == pytest.approx(d2b, rel=1e-10, abs=1e-14)
        assert kind == kb
        kinds.add(kind)
    assert kinds == {"F", "E", "V"}


def test_segment_segment_against_brute_force():
    from scipy.optimize import minimize
    rng = np.random.default_rng(2)
    kinds = set()
    for _ in range(200):
        p1, q1, p2, q2 = rng.normal(size=(4, 3))
        s, t, d2 = col.segment_segment(tuple(p1), tuple(q1), tuple(p2), tuple(q2))
        f = lambda z: np.sum((p1 + z[0] * (q1 - p1) - p2 - z[1] * (q2 - p2)) ** 2)
        g = np.linspace(0, 1, 41)
        S, T = np.meshgrid(g, g)
        vals = np.array([f((a, b)) for a, b in zip(S.ravel(), T.ravel())])
        k = int(np.argmin(vals))
        r = minimize(f, [S.ravel()[k], T.ravel()[k]], bounds=[(0, 1), (0, 1)], method="L-BFGS-B",
                     options=dict(ftol=1e-15, gtol=1e-12))
        assert d2 == pytest.approx(r.fun, rel=1e-7, abs=1e-12)
        assert d2 <= r.fun * (1 + 1e-9) + 1e-15
        kinds.add((0.0 < s < 1.0, 0.0 < t < 1.0))
    assert len(kinds) >= 3


def scene(**kw):
    p = synth.drop_scene(**kw)
    S = col.Surface(p["surf_points"], p["surf_edges"], p["surf_tris"], p["n_free"], p["surf_len2"])
    return p, S


def test_detect_types_distances_and_completeness():
    """Every stencil's type-fixed distance equals its pair's distance, and
    every pair closer than sqrt(dhat) is found (exhaustive search)."""
    p, S = scene(gap=0.004)
    st = ts.Stepper(p, S)
    xa = st.xall(p["x0"])
    ct, ci, eps = S.detect(xa, p["dhat"])
    assert len(ct) > 20 and set(ct.tolist()) >= {0, 1, 2}
    for t, ids in zip(ct, ci):
        xs = torch.zeros(4, 3)
        used = [int(v) for v in ids if v >= 0]
        xs[:len(used)] = torch.as_tensor(xa[used])
        d_type = float(en.DIST[int(t)](xs))
        assert d_type < p["dhat"] * (1 + 1e-9)
    # exhaustive: all pairs by primitive distance
    X = [tuple(r) for r in xa]
    n_pt = n_ee = 0
    for v in S.points:
        for tri in S.tris:
            if v in tri or (v >= S.n_free and (tri >= S.n_free).all()):
                continue
            n_pt += col.point_triangle(X[v], X[tri[0]], X[tri[1]], X[tri[2]])[2] < p["dhat"]
    E = S.edges
    for i in range(len(E)):
        for j in range(i + 1, len(E)):
            if E[i][0] in E[j] or E[i][1] in E[j] or ((E[i] >= S.n_free).all() and (E[j] >= S.n_free).all()):
                continue
            n_ee += col.segment_segment(X[E[i][0]], X[E[i][1]], X[E[j][0]], X[E[j][1]])[2] < p["dhat"]
    assert len(ct) == n_pt + n_ee
    # EE stencils carry the mollifier thresholds of their two edges
    ee = ct == 1
    assert (eps[ee] > 0).all() and (eps[~ee] == 0).all()


def test_pair_distance_matches_type_fixed_distance_on_every_stencil():
    p, S = scene(gap=0.004)
    xa = ts.Stepper(p, S).xall(p["x0"])
    ct, ci, _ = S.detect(xa, p["dhat"])
    X = [tuple(r) for r in xa]
    for t, ids in zip(ct, ci):
        used = [int(v) for v in ids if v >= 0]
        xs = torch.zeros(4, 3)
        xs[:len(used)] = torch.as_tensor(xa[used])
        d_type = float(en.DIST[int(t)](xs))
        if t == 0:
            d_pair = col.point_triangle(X[used[0]], X[used[1]], X[used[2]], X[used[3]])[2]
        elif t == 1:
            d_pair = col.segment_segment(X[used[0]], X[used[1]], X[used[2]], X[used[3]])[2]
        elif t == 2:
            d_pair = brute_point_segment(xa[used[0]], xa[used[1]], xa[used[2]])
        else:
            d_pair = float(np.sum((xa[used[0]] - xa[used[1]]) ** 2))
        assert d_type == pytest.approx(d_pair, rel=1e-8, abs=1e-16), (t, ids)


def brute_point_segment(p, a, b):
    t = np.clip(np.dot(p - a, b - a) / np.dot(b - a, b - a), 0, 1)
    return float(np.sum((p - a - t * (b - a)) ** 2))


def test_accd_point_falling_on_a_triangle():
    """Exact time of impact h0 / v: ACCD stops before it, with the distance
    kept at or above s times its start, and not far before it."""
    tri = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)]
    for h0, v, s in ((0.1, 0.3, 0.1), (0.05, 1.0, 0.2), (0.2, 0.25, 0.1)):
        x4 = [(0.25, 0.25, h0)] + tri
        p4 = [(0.0, 0.0, -v)] + [(0.0, 0.0, 0.0)] * 3
        t = col.accd(x4, p4, "PT", s=s, t_c=1.0)
        toi = h0 / v
        assert t < toi
        assert h0 - v * t >= s * h0 * (1 - 1e-12)
        assert t >= 0.8 * (1 - s) * toi
    # moving apart: no stop
    x4 = [(0.25, 0.25, 0.1)] + tri
    p4 = [(0.0, 0.0, 0.5)] + [(0.0, 0.0, 0.0)] * 3
    assert col.accd(x4, p4, "PT", 0.1, 1.0) == 1.0


def test_accd_is_conservative_on_random_trajectories():
    rng = np.random.default_rng(5)
    for k in range(60):
        kind = "PT" if k % 2 == 0 else "EE"
        x4 = [tuple(v) for v in rng.normal(size=(4, 3))]
        p4 = [tuple(v) for v in 2.0 * rng.normal(size=(4, 3))]
        t = col.accd(x4, p4, kind, 0.1, 1.0)
        d0 = math.sqrt(col.pair_distance2(x4, kind))
        for tau in np.linspace(0.0, t, 50):
            xt = [tuple(np.asarray(a) + tau * np.asarray(b)) for a, b in zip(x4, p4)]
            assert math.sqrt(col.pair_distance2(xt, kind)) >= 0.099 * d0


def test_free_fall_is_implicit_euler_closed_form():
    """Far from the ground and at rest shape, one frame lands on
    x0 + h v0 + h^2 g exactly (the elastic terms see a rigid translation) and
    v1 = v0 + h g."""
    p, S = scene(gap=0.5, v0=-0.3)
    st = ts.Stepper(p, S)
    x1, v1, info = st.frame(p["x0"], p["v0"], rtol=1e-12)
    h = p["h"]
    g = np.array([0.0, 0.0, -9.81])
    assert np.abs(x1 - (p["x0"] + h * p["v0"] + h * h * g)).max() <= 1e-12
    assert np.abs(v1 - (p["v0"] + h * g)).max() <= 1e-9
    assert info["contacts"] == [0, 0] and info["newton_iters"] == 1


def test_frames_keep_distances_positive_and_energy_decreasing():
    p, S = scene()
    st = ts.Stepper(p, S)
    x, v = p["x0"], p["v0"]
    for f in range(3):
        x, v, info = st.frame(x, v)
        E = info["energies"]
        assert all(E[k + 1] <= E[k] + 1e-12 * abs(E[k]) for k in range(len(E) - 1))
        assert ts.min_distance2(S, st.xall(x)) > 0.0
    assert max(info["contacts"]) > 0
