"""Proximity search and continuous collision detection for time stepping
(float64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper leaves collision detection and CCD to an external module (section
"Limitations": it uses GIPC's, specialised for linear parameterisations, and
times it as "CCD+CD+LargestStep").  Incremental Potential Contact's own
definitions are used here:

* The barrier sums over every point-triangle pair and every edge-edge pair of
  the surface (no shared vertex, at least one free vertex) whose distance is
  below dhat, each pair with the distance between its closest features.  A
  pair is therefore classified by where its closest points lie (point-triangle:
  the face, an edge or a vertex -> PT, PE or PP; edge-edge: both interiors, an
  endpoint, or two endpoints -> EE, PE or PP) and becomes one stencil of that
  type, whose closed-form distance equals the pair's distance.  Pairs are not
  merged (a point near an edge shared by two triangles gives two PE stencils,
  which keeps the total energy continuous across region boundaries).
* The closest features follow the textbook constructions of Ericson,
  Real-Time Collision Detection (2005), section 5.1.5 (point-triangle, by
  Voronoi regions) and section 5.1.9 (segment-segment, clamped parameters).
* The step bound is additive CCD (Li, Kaufman, Jiang 2021, "Codimensional
  Incremental Potential Contact", the ACCD algorithm): conservative advancement
  along the linear trajectory with the per-pair bound of the relative speed,
  stopping once the distance falls below a fraction s of its start value.

The arithmetic is written operation by operation on Python floats (IEEE
double, no fused multiply-add) so that every comparison that decides a type,
a candidate or a stopping step is taken on exactly specified values.

Candidate pairs: a point-triangle / edge-edge pair is tested when the
axis-aligned boxes of its two primitives, each inflated by r on every side,
overlap (proximity: r = sqrt(dhat) / 2; CCD: boxes of the swept primitives
over [x, x + t_max p], same r), which keeps every pair that can matter.
"""
from __future__ import annotations

import math

import numpy as np

PT, EE, PE, PP = 0, 1, 2, 3


# ------------------------------------------------------------ small vector ops
def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _d2(a, b):
    d = _sub(a, b)
    return _dot(d, d)


def _clamp01(v):
    return 0.0 if v < 0.0 else (1.0 if v > 1.0 else v)


# ------------------------------------------------------------ closest features
def point_triangle(p, a, b, c):
    """Closest feature of triangle (a, b, c) to p (Ericson 5.1.5).  Returns
    (kind, local ids, squared distance): kind 'F' (face, ids (0, 1, 2)), 'E'
    (edge, two of 0, 1, 2) or 'V' (vertex, one)."""
    ab, ac, ap = _sub(b, a), _sub(c, a), _sub(p, a)
    d1, d2 = _dot(ab, ap), _dot(ac, ap)
    if d1 <= 0.0 and d2 <= 0.0:
        return "V", (0,), _d2(p, a)
    bp = _sub(p, b)
    d3, d4 = _dot(ab, bp), _dot(ac, bp)
    if d3 >= 0.0 and d4 <= d3:
        return "V", (1,), _d2(p, b)
    vc = d1 * d4 - d3 * d2
    if vc <= 0.0 and d1 >= 0.0 and d3 <= 0.0:
        v = d1 / (d1 - d3)
        q = (a[0] + v * ab[0], a[1] + v * ab[1], a[2] + v * ab[2])
        return "E", (0, 1), _d2(p, q)
    cp = _sub(p, c)
    d5, d6 = _dot(ab, cp), _dot(ac, cp)
    if d6 >= 0.0 and d5 <= d6:
        return "V", (2,), _d2(p, c)
    vb = d5 * d2 - d1 * d6
    if vb <= 0.0 and d2 >= 0.0 and d6 <= 0.0:
        w = d2 / (d2 - d6)
        q = (a[0] + w * ac[0], a[1] + w * ac[1], a[2] + w * ac[2])
        return "E", (0, 2), _d2(p, q)
    va = d3 * d6 - d5 * d4
    if va <= 0.0 and (d4 - d3) >= 0.0 and (d5 - d6) >= 0.0:
        w = (d4 - d3) / ((d4 - d3) + (d5 - d6))
        bc = _sub(c, b)
        q = (b[0] + w * bc[0], b[1] + w * bc[1], b[2] + w * bc[2])
        return "E", (1, 2), _d2(p, q)
    den = 1.0 / (va + vb + vc)
    v, w = vb * den, vc * den
    q = (a[0] + ab[0] * v + ac[0] * w, a[1] + ab[1] * v + ac[1] * w, a[2] + ab[2] * v + ac[2] * w)
    return "F", (0, 1, 2), _d2(p, q)


def segment_segment(p1, q1, p2, q2):
    """Closest points of segments p1q1 and p2q2 (Ericson 5.1.9; both of
    positive length).  Returns (s, t, squared distance), s on the first
    segment and t on the second, each clamped to [0, 1]."""
    d1, d2, r = _sub(q1, p1), _sub(q2, p2), _sub(p1, p2)
    a, e, f = _dot(d1, d1), _dot(d2, d2), _dot(d2, r)
    c, b = _dot(d1, r), _dot(d1, d2)
    den = a * e - b * b
    s = _clamp01((b * f - c * e) / den) if den != 0.0 else 0.0
    t = (b * s + f) / e
    if t < 0.0:
        t = 0.0
        s = _clamp01(-c / a)
    elif t > 1.0:
        t = 1.0
        s = _clamp01((b - c) / a)
    c1 = (p1[0] + d1[0] * s, p1[1] + d1[1] * s, p1[2] + d1[2] * s)
    c2 = (p2[0] + d2[0] * t, p2[1] + d2[1] * t, p2[2] + d2[2] * t)
    return s, t, _d2(c1, c2)


def pt_stencil(pid, tri, kind, loc):
    """The stencil of a point-triangle pair from its closest feature."""
    if kind == "F":
        return PT, (pid, tri[0], tri[1], tri[2])
    if kind == "E":
        return PE, (pid, tri[loc[0]], tri[loc[1]], -1)
    return PP, (pid, tri[loc[0]], -1, -1)


def ee_stencil(ea, eb, s, t):
    """The stencil of an edge-edge pair from its closest-point parameters."""
    sa = 0 if s == 0.0 else (1 if s == 1.0 else -1)
    tb = 0 if t == 0.0 else (1 if t == 1.0 else -1)
    if sa < 0 and tb < 0:
        return EE, (ea[0], ea[1], eb[0], eb[1])
    if sa >= 0 and tb < 0:
        return PE, (ea[sa], eb[0], eb[1], -1)
    if sa < 0 and tb >= 0:
        return PE, (eb[tb], ea[0], ea[1], -1)
    return PP, (ea[sa], eb[tb], -1, -1)


# ------------------------------------------------------------ candidates
def _boxes(x, prims, r):
    P = x[np.asarray(prims, np.int64)]  # (m, k, 3)
    return P.min(axis=1) - r, P.max(axis=1) + r


def _swept_boxes(x, p, t, prims, r):
    a = x[np.asarray(prims, np.int64)]
    b = (x + t * p)[np.asarray(prims, np.int64)]
    return np.minimum(a.min(axis=1), b.min(axis=1)) - r, np.maximum(a.max(axis=1), b.max(axis=1)) + r


def _overlap(lo_a, hi_a, lo_b, hi_b):
    """(na, nb) mask of overlapping boxes (closed intervals on all three axes)."""
    m = np.ones((lo_a.shape[0], lo_b.shape[0]), bool)
    for k in range(3):
        m &= (lo_a[:, None, k] <= hi_b[None, :, k]) & (lo_b[None, :, k] <= hi_a[:, None, k])
    return m


class Surface:
    """Collision surface: point ids, edges (ne, 2), triangles (nt, 3) in the
    vertex id space (free ids < n_free, then n_fixed fixed ids, then affine-body
    vertices with body_of[k]), optional squared rest edge lengths (the EE
    mollifier's thresholds 1e-3 |a|^2 |b|^2).  A pair needs a movable vertex
    (free or on a body) and is skipped when all its vertices lie on one body."""

    def __init__(self, points, edges, tris, n_free, edge_rest_len2=None, n_fixed=None, body_of=None):
        self.points = np.asarray(points, np.int64)
        self.edges = np.asarray(edges, np.int64).reshape(-1, 2)
        self.tris = np.asarray(tris, np.int64).reshape(-1, 3)
        self.n_free = int(n_free)
        self.len2 = None if edge_rest_len2 is None else np.asarray(edge_rest_len2, np.float64)
        self.base = None if n_fixed is None else int(n_free) + int(n_fixed)
        self.body_of = None if body_of is None else np.asarray(body_of, np.int64)

    def _keep(self, ids):
        """The pair of these vertex ids moves, and not as one body."""
        ids = np.asarray(ids, np.int64)
        if self.base is None:
            return bool((ids < self.n_free).any())
        mov = (ids < self.n_free) | (ids >= self.base)
        if not mov.any():
            return False
        if (ids >= self.base).all():
            b = self.body_of[ids - self.base]
            if (b == b[0]).all():
                return False
        return True

    def _pt_candidates(self, lo_p, hi_p, lo_t, hi_t):
        m = _overlap(lo_p, hi_p, lo_t, hi_t)
        out = []
        for i, j in zip(*np.nonzero(m)):  # (point, triangle) in ascending order
            v, tri = int(self.points[i]), self.tris[j]
            if v in tri or not self._keep([v, *tri]):
                continue
            out.append((int(i), int(j)))
        return out

    def _ee_candidates(self, lo_e, hi_e):
        m = _overlap(lo_e, hi_e, lo_e, hi_e)
        out = []
        for i, j in zip(*np.nonzero(np.triu(m, 1))):
            ea, eb = self.edges[i], self.edges[j]
            if ea[0] in eb or ea[1] in eb or not self._keep([*ea, *eb]):
                continue
            out.append((int(i), int(j)))
        return out

    def candidates(self, x, r):
        """Point-triangle and edge-edge candidates at positions x (all ids)."""
        lo_p, hi_p = _boxes(x, self.points[:, None], r)
        lo_t, hi_t = _boxes(x, self.tris, r)
        lo_e, hi_e = _boxes(x, self.edges, r)
        return self._pt_candidates(lo_p, hi_p, lo_t, hi_t), self._ee_candidates(lo_e, hi_e)

    def swept_candidates(self, x, p, t, r):
        lo_p, hi_p = _swept_boxes(x, p, t, self.points[:, None], r)
        lo_t, hi_t = _swept_boxes(x, p, t, self.tris, r)
        lo_e, hi_e = _swept_boxes(x, p, t, self.edges, r)
        return self._pt_candidates(lo_p, hi_p, lo_t, hi_t), self._ee_candidates(lo_e, hi_e)

    # -------------------------------------------------------- proximity
    def detect(self, x, dhat):
        """Contact stencils at positions x (all vertex ids, (n_all, 3)): every
        candidate pair whose squared distance is below dhat, as (ctype (m,),
        cidx (m, 4) -1 padded, ee_eps (m,) or None), point-triangle pairs
        first by (point, triangle), then edge-edge pairs by (edge, edge)."""
        x = np.asarray(x, np.float64)
        pts, ees = self.candidates(x, 0.5 * math.sqrt(dhat))
        ct, ci, eps = [], [], []
        X = [tuple(float(c) for c in row) for row in x]
        for i, j in pts:
            v, tri = int(self.points[i]), [int(a) for a in self.tris[j]]
            kind, loc, d2 = point_triangle(X[v], X[tri[0]], X[tri[1]], X[tri[2]])
            if d2 < dhat:
                t, ids = pt_stencil(v, tri, kind, loc)
                ct.append(t)
                ci.append(ids)
                eps.append(0.0)
        for i, j in ees:
            ea, eb = [int(a) for a in self.edges[i]], [int(a) for a in self.edges[j]]
            s, t, d2 = segment_segment(X[ea[0]], X[ea[1]], X[eb[0]], X[eb[1]])
            if d2 < dhat:
                ty, ids = ee_stencil(ea, eb, s, t)
                ct.append(ty)
                ci.append(ids)
                eps.append(1e-3 * self.len2[i] * self.len2[j] if (ty == EE and self.len2 is not None) else 0.0)
        ct = np.asarray(ct, np.int32)
        ci = np.asarray(ci, np.int32).reshape(-1, 4)
        return ct, ci, (np.asarray(eps) if self.len2 is not None else None)

    # -------------------------------------------------------- CCD
    def ccd(self, x, p, t_max=1.0, s=0.1, dhat=1e-3):
        """Largest conservative step: min over the swept candidates of ACCD's
        step (t_max when none stops earlier)."""
        x = np.asarray(x, np.float64)
        p = np.asarray(p, np.float64)
        pts, ees = self.swept_candidates(x, p, t_max, 0.5 * math.sqrt(dhat))
        X = [tuple(float(c) for c in row) for row in x]
        Pd = [tuple(float(c) for c in row) for row in p]
        t = t_max
        for i, j in pts:
            v, tri = int(self.points[i]), [int(a) for a in self.tris[j]]
            ids = [v] + tri
            t = min(t, accd([X[k] for k in ids], [Pd[k] for k in ids], "PT", s, t))
        for i, j in ees:
            ids = [int(a) for a in self.edges[i]] + [int(a) for a in self.edges[j]]
            t = min(t, accd([X[k] for k in ids], [Pd[k] for k in ids], "EE", s, t))
        return t


def pair_distance2(x4, kind):
    """Squared distance of a point-triangle (x4 = p, a, b, c) or edge-edge
    (x4 = a0, a1, b0, b1) pair."""
    if kind == "PT":
        return point_triangle(x4[0], x4[1], x4[2], x4[3])[2]
    return segment_segment(x4[0], x4[1], x4[2], x4[3])[2]


ACCD_MAX_STEPS = 10000


def accd(x4, p4, kind, s=0.1, t_c=1.0):
    """Additive CCD of one pair along x + t p, t in [0, t_c] (Li, Kaufman,
    Jiang 2021): returns the step reached before the distance fell below s
    times its start value, or t_c if it never does within t_c.  The relative
    motion bound l_p: after removing the mean displacement, the largest
    displacement on each side added (point + triangle, edge + edge); a step
    of (1 - s) d / l_p (first) or 0.9 d / l_p (later) cannot close the gap.
    After ACCD_MAX_STEPS advances the step reached so far is returned (it is
    safe: every advance kept the distance positive); a pair already at
    distance 0 returns 0."""
    pm = tuple(sum(q[k] for q in p4) / 4.0 for k in range(3))
    pr = [_sub(q, pm) for q in p4]
    nrm = [math.sqrt(_dot(q, q)) for q in pr]
    if kind == "PT":
        lp = nrm[0] + max(nrm[1], nrm[2], nrm[3])
    else:
        lp = max(nrm[0], nrm[1]) + max(nrm[2], nrm[3])
    if lp == 0.0:
        return t_c
    x = [tuple(q) for q in x4]
    d = math.sqrt(pair_distance2(x, kind))
    if d == 0.0:
        return 0.0
    g = s * d
    t = 0.0
    tl = (1.0 - s) * d / lp
    for _ in range(ACCD_MAX_STEPS):
        x = [(q[0] + tl * r[0], q[1] + tl * r[1], q[2] + tl * r[2]) for q, r in zip(x, pr)]
        d = math.sqrt(pair_distance2(x, kind))
        if t > 0.0 and d < g:
            return t
        t = t + tl
        if t > t_c:
            return t_c
        tl = 0.9 * d / lp
    return t
