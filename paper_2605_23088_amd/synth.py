"""Seeded synthetic inputs shaped like the paper's scenes.

This module builds problem *inputs* only: tetrahedral blocks, rest shapes,
lumped masses, contact stencil lists and targets.  It holds none of the
method's arithmetic (no energy, distance, derivative, projection, assembly or
solve), so the CPU reference and the GPU library can both consume what it
returns without sharing any of the computation they are compared on.

The paper's meshes (bunny, cloth) are not available; these generators stand in
for them (the paper's scenes are described in its "Examples" section and in
Table 1).

A problem is a plain ``dict`` of numpy arrays and scalars:

``n_free``        free vertices (3 DoF each); vertex ids ``0 .. n_free-1``
``x0``            (n_free, 3) f64 current positions of the free vertices
``x_fixed``       (n_fixed, 3) f64 positions of fixed vertices; a vertex id
                  ``i >= n_free`` names fixed vertex ``i - n_free``
``mass``          (n_free,) f64 lumped vertex masses
``x_tilde``       (n_free, 3) f64 inertial target (ignored when ``static``)
``tet_idx``       (n_t, 4) int32 vertex ids, positively oriented at rest
``dm_inv``        (n_t, 3, 3) f64 inverse rest edge matrices
``vol``           (n_t,) f64 rest volumes
``mu``, ``lam``   Lame parameters (scalars) or ``mu_t``/``lam_t`` (n_t,) arrays
``ctype``         (n_c,) int32 stencil type: 0 PT, 1 EE, 2 PE, 3 PP
``cidx``          (n_c, 4) int32 vertex ids, -1 for unused trailing entries
``h``, ``kappa``, ``dhat``, ``gravity``, ``rho``, ``static``
"""
from __future__ import annotations

import numpy as np

PT, EE, PE, PP = 0, 1, 2, 3
GRAVITY = np.array([0.0, 0.0, -9.81])

# Seeds of the five standard workloads.
SEEDS = {"C1": 20261, "C2": 20262, "C3": 20263, "C4": 20264, "C5": 20265}


def lame(E, nu):
    """Young's modulus / Poisson ratio -> (mu, lambda) (standard conversion)."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def _streams(seed):
    """Independent sub-streams, in the order [positions/F, contacts, theta, target]."""
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


# --------------------------------------------------------------------------
# Kuhn-split grid blocks
# --------------------------------------------------------------------------

def grid_vertices(nx, ny, nz, a, origin=(0.0, 0.0, 0.0)):
    """Lexicographic vertex positions, id = i + (nx+1)(j + (ny+1)k)."""
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1).astype(np.float64) * a
    return X + np.asarray(origin, dtype=np.float64)


def grid_vid(nx, ny, i, j, k):
    return i + (nx + 1) * (j + (ny + 1) * k)


def kuhn_tets(nx, ny, nz):
    """Six tets per cube cell along the v000 -> v111 diagonal (all cells alike).

    For each axis permutation p the tet follows the monotone lattice path
    v000 -> v000+e_p0 -> v000+e_p0+e_p1 -> v111.  Odd permutations have the
    middle two vertices swapped so that every tet is positively oriented.
    """
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    offs = []
    for p in perms:
        e = np.eye(3, dtype=np.int64)
        path = [np.zeros(3, np.int64), e[p[0]], e[p[0]] + e[p[1]], np.ones(3, np.int64)]
        D = np.stack([path[1] - path[0], path[2] - path[0], path[3] - path[0]], axis=1)
        if np.linalg.det(D) < 0:
            path[1], path[2] = path[2], path[1]
        offs.append(path)
    offs = np.array(offs)  # (6, 4, 3)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)  # (cells, 3)
    corner = base[:, None, None, :] + offs[None, :, :, :]  # (cells, 6, 4, 3)
    vid = grid_vid(nx, ny, corner[..., 0], corner[..., 1], corner[..., 2])
    return vid.reshape(-1, 4).astype(np.int64)


def face_triangles(nx, ny, k):
    """Triangles of the horizontal face z-layer k (each cell split along its
    (0,0)-(1,1) diagonal, which is the diagonal the Kuhn tets induce on the
    top and bottom faces).  Returns (2*nx*ny, 3) vertex ids."""
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i, j = i.ravel(), j.ravel()
    v00 = grid_vid(nx, ny, i, j, k)
    v10 = grid_vid(nx, ny, i + 1, j, k)
    v01 = grid_vid(nx, ny, i, j + 1, k)
    v11 = grid_vid(nx, ny, i + 1, j + 1, k)
    return np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v01, v11], 1)]).astype(np.int64)


def face_edges(nx, ny, k):
    """Edges of face layer k: x-edges, y-edges and the (0,0)-(1,1) diagonals."""
    out = []
    j, i = np.meshgrid(np.arange(ny + 1), np.arange(nx), indexing="ij")
    out.append(np.stack([grid_vid(nx, ny, i, j, k), grid_vid(nx, ny, i + 1, j, k)], -1).reshape(-1, 2))
    j, i = np.meshgrid(np.arange(ny), np.arange(nx + 1), indexing="ij")
    out.append(np.stack([grid_vid(nx, ny, i, j, k), grid_vid(nx, ny, i, j + 1, k)], -1).reshape(-1, 2))
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    out.append(np.stack([grid_vid(nx, ny, i, j, k), grid_vid(nx, ny, i + 1, j + 1, k)], -1).reshape(-1, 2))
    return np.concatenate(out).astype(np.int64)


def haar_rotations(rng, n):
    """n rotation matrices uniform on SO(3) (normalised Gaussian quaternions)."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _edge_matrix(X, tets):
    """Columns X1-X0, X2-X0, X3-X0 (the rest-shape input of each tet)."""
    return np.stack([X[tets[:, 1]] - X[tets[:, 0]],
                     X[tets[:, 2]] - X[tets[:, 0]],
                     X[tets[:, 3]] - X[tets[:, 0]]], axis=2)


def _lumped_mass(n, tets, vol, rho):
    m = np.zeros(n)
    np.add.at(m, tets.ravel(), np.repeat(rho * vol / 4.0, 4))
    return m


def _random_rest_shapes(rng, X, tets, smin=0.7, smax=1.4):
    """Rest shapes such that x = X has deformation gradient U diag(s) V^T in every
    tet: Dm^-1 := Ds(X)^-1 F_t and V_t = |det Ds(X)| / (6 det F_t)."""
    nt = tets.shape[0]
    U = haar_rotations(rng, nt)
    Vr = haar_rotations(rng, nt)
    s = rng.uniform(smin, smax, size=(nt, 3))
    F = np.einsum("nij,nj,nkj->nik", U, s, Vr)
    Ds = _edge_matrix(X, tets)
    dm_inv = np.linalg.solve(Ds, F)
    vol = np.abs(np.linalg.det(Ds)) / (6.0 * np.prod(s, axis=1))
    return dm_inv, vol


def _pack(n_free, x0, x_fixed, mass, x_tilde, tets, dm_inv, vol, ctype, cidx, **kw):
    p = dict(
        n_free=int(n_free),
        x0=np.ascontiguousarray(x0, dtype=np.float64),
        x_fixed=np.ascontiguousarray(x_fixed, dtype=np.float64).reshape(-1, 3),
        mass=np.ascontiguousarray(mass, dtype=np.float64),
        x_tilde=np.ascontiguousarray(x_tilde, dtype=np.float64),
        tet_idx=np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4),
        dm_inv=np.ascontiguousarray(dm_inv, dtype=np.float64).reshape(-1, 3, 3),
        vol=np.ascontiguousarray(vol, dtype=np.float64),
        ctype=np.ascontiguousarray(ctype, dtype=np.int32),
        cidx=np.ascontiguousarray(cidx, dtype=np.int32).reshape(-1, 4),
        gravity=GRAVITY.copy(),
        static=False,
    )
    p.update(kw)
    return p


# --------------------------------------------------------------------------
# Contacts against a fixed collider under the bottom face
# --------------------------------------------------------------------------

def _collider_contacts(rng, X, nx, ny, n_pt, n_ee, n_free, dlo=1e-4, dhi=1e-3, tri_ok=None, ee_angle=None):
    """PT and EE stencils between the bottom face (z = 0) of a grid block and a
    private fixed feature per stencil placed below it.

    PT: a uniformly chosen bottom triangle (among those where `tri_ok`, a mask
        over the bottom triangles, is set) and a fixed point at
        centroid - sqrt(d) z, d ~ U(dlo, dhi) (d is a squared distance).
    EE: a uniformly chosen bottom edge and a fixed horizontal edge of length a,
        perpendicular to it, through midpoint - sqrt(d) z; with ee_angle =
        (lo, hi) the fixed edge instead makes an angle +-U(lo, hi) (radians)
        with the bottom edge (near-parallel pairs for the edge-edge mollifier;
        the lines still cross above each other's midpoints).
    Both are interior-type by construction.  Returns (ctype, cidx, x_fixed)."""
    tris = face_triangles(nx, ny, 0)
    edges = face_edges(nx, ny, 0)
    a = X[1, 0] - X[0, 0]
    fixed = []
    ctype, cidx = [], []
    if n_pt:
        pool = tris if tri_ok is None else tris[tri_ok]
        t = pool[rng.integers(0, pool.shape[0], size=n_pt)]
        d = rng.uniform(dlo, dhi, size=n_pt)
        c = X[t].mean(axis=1)
        c[:, 2] -= np.sqrt(d)
        fid = n_free + np.arange(n_pt)
        fixed.append(c)
        ctype.append(np.full(n_pt, PT))
        cidx.append(np.stack([fid, t[:, 0], t[:, 1], t[:, 2]], 1))
    if n_ee:
        e = edges[rng.integers(0, edges.shape[0], size=n_ee)]
        d = rng.uniform(dlo, dhi, size=n_ee)
        p0, p1 = X[e[:, 0]], X[e[:, 1]]
        mid = 0.5 * (p0 + p1)
        mid[:, 2] -= np.sqrt(d)
        dirn = p1 - p0
        perp = np.stack([-dirn[:, 1], dirn[:, 0], np.zeros(n_ee)], 1)
        perp /= np.linalg.norm(perp, axis=1, keepdims=True)
        if ee_angle is not None:
            th = rng.uniform(ee_angle[0], ee_angle[1], size=n_ee) * rng.choice([-1.0, 1.0], size=n_ee)
            u = dirn / np.linalg.norm(dirn, axis=1, keepdims=True)
            perp = np.cos(th)[:, None] * u + np.sin(th)[:, None] * perp
        q0 = mid - 0.5 * a * perp
        q1 = mid + 0.5 * a * perp
        base = n_free + n_pt
        fid0 = base + 2 * np.arange(n_ee)
        fixed.append(np.stack([q0, q1], 1).reshape(-1, 3))
        ctype.append(np.full(n_ee, EE))
        cidx.append(np.stack([e[:, 0], e[:, 1], fid0, fid0 + 1], 1))
    if not ctype:
        return np.zeros(0, np.int32), np.zeros((0, 4), np.int32), np.zeros((0, 3))
    return (np.concatenate(ctype).astype(np.int32), np.concatenate(cidx).astype(np.int32),
            np.concatenate(fixed))


def block_problem(nx, ny, nz, a, n_pt, n_ee, seed, E=1e5, nu=0.4, rho=1000.0, h=1e-2,
                  kappa=1e4, dhat=1e-3, random_F=True, name="block", dlo=1e-4, dhi=1e-3, ee_angle=None):
    """A Kuhn block [0, nx a] x [0, ny a] x [0, nz a] at its exact grid positions,
    with seeded per-tet rest shapes (so x0 carries random deformation gradients
    with singular values in [0.7, 1.4]) and n_pt + n_ee contact stencils against
    a fixed collider under the bottom face, squared distances U(dlo, dhi) (a
    range reaching past dhat gives inactive stencils).  All block vertices are
    free.  With ee_angle the collider edges are near-parallel to their bottom
    edges (see _collider_contacts) and the problem carries `ee_eps`, IPC's
    mollifier thresholds 1e-3 |e_a|^2 |e_b|^2 of every EE stencil from the
    edge lengths at x0 (0 for the other stencils)."""
    r_pos, r_con, _, _ = _streams(seed)
    X = grid_vertices(nx, ny, nz, a)
    tets = kuhn_tets(nx, ny, nz)
    if random_F:
        dm_inv, vol = _random_rest_shapes(r_pos, X, tets)
    else:
        Ds = _edge_matrix(X, tets)
        dm_inv, vol = np.linalg.inv(Ds), np.abs(np.linalg.det(Ds)) / 6.0
    n = X.shape[0]
    mass = _lumped_mass(n, tets, vol, rho)
    ctype, cidx, x_fixed = _collider_contacts(r_con, X, nx, ny, n_pt, n_ee, n, dlo, dhi, ee_angle=ee_angle)
    mu, lam = lame(E, nu)
    x_tilde = X + h * h * GRAVITY
    p = _pack(n, X, x_fixed, mass, x_tilde, tets, dm_inv, vol, ctype, cidx,
              mu=mu, lam=lam, h=h, kappa=kappa, dhat=dhat, rho=rho, name=name,
              grid=(nx, ny, nz), spacing=a)
    if ee_angle is not None:
        xa = np.concatenate([X, x_fixed])
        ee = ctype == EE
        ea = xa[cidx[ee, 1]] - xa[cidx[ee, 0]]
        eb = xa[cidx[ee, 3]] - xa[cidx[ee, 2]]
        eps = np.zeros(len(ctype))
        eps[ee] = 1e-3 * (ea * ea).sum(1) * (eb * eb).sum(1)
        p["ee_eps"] = eps
    return p


# --------------------------------------------------------------------------
# The five standard workloads
# --------------------------------------------------------------------------

def _seg_cross_2d(p, r, q, s):
    """Proper crossing of 2-D segments p + t r and q + u s; returns (ok, t, u)."""
    den = r[0] * s[1] - r[1] * s[0]
    if abs(den) < 1e-12:
        return False, 0.0, 0.0
    w = q - p
    t = (w[0] * s[1] - w[1] * s[0]) / den
    u = (w[0] * r[1] - w[1] * r[0]) / den
    return (0.0 < t < 1.0 and 0.0 < u < 1.0), t, u


def c1_two_cubes(seed=SEEDS["C1"], margin=0.04):
    """Two stacked 4x4x4-cell Neo-Hookean cubes (384 tets, 125 vertices each),
    E = 1e5, nu = 0.4, rho = 1000, h = 1e-2, positions jittered N(0, 1e-3),
    d_hat = 1e-3, kappa = 1e4.

    Cube A is [0,1]^3; cube B is A shifted by (0.125, 0.0625, 1.02).  The stencil
    list holds every point-triangle pair whose point projects inside the
    triangle (A's top face vs B's bottom vertices and B's bottom face vs A's top
    vertices) and every non-parallel edge-edge pair of those two faces whose
    projections cross.  The 0.02 m gap makes the squared distance 4e-4 < d_hat;
    every kept pair lies at least `margin` metres (in the horizontal plane) from
    the boundary of its closest-feature region, which the generator asserts, so
    all stencils are interior-type PT or EE."""
    n1 = 4
    a = 0.25
    r_pos = _streams(seed)[0]
    XA = grid_vertices(n1, n1, n1, a)
    off = np.array([0.125, 0.0625, 1.02])
    XB = XA + off
    X = np.concatenate([XA, XB])
    nA = XA.shape[0]
    tA = kuhn_tets(n1, n1, n1)
    tets = np.concatenate([tA, tA + nA])
    Ds = _edge_matrix(X, tets)
    dm_inv = np.linalg.inv(Ds)
    vol = np.abs(np.linalg.det(Ds)) / 6.0
    rho, h = 1000.0, 1e-2
    n = X.shape[0]
    mass = _lumped_mass(n, tets, vol, rho)
    x0 = X + r_pos.normal(0.0, 1e-3, size=X.shape)

    topA = face_triangles(n1, n1, n1)
    botB = face_triangles(n1, n1, 0) + nA
    topA_v = np.unique(topA)
    botB_v = np.unique(botB)
    ctype, cidx = [], []

    def tri_pairs(points, tris):
        for pv in points:
            P = X[pv, :2]
            for t in tris:
                A, B, C = X[t[0], :2], X[t[1], :2], X[t[2], :2]
                # distances (metres) from P to the three edge lines, signed inward
                ds = []
                for U, W, O in ((A, B, C), (B, C, A), (C, A, B)):
                    e = W - U
                    nrm = np.array([-e[1], e[0]]) / np.hypot(e[0], e[1])
                    if np.dot(O - U, nrm) < 0:
                        nrm = -nrm
                    ds.append(np.dot(P - U, nrm))
                if min(ds) > 0:
                    assert min(ds) >= margin, "C1 PT pair too close to a region boundary"
                    ctype.append(PT)
                    cidx.append([pv, t[0], t[1], t[2]])

    tri_pairs(botB_v, topA)
    tri_pairs(topA_v, botB)

    eA = face_edges(n1, n1, n1)
    eB = face_edges(n1, n1, 0) + nA
    for ea in eA:
        p, r = X[ea[0], :2], X[ea[1], :2] - X[ea[0], :2]
        for eb in eB:
            q, s = X[eb[0], :2], X[eb[1], :2] - X[eb[0], :2]
            cr = r[0] * s[1] - r[1] * s[0]
            if cr * cr < 1e-3 * np.dot(r, r) * np.dot(s, s):
                continue  # near-parallel pair: dropped
            ok, t, u = _seg_cross_2d(p, r, q, s)
            if not ok:
                continue
            La, Lb = np.hypot(*r), np.hypot(*s)
            assert min(t, 1 - t) * La >= margin and min(u, 1 - u) * Lb >= margin, \
                "C1 EE pair too close to a region boundary"
            ctype.append(EE)
            cidx.append([ea[0], ea[1], eb[0], eb[1]])

    mu, lam = lame(1e5, 0.4)
    return _pack(n, x0, np.zeros((0, 3)), mass, x0 + h * h * GRAVITY, tets, dm_inv, vol,
                 np.array(ctype), np.array(cidx), mu=mu, lam=lam, h=h, kappa=1e4,
                 dhat=1e-3, rho=rho, name="C1")


def c2_block(seed=SEEDS["C2"], cells=40, n_pt=200_000, n_ee=200_000):
    """Plain FP64 at scale: 40^3-cell block (384,000 tets, 68,921 vertices) with
    seeded random deformation gradients and 200k PT + 200k EE stencils against
    a fixed flat collider, squared distances uniform in (1e-4, 1e-3)."""
    return block_problem(cells, cells, cells, 1.0 / cells, n_pt, n_ee, seed, name="C2")


def c4_block(seed=SEEDS["C4"], n_pt=750_000, n_ee=750_000):
    """Precision-form workload: 80x80x52 cells (1,996,800 tets, 347,733 vertices)
    with 750k PT + 750k EE collider stencils."""
    return block_problem(80, 80, 52, 1.0 / 80, n_pt, n_ee, seed, name="C4")


def c5_static(seed=SEEDS["C5"], nx=48, ny=48, nz=29, a=0.02, n_pt=300_000, nu=0.4,
              rho=1000.0, kappa=136.0, dhat=1e-3, pin="rim"):
    """Differentiation-form workload: static equilibrium of a 48x48x29-cell block
    (400,896 tets, 72,030 vertices) under gravity, per-tet Young's modulus
    theta log-uniform in [5e4, 2e5], 300k PT stencils against fixed points
    under the bottom face, and fixed vertices `pin`: "rim" (default) the
    boundary ring of the bottom face (192 vertices), "corners" its 4 corners.
    The PT stencils avoid bottom triangles whose 3 vertices are all fixed.
    Also returns a seeded target x_tgt = x0 + N(0, 1e-3).

    The contacts act along the normals of the bottom triangles, so once the
    bottom sags they push sideways as well; with only the 4 corners fixed,
    nothing but the shear of the elements at those 4 vertices holds the block,
    and it slides off as a near-rigid body (an almost singular exact Hessian).
    The fixed rim holds it.

    kappa = 136: at x0 the barriers' total upward force on the free vertices
    of the default block (38.42 kappa N) equals their weight (5,240.0 N) to
    within 0.3 %, so the block rests on the contact layer.  The two cubes' kappa = 1e4 would push up with
    about 76 times the weight against the fixed vertices.  Smaller blocks pass
    their own kappa."""
    r_pos, r_con, r_theta, r_tgt = _streams(seed)
    X = grid_vertices(nx, ny, nz, a)
    tets = kuhn_tets(nx, ny, nz)
    Ds = _edge_matrix(X, tets)
    dm_inv, vol = np.linalg.inv(Ds), np.abs(np.linalg.det(Ds)) / 6.0
    nv = X.shape[0]
    if pin == "corners":
        pinned = np.array([grid_vid(nx, ny, i, j, 0) for i in (0, nx) for j in (0, ny)])
    elif pin == "rim":
        pinned = np.array([grid_vid(nx, ny, i, j, 0) for j in range(ny + 1) for i in range(nx + 1)
                           if i in (0, nx) or j in (0, ny)])
    else:
        raise ValueError(f"unknown pin set {pin!r}")
    is_fixed = np.zeros(nv, bool)
    is_fixed[pinned] = True
    free = np.flatnonzero(~is_fixed)
    n_free = free.size
    n_pin = pinned.size
    new_id = np.empty(nv, np.int64)
    new_id[free] = np.arange(n_free)
    new_id[pinned] = n_free + np.arange(n_pin)
    # contacts (vertex ids in the original numbering, fixed partners after the
    # pinned vertices) on bottom triangles with at least one free vertex
    tri_ok = None if pin == "corners" else ~is_fixed[face_triangles(nx, ny, 0)].all(axis=1)
    ctype, cidx, x_part = _collider_contacts(r_con, X, nx, ny, n_pt, 0, nv, tri_ok=tri_ok)
    cidx = cidx.astype(np.int64)
    part = cidx[:, 0] - nv
    tri = new_id[cidx[:, 1:]]
    cidx = np.concatenate([(n_free + n_pin + part)[:, None], tri], 1)
    theta = np.exp(r_theta.uniform(np.log(5e4), np.log(2e5), size=tets.shape[0]))
    mu1, lam1 = lame(1.0, nu)
    mass_all = _lumped_mass(nv, tets, vol, rho)
    x0 = X[free]
    x_tgt = x0 + r_tgt.normal(0.0, 1e-3, size=x0.shape)
    x_fixed = np.concatenate([X[pinned], x_part])
    return _pack(n_free, x0, x_fixed, mass_all[free], np.zeros_like(x0), new_id[tets], dm_inv,
                 vol, ctype, cidx, mu_t=theta * mu1, lam_t=theta * lam1, theta=theta,
                 mu1=mu1, lam1=lam1, h=1.0, kappa=kappa, dhat=dhat, rho=rho, static=True,
                 x_tgt=x_tgt, name="C5", grid=(nx, ny, nz), spacing=a)


VERTEX_INDEX_KEYS = ("tet_idx", "cidx", "tri_idx", "hinge_idx")
VERTEX_ROW_KEYS = ("x0", "mass", "x_tilde", "v0", "x_tgt")


def permute_vertices(prob, seed=12345):
    """The same problem with its free vertices relabelled by a seeded random
    permutation (new id perm[v] for old vertex v; fixed ids and -1 padding
    unchanged), as the paper does to keep SpMV timings free of favourable
    memory locality (section "SpMV" of the evaluation).  Returns (problem, perm)."""
    n = int(prob["n_free"])
    perm = np.random.default_rng(seed).permutation(n).astype(np.int64)
    q = dict(prob)
    for key in VERTEX_ROW_KEYS:
        if key in prob and prob[key] is not None:
            a = np.asarray(prob[key])
            if a.shape[0] == n:
                b = np.empty_like(a)
                b[perm] = a
                q[key] = b
    for key in VERTEX_INDEX_KEYS:
        if key in prob and prob[key] is not None and len(prob[key]):
            idx = np.asarray(prob[key])
            free = (idx >= 0) & (idx < n)
            out = idx.copy()
            out[free] = perm[idx[free]]
            q[key] = out.astype(idx.dtype)
    return q, perm


def small_block(seed=7, nx=5, ny=4, nz=3, n_pt=150, n_ee=150, **kw):
    """A few-hundred-tet version of the metric workload for fast parity runs."""
    return block_problem(nx, ny, nz, 1.0 / max(nx, ny, nz), n_pt, n_ee, seed,
                         name=f"block{nx}x{ny}x{nz}", **kw)


# --------------------------------------------------------------------------
# Cloth sheets and the heterogeneous workload
# --------------------------------------------------------------------------

def sheet(n, angle, center=(0.5, 0.5)):
    """A unit square sheet of n x n cells rotated by `angle` about `center` in
    the horizontal plane.  Returns rest coordinates (V, 2) in the sheet frame,
    world (x, y) of every vertex, CCW triangles (2 per cell, split along the
    (0,0)-(1,1) diagonal), and hinges (e0, e1, w1, w2) over interior edges with
    (e0, e1, w1) and (e1, e0, w2) the two triangles (so the two unnormalised
    normals (e1 - e0) x (w1 - e0) and (w2 - e0) x (e1 - e0) agree on a flat
    sheet)."""
    j, i = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    uv = np.stack([i.ravel(), j.ravel()], 1).astype(np.float64) / n
    c, s = np.cos(angle), np.sin(angle)
    d = uv - 0.5
    xy = np.stack([c * d[:, 0] - s * d[:, 1], s * d[:, 0] + c * d[:, 1]], 1) + np.asarray(center)
    vid = lambda a, b: a + (n + 1) * b
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    v00, v10, v01, v11 = vid(ii, jj), vid(ii + 1, jj), vid(ii, jj + 1), vid(ii + 1, jj + 1)
    tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v11, v01], 1)])
    # hinges from the directed edges of the CCW triangles
    de = np.concatenate([tris[:, [0, 1, 2]], tris[:, [1, 2, 0]], tris[:, [2, 0, 1]]])  # (e0, e1, wing)
    key = de[:, 0] * (n + 1) ** 2 + de[:, 1]
    twin = de[:, 1] * (n + 1) ** 2 + de[:, 0]
    order = np.argsort(key)
    pos = np.searchsorted(key[order], twin)
    pos = np.minimum(pos, len(key) - 1)
    has = key[order][pos] == twin
    a_idx = np.flatnonzero(has & (de[:, 0] < de[:, 1]))
    b_idx = order[pos[a_idx]]
    hinges = np.stack([de[a_idx, 0], de[a_idx, 1], de[a_idx, 2], de[b_idx, 2]], 1)
    return uv, xy, tris.astype(np.int64), hinges.astype(np.int64)


def _tri_wave(t):
    return 2.0 * np.abs(t - np.floor(t + 0.5))


def _closest_pt_triangle(p, a, b, c):
    """Closest point of triangles (a, b, c) to points p (vectorised Voronoi-region
    test of Ericson, Real-Time Collision Detection, sec. 5.1.5).  Returns the
    squared distance and the region: 0 face, 1 edge ab, 2 edge bc, 3 edge ca,
    4 vertex a, 5 vertex b, 6 vertex c."""
    ab, ac, ap = b - a, c - a, p - a
    d1, d2 = (ab * ap).sum(1), (ac * ap).sum(1)
    bp = p - b
    d3, d4 = (ab * bp).sum(1), (ac * bp).sum(1)
    cp = p - c
    d5, d6 = (ab * cp).sum(1), (ac * cp).sum(1)
    va = d3 * d6 - d5 * d4
    vb = d5 * d2 - d1 * d6
    vc = d1 * d4 - d3 * d2
    region = np.zeros(len(p), np.int64)
    q = np.empty_like(p)
    denom = va + vb + vc
    with np.errstate(divide="ignore", invalid="ignore"):
        v = vb / denom
        w = vc / denom
    q[:] = a + ab * v[:, None] + ac * w[:, None]
    # edges
    m_ab = (vc <= 0) & (d1 >= 0) & (d3 <= 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_ab = d1 / (d1 - d3)
    q[m_ab] = (a + ab * t_ab[:, None])[m_ab]
    region[m_ab] = 1
    m_ac = (vb <= 0) & (d2 >= 0) & (d6 <= 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_ac = d2 / (d2 - d6)
    q[m_ac] = (a + ac * t_ac[:, None])[m_ac]
    region[m_ac] = 3
    m_bc = (va <= 0) & ((d4 - d3) >= 0) & ((d5 - d6) >= 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        t_bc = (d4 - d3) / ((d4 - d3) + (d5 - d6))
    q[m_bc] = (b + (c - b) * t_bc[:, None])[m_bc]
    region[m_bc] = 2
    # vertices
    m_a = (d1 <= 0) & (d2 <= 0)
    m_b = (d3 >= 0) & (d4 <= d3)
    m_c = (d6 >= 0) & (d5 <= d6)
    q[m_a], region[m_a] = a[m_a], 4
    q[m_b], region[m_b] = b[m_b], 5
    q[m_c], region[m_c] = c[m_c], 6
    return ((p - q) ** 2).sum(1), region


def _closest_seg_seg(p1, q1, p2, q2):
    """Closest points of segments p1q1 and p2q2 (Ericson sec. 5.1.9, vectorised,
    non-degenerate segments).  Returns squared distance, s, t (parameters on
    each segment, clamped to [0, 1])."""
    d1, d2, r = q1 - p1, q2 - p2, p1 - p2
    a, e, f = (d1 * d1).sum(1), (d2 * d2).sum(1), (d2 * r).sum(1)
    c, b = (d1 * r).sum(1), (d1 * d2).sum(1)
    denom = a * e - b * b
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(denom > 0, np.clip((b * f - c * e) / denom, 0.0, 1.0), 0.0)
        t = (b * s + f) / e
    lo, hi = t < 0, t > 1
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(lo, np.clip(-c / a, 0, 1), np.where(hi, np.clip((b - c) / a, 0, 1), s))
    t = np.clip(t, 0, 1)
    c1 = p1 + d1 * s[:, None]
    c2 = p2 + d2 * t[:, None]
    return ((c1 - c2) ** 2).sum(1), s, t


def _pairs_near(pts_xy, prim_lo_xy, prim_hi_xy, cell, reach):
    """Hashed proximity search in the horizontal plane: every (point, primitive)
    pair whose point lies within `reach` of the primitive's xy bounding box.
    Primitives are hashed into every cell of side `cell` their grown box
    touches; points look up their own cell, then the exact box test filters."""
    glo = prim_lo_xy - reach
    ghi = prim_hi_xy + reach
    klo = np.floor(glo / cell).astype(np.int64)
    khi = np.floor(ghi / cell).astype(np.int64)
    span = khi - klo + 1
    base = np.floor(min(pts_xy[:, 0].min(), glo[:, 0].min()) / cell) - 1, \
        np.floor(min(pts_xy[:, 1].min(), glo[:, 1].min()) / cell) - 1
    width = 4 + int(np.ceil((max(pts_xy[:, 0].max(), ghi[:, 0].max()) / cell) - base[0]))
    cells, owners = [], []
    for dx in range(int(span[:, 0].max())):
        for dy in range(int(span[:, 1].max())):
            o = np.flatnonzero((dx < span[:, 0]) & (dy < span[:, 1]))
            cells.append((klo[o, 0] + dx - int(base[0])) + width * (klo[o, 1] + dy - int(base[1])))
            owners.append(o)
    cells = np.concatenate(cells)
    owners = np.concatenate(owners)
    order = np.argsort(cells, kind="stable")
    cells, owners = cells[order], owners[order]
    kp = np.floor(pts_xy / cell).astype(np.int64)
    ph = (kp[:, 0] - int(base[0])) + width * (kp[:, 1] - int(base[1]))
    lo = np.searchsorted(cells, ph, "left")
    cnt = np.searchsorted(cells, ph, "right") - lo
    pi = np.repeat(np.arange(len(ph)), cnt)
    first = np.repeat(lo - (np.cumsum(cnt) - cnt), cnt)
    oi = owners[np.arange(len(pi)) + first]
    q = pts_xy[pi]
    inside = np.all((q >= glo[oi]) & (q <= ghi[oi]), axis=1)
    return pi[inside], oi[inside]


def _xy_box(X, prims):
    P = X[prims][..., :2]
    return P.min(axis=1), P.max(axis=1)


def _point_side(Xp, pid, Xt, tris, dhat, reach, cell):
    """Points `pid` of one layer against the triangles of another: Voronoi-region
    classification of every candidate within the window, d < dhat.  Returns
    (point, tri-local) index arrays and the region code per kept pair."""
    lo, hi = _xy_box(Xt, tris)
    pi, ti = _pairs_near(Xp[pid, :2], lo, hi, cell, reach)
    P = Xp[pid[pi]]
    d, reg = _closest_pt_triangle(P, Xt[tris[ti, 0]], Xt[tris[ti, 1]], Xt[tris[ti, 2]])
    keep = d < dhat
    return pid[pi[keep]], ti[keep], reg[keep], d[keep]


def _proximity(layers, dhat, reach, cell, eps_cross=1e-3):
    """Typed proximity stencils between every pair of distinct layers (global
    vertex ids).  Each layer is (X, off, surface triangles, surface edges,
    surface points) in its own local ids.  Returns {type: (m, 4) int64 pool}
    deduplicated by canonical tuple, and the matching squared distances."""
    pools = {PT: [], EE: [], PE: [], PP: []}
    dists = {PT: [], EE: [], PE: [], PP: []}
    edge_of_region = np.array([[0, 1], [1, 2], [2, 0]])
    for l in range(len(layers)):
        for u in range(len(layers)):
            if l == u:
                continue
            XL, oL, tL, eL, vL = layers[l]
            XU, oU, tU, eU, vU = layers[u]
            # points of U against triangles of L (both orders are visited)
            p, t, reg, d = _point_side(XU, vU, XL, tL, dhat, reach, cell)
            face = reg == 0
            pools[PT].append(np.stack([p[face] + oU, *(tL[t[face]].T + oL)], 1))
            dists[PT].append(d[face])
            ed = (reg >= 1) & (reg <= 3)
            e = tL[t[ed][:, None], edge_of_region[reg[ed] - 1]] + oL
            e.sort(axis=1)
            pools[PE].append(np.stack([p[ed] + oU, e[:, 0], e[:, 1], np.full(ed.sum(), -1)], 1))
            dists[PE].append(d[ed])
            vx = reg >= 4
            q = tL[t[vx], reg[vx] - 4] + oL
            a_, b_ = p[vx] + oU, q
            pools[PP].append(np.stack([np.minimum(a_, b_), np.maximum(a_, b_), np.full(vx.sum(), -1),
                                       np.full(vx.sum(), -1)], 1))
            dists[PP].append(d[vx])
            if u < l:
                continue
            # edges of U against edges of L (each unordered layer pair once)
            mid = 0.5 * (XU[eU[:, 0], :2] + XU[eU[:, 1], :2])
            lo, hi = _xy_box(XL, eL)
            ui, li = _pairs_near(mid, lo, hi, cell, reach)
            p1, q1 = XU[eU[ui, 0]], XU[eU[ui, 1]]
            p2, q2 = XL[eL[li, 0]], XL[eL[li, 1]]
            dd, s, tt = _closest_seg_seg(p1, q1, p2, q2)
            cr = np.cross(q1 - p1, q2 - p2)
            ok = (cr * cr).sum(1) >= eps_cross * ((q1 - p1) ** 2).sum(1) * ((q2 - p2) ** 2).sum(1)
            ok &= (dd < dhat) & (s > 0) & (s < 1) & (tt > 0) & (tt < 1)
            A = eU[ui[ok]] + oU
            B = eL[li[ok]] + oL
            lo_first = A[:, 0] < B[:, 0]
            pools[EE].append(np.where(lo_first[:, None], np.concatenate([A, B], 1), np.concatenate([B, A], 1)))
            dists[EE].append(dd[ok])
    out, dout = {}, {}
    for t in pools:
        P = np.concatenate(pools[t]).astype(np.int64)
        D = np.concatenate(dists[t])
        P, first = np.unique(P, axis=0, return_index=True)
        out[t], dout[t] = P, D[first]
    return out, dout


def c3_cloth(seed=SEEDS["C3"], block=(50, 50, 20), a=0.02, sheet_cells=250, n_sheets=4,
             counts=(400_000, 400_000, 150_000, 50_000), E=1e5, nu=0.4, E_c=1e5, nu_c=0.3, rho=1000.0,
             thickness=1e-3, k_b=0.055, h=1e-2, kappa=1.0, dhat=1e-3, reach=None, name="C3"):
    """Heterogeneous workload: a Kuhn tet block (per-tet random rest shapes as in
    the 40^3 workload, top face flat) under `n_sheets` stacked cloth sheets
    (StVK membrane + dihedral bending, flat at rest), sheet k rotated by
    7.5 + 15k degrees about the vertical axis through (0.5, 0.5), heights given
    by nested gap fields z_k = z_top + sum_{j<=k} g_j with
    g_j = sqrt(10^(-5 + 2 w_j)), w_j = tri(4 (x cos b_j + y sin b_j)), b_j seeded.

    kappa = 1 (not the two cubes' 1e4): with 1.6e-5 kg cloth vertices a barrier
    stiffness of 1e4 makes block-Jacobi PCG need 1e4-1e5 iterations even on
    small versions of this scene; at 1 it needs ~1e3.

    Contacts: a near-field hashed proximity search (window `reach`, default one
    sheet spacing) between every pair of layers, Voronoi-region classification
    of point-triangle candidates into PT / PE / PP, interior-closest-point EE
    candidates with IPC's near-parallel cut, d < dhat, de-duplication by
    canonical tuple, then seeded subsampling to exactly `counts`
    (PT, EE, PE, PP).  Fails if a type has fewer candidates than asked for."""
    r_pos, r_con, r_beta, _ = _streams(seed)
    nx, ny, nz = block
    Xb = grid_vertices(nx, ny, nz, a)
    tets = kuhn_tets(nx, ny, nz)
    dm_inv, vol = _random_rest_shapes(r_pos, Xb, tets)
    nb = Xb.shape[0]
    ztop = nz * a
    betas = r_beta.uniform(0, 2 * np.pi, n_sheets)
    spacing = 1.0 / sheet_cells
    reach = spacing if reach is None else reach
    top_k = nz
    layers = [(Xb, 0, face_triangles(nx, ny, top_k), face_edges(nx, ny, top_k),
               np.unique(face_triangles(nx, ny, top_k)))]
    tri_all, dm2_all, area_all, hinge_all, hstiff_all, Xs = [], [], [], [], [], []
    off = nb

    def gap(j, xy):
        w = _tri_wave(4.0 * (xy[:, 0] * np.cos(betas[j]) + xy[:, 1] * np.sin(betas[j])))
        return np.sqrt(10.0 ** (-5.0 + 2.0 * w))

    for k in range(n_sheets):
        uv, xy, tris, hinges = sheet(sheet_cells, np.deg2rad(7.5 + 15.0 * k))
        # nested fields evaluated at this sheet's own world (x, y)
        z = ztop + sum(gap(j, xy) for j in range(k + 1))
        X = np.concatenate([xy, z[:, None]], 1)
        Xs.append(X)
        Dm = np.stack([uv[tris[:, 1]] - uv[tris[:, 0]], uv[tris[:, 2]] - uv[tris[:, 0]]], 2)
        dm2_all.append(np.linalg.inv(Dm))
        area_all.append(0.5 * np.abs(np.linalg.det(Dm)))
        tri_all.append(tris + off)
        e2 = ((uv[hinges[:, 1]] - uv[hinges[:, 0]]) ** 2).sum(1)
        u1, u2 = uv[hinges[:, 1]] - uv[hinges[:, 0]], uv[hinges[:, 2]] - uv[hinges[:, 0]]
        u3 = uv[hinges[:, 3]] - uv[hinges[:, 0]]
        A12 = 0.5 * (np.abs(u1[:, 0] * u2[:, 1] - u1[:, 1] * u2[:, 0]) +
                     np.abs(u1[:, 0] * u3[:, 1] - u1[:, 1] * u3[:, 0]))
        hinge_all.append(hinges + off)
        hstiff_all.append(k_b * 3.0 * e2 / A12)
        edges = np.unique(np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), 1), axis=0)
        layers.append((X, off, tris, edges, np.arange(X.shape[0])))
        off += X.shape[0]
    pool, pdist = _proximity(layers, dhat, reach, cell=max(reach, spacing))
    ctype, cidx, dsel = [], [], []
    for t, want in zip((PT, EE, PE, PP), counts):
        if len(pool[t]) < want:
            raise RuntimeError(f"{name}: only {len(pool[t])} candidates of type {t} for {want} stencils")
        pick = np.sort(r_con.choice(len(pool[t]), want, replace=False))
        cidx.append(pool[t][pick])
        dsel.append(pdist[t][pick])
        ctype.append(np.full(want, t))
    X0 = np.concatenate([Xb] + Xs)
    n = X0.shape[0]
    tri_idx = np.concatenate(tri_all)
    tri_area = np.concatenate(area_all)
    mass = _lumped_mass(n, tets, vol, rho)
    np.add.at(mass, tri_idx.ravel(), np.repeat(rho * thickness * tri_area / 3.0, 3))
    mu, lam = lame(E, nu)
    hidx = np.concatenate(hinge_all)
    p = _pack(n, X0, np.zeros((0, 3)), mass, X0 + h * h * GRAVITY, tets, dm_inv, vol,
              np.concatenate(ctype), np.concatenate(cidx), mu=mu, lam=lam, h=h, kappa=kappa, dhat=dhat,
              rho=rho, name=name)
    p.update(tri_idx=np.ascontiguousarray(tri_idx, dtype=np.int32),
             tri_dm_inv=np.ascontiguousarray(np.concatenate(dm2_all)),
             tri_area=np.ascontiguousarray(tri_area),
             mu_c=E_c / (2.0 * (1.0 + nu_c)), lam_c=E_c * nu_c / (1.0 - nu_c * nu_c), thickness=thickness,
             hinge_idx=np.ascontiguousarray(hidx, dtype=np.int32),
             hinge_rest=np.ascontiguousarray(np.stack([np.zeros(len(hidx)), np.concatenate(hstiff_all)], 1)),
             contact_d=np.concatenate(dsel),
             pool_sizes={int(t): int(len(pool[t])) for t in pool})
    return p


def small_cloth(seed=31, counts=(250, 250, 100, 40)):
    """A few-thousand-stencil version of the heterogeneous workload: a 6x6x2
    block under two 14x14 sheets."""
    return c3_cloth(seed=seed, block=(6, 6, 2), a=1.0 / 6, sheet_cells=14, n_sheets=2, counts=counts,
                    name="cloth_small")


# --------------------------------------------------------------------------
# Affine bodies mixed with free vertices
# --------------------------------------------------------------------------

def affine_block(seed=41, nx=5, ny=4, nz=3, n_pt=120, n_ee=120, n_pp=40, n_pt1=60, n_pp2=30, n_ee2=30,
                 n_fixed_pt=20, k_orth=1e5, body_mass=1.0, dhi=1e-3, **kw):
    """A free Kuhn block between two affine bodies (p = A r + t per body
    vertex), with contact stencils of every parameterisation mix:

    * body 0 under the block: n_pt points below bottom triangles (PT: body
      point, free triangle) and n_ee edges below bottom edges (EE: free edge,
      body edge), placed like the fixed collider of ``block_problem``;
    * body 1 above the block: n_pt1 points above top triangles (PT), n_pp
      points above top vertices (PP: free point, body point);
    * body 0 against body 1: n_pp2 PP and n_ee2 EE stencils (two bodies);
    * n_fixed_pt ordinary PT stencils (fixed point, free bottom triangle).

    Squared distances U(1e-4, dhi).  Each body's A starts as a seeded small
    perturbation of the identity (rest positions chosen so the vertices sit
    where placed), t = 0; its mass matrix is M4 = sum_v m_v w_v w_v^T,
    w = (r, 1), with the body's mass spread evenly over its vertices; the
    inertial target moves t by h^2 g.  The degree-of-freedom vector is
    X0 = [free x0; a_1, a_2, a_3, t of each body]."""
    r_pos, r_con, r_body, _ = _streams(seed)
    p = block_problem(nx, ny, nz, 1.0 / max(nx, ny, nz), n_pt + n_fixed_pt, n_ee, seed, dhi=dhi, **kw)
    X = p["x0"]
    n = p["n_free"]
    a = p["spacing"]
    ztop = nz * a
    ct, ci, xf = p["ctype"], p["cidx"].copy(), p["x_fixed"]
    # the collider features of the first n_pt PT and of every EE become body-0 vertices
    pt_rows = np.flatnonzero(ct == PT)
    ee_rows = np.flatnonzero(ct == EE)
    to_body = np.concatenate([pt_rows[:n_pt], ee_rows])
    keep = np.setdiff1d(np.arange(len(ct)), to_body)
    body_pts, body_of = [], []
    bct, bci = [], []

    def add_vertex(x, b):
        body_pts.append(np.asarray(x, np.float64))
        body_of.append(b)
        return len(body_pts) - 1

    for s in to_body:
        ids = ci[s].copy()
        for j in range(4):
            v = ids[j]
            if v >= n:  # a collider vertex: move it to body 0
                ids[j] = -2 - add_vertex(xf[v - n], 0)
        bct.append(ct[s])
        bci.append(ids)
    # ordinary contacts keep their own fixed points (renumbered compactly)
    fx_old = sorted({int(v) for s in keep for v in ci[s] if v >= n})
    remap = {v: n + i for i, v in enumerate(fx_old)}
    ct_o = ct[keep].astype(np.int32)
    ci_o = np.array([[remap.get(int(v), int(v)) for v in ci[s]] for s in keep], np.int32).reshape(-1, 4)
    x_fixed = xf[np.array(fx_old, np.int64) - n] if fx_old else np.zeros((0, 3))
    # body 1 above the top face
    tris = face_triangles(nx, ny, nz)
    verts_top = np.flatnonzero(np.abs(X[:, 2] - ztop) < 1e-12)
    d = r_con.uniform(1e-4, dhi, size=n_pt1)
    t = tris[r_con.integers(0, tris.shape[0], size=n_pt1)]
    for s in range(n_pt1):
        c = X[t[s]].mean(axis=0) + np.array([0.0, 0.0, np.sqrt(d[s])])
        bct.append(PT)
        bci.append(np.array([-2 - add_vertex(c, 1), t[s][0], t[s][1], t[s][2]]))
    d = r_con.uniform(1e-4, dhi, size=n_pp)
    vv = verts_top[r_con.integers(0, verts_top.size, size=n_pp)]
    for s in range(n_pp):
        bct.append(PP)
        bci.append(np.array([vv[s], -2 - add_vertex(X[vv[s]] + [0.0, 0.0, np.sqrt(d[s])], 1), -1, -1]))
    # body 0 against body 1: PP next to body-0 points, EE crossing under body-0 edges
    b0 = [k for k in range(len(body_pts)) if body_of[k] == 0]
    d = r_con.uniform(1e-4, dhi, size=n_pp2)
    for s in range(n_pp2):
        k0 = b0[r_con.integers(0, len(b0))]
        ang = r_con.uniform(0.0, 2 * np.pi)
        off = np.sqrt(d[s]) * np.array([np.cos(ang), np.sin(ang), 0.0])
        bct.append(PP)
        bci.append(np.array([-2 - k0, -2 - add_vertex(body_pts[k0] + off, 1), -1, -1]))
    ee_body = [s for s in range(len(bct)) if bct[s] == EE]
    d = r_con.uniform(1e-4, dhi, size=n_ee2)
    for s in range(n_ee2):
        src = bci[ee_body[r_con.integers(0, len(ee_body))]]
        k0, k1 = -2 - src[2], -2 - src[3]  # the body-0 edge of a free/body EE stencil
        q0, q1 = body_pts[k0], body_pts[k1]
        mid = 0.5 * (q0 + q1) - np.array([0.0, 0.0, np.sqrt(d[s])])
        dirn = q1 - q0
        perp = np.array([-dirn[1], dirn[0], 0.0]) / np.linalg.norm(dirn[:2])
        e0 = add_vertex(mid - 0.5 * a * perp, 1)
        e1 = add_vertex(mid + 0.5 * a * perp, 1)
        bct.append(EE)
        bci.append(np.array([-2 - k0, -2 - k1, -2 - e0, -2 - e1]))
    body_pts = np.array(body_pts)
    body_of = np.array(body_of, np.int64)
    nfix = x_fixed.shape[0]
    bci = np.array(bci, np.int64)
    bci = np.where(bci <= -2, n + nfix + (-2 - bci), bci).astype(np.int32)
    # body degrees of freedom: A = I + small seeded perturbation, t = 0; rest r = A^-1 p
    nb = 2
    q0 = np.zeros((nb, 4, 3))
    rest = np.zeros_like(body_pts)
    M4 = np.zeros((nb, 4, 4))
    for b in range(nb):
        A = np.eye(3) + r_body.normal(0.0, 1e-3, (3, 3))
        q0[b, :3] = A.T  # rows a_j = columns of A
        sel = np.flatnonzero(body_of == b)
        rest[sel] = np.linalg.solve(A, body_pts[sel].T).T
        w = np.concatenate([rest[sel], np.ones((sel.size, 1))], 1)
        M4[b] = (body_mass / sel.size) * (w.T @ w)
    qt = q0.copy()
    qt[:, 3] += p["h"] ** 2 * GRAVITY
    p.update(ctype=ct_o, cidx=ci_o, x_fixed=x_fixed, n_bodies=nb, body_q0=q0, body_qt=qt, body_M4=M4,
             body_k=np.full(nb, k_orth), abd_body=body_of, abd_rest=rest,
             bctype=np.array(bct, np.int32), bcidx=bci,
             X0=np.concatenate([X, q0.reshape(-1, 3)]), name=f"affine{nx}x{ny}x{nz}")
    if p.get("ee_eps") is not None:  # near-parallel collider edges (ee_angle): thresholds follow their stencils
        eps = p["ee_eps"]
        p["ee_eps"] = eps[keep]
        p["bee_eps"] = np.concatenate([eps[to_body], np.zeros(len(bct) - len(to_body))])
    return p


# --------------------------------------------------------------------------
# Time stepping with contact: a block dropped onto a fixed ground
# --------------------------------------------------------------------------

def boundary_surface(tets):
    """Boundary triangles of a tet mesh (faces of exactly one tet), their
    edges and vertices."""
    tets = np.asarray(tets, np.int64)
    faces = np.concatenate([tets[:, [1, 2, 3]], tets[:, [0, 3, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 1]]])
    key = np.sort(faces, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    tris = faces[cnt[inv.ravel()] == 1]
    e = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), axis=1)
    edges = np.unique(e, axis=0)
    return tris, edges, np.unique(tris)


def ground_grid(cells, size, angle, center, z=0.0):
    """A flat square of cells x cells (each split along a diagonal), side
    `size`, rotated by `angle` about the vertical through `center`: vertices,
    triangles, edges (local ids)."""
    t = np.linspace(-0.5 * size, 0.5 * size, cells + 1)
    gx, gy = np.meshgrid(t, t, indexing="xy")
    c, s_ = np.cos(angle), np.sin(angle)
    V = np.stack([center[0] + c * gx.ravel() - s_ * gy.ravel(), center[1] + s_ * gx.ravel() + c * gy.ravel(),
                  np.full(gx.size, z)], 1)
    vid = lambda i, j: j * (cells + 1) + i
    tris, edges = [], set()
    for j in range(cells):
        for i in range(cells):
            a, b, cc, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris += [(a, b, cc), (a, cc, d)]
            for u, w in ((a, b), (b, cc), (cc, a), (cc, d), (d, a)):
                edges.add((min(u, w), max(u, w)))
    return V, np.array(tris, np.int64), np.array(sorted(edges), np.int64)


def drop_scene(seed=51, nx=3, ny=3, nz=2, a=0.1, gap=0.012, v0=-1.0, ground_cells=5, ground_size=0.6,
               ground_angle=0.37, h=1e-2, E=1e5, nu=0.4, rho=1000.0, kappa=1e3, dhat=1e-4, jitter=1e-3):
    """A free Kuhn block (rest shape = its initial shape) a gap above a fixed,
    rotated ground grid, falling at v0 (m/s, vertical): the time-stepping
    scene.  The block's vertices are jittered by N(0, jitter^2 a^2) (so no
    edge pair is exactly parallel) before the rest shapes are taken.  The
    collision surface: the block's boundary triangles, edges and vertices, and
    the ground's (fixed ids n_free + k).  Keys: the problem (no contacts),
    `v0` (n, 3), surface arrays `surf_points`, `surf_edges`, `surf_tris`,
    `surf_len2` (squared rest edge lengths), `cell` (grid cell size)."""
    rng = np.random.default_rng(seed)
    X = grid_vertices(nx, ny, nz, a, origin=(0.0, 0.0, gap))
    X = X + rng.normal(0.0, jitter * a, X.shape)
    X[:, 2] = np.maximum(X[:, 2], gap * 0.5)
    tets = kuhn_tets(nx, ny, nz)
    Ds = _edge_matrix(X, tets)
    dm_inv, vol = np.linalg.inv(Ds), np.abs(np.linalg.det(Ds)) / 6.0
    n = X.shape[0]
    mass = _lumped_mass(n, tets, vol, rho)
    center = (0.5 * nx * a + 0.013, 0.5 * ny * a - 0.021)
    G, gt, ge = ground_grid(ground_cells, ground_size, ground_angle, center)
    mu, lam = lame(E, nu)
    v = np.zeros((n, 3))
    v[:, 2] = v0
    x_tilde = X + h * v + h * h * GRAVITY
    p = _pack(n, X, G, mass, x_tilde, tets, dm_inv, vol, np.zeros(0, np.int32), np.zeros((0, 4), np.int32),
              mu=mu, lam=lam, h=h, kappa=kappa, dhat=dhat, rho=rho, name=f"drop{nx}x{ny}x{nz}", spacing=a)
    bt, be, bp = boundary_surface(tets)
    tris = np.concatenate([bt, gt + n])
    edges = np.concatenate([be, ge + n])
    points = np.concatenate([bp, np.arange(G.shape[0]) + n])
    xa = np.concatenate([X, G])
    len2 = ((xa[edges[:, 1]] - xa[edges[:, 0]]) ** 2).sum(1)
    p.update(v0=v, surf_points=points.astype(np.int32), surf_edges=edges.astype(np.int32),
             surf_tris=tris.astype(np.int32), surf_len2=len2, cell=max(a, ground_size / ground_cells) * 1.01)
    return p


def drop_body_scene(seed=52, nx=3, ny=3, nz=2, a=0.1, bc=2, ab=0.1, gap=0.012, v0=-1.0, ground_cells=5,
                    ground_size=0.6, ground_angle=0.37, h=1e-2, E=1e5, nu=0.4, rho=1000.0, kappa=1e3, dhat=1e-4,
                    k_orth=1e5, jitter=1e-3):
    """The drop scene with an affine cube stacked on the free block: the cube
    (bc^3 cells of side ab, its boundary vertices as body vertices with rest
    positions where they start, A = I, t = 0) a gap above the block's top, the
    block a gap above the ground, both falling at v0.  Body mass rho (bc ab)^3
    spread evenly over its vertices (M4 = sum m w w^T, w = (r, 1)),
    orthogonality stiffness k_orth.  The collision surface adds the cube's
    boundary triangles, edges and points (body vertex ids n_free + n_fixed + k).
    Rows: X0 = [free x0; a_1, a_2, a_3, t], V0 likewise."""
    p = drop_scene(seed=seed, nx=nx, ny=ny, nz=nz, a=a, gap=gap, v0=v0, ground_cells=ground_cells,
                   ground_size=ground_size, ground_angle=ground_angle, h=h, E=E, nu=nu, rho=rho, kappa=kappa,
                   dhat=dhat, jitter=jitter)
    rng = np.random.default_rng(seed + 1)
    n, nfix = p["n_free"], p["x_fixed"].shape[0]
    top = p["x0"][:, 2].max()
    # the cube, centred over the block, rotated a little about z (no parallel edges with the block)
    C = grid_vertices(bc, bc, bc, ab)
    C = C - C.mean(axis=0)
    th = 0.21
    R = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    C = C @ R.T + np.array([0.5 * nx * a, 0.5 * ny * a, top + gap + 0.5 * bc * ab])
    C = C + rng.normal(0.0, jitter * ab, C.shape)
    ctets = kuhn_tets(bc, bc, bc)
    bt, be, bp = boundary_surface(ctets)
    local = -np.ones(C.shape[0], np.int64)
    local[bp] = np.arange(bp.size)
    rest = C[bp]
    nbv = rest.shape[0]
    base = n + nfix
    m = rho * (bc * ab) ** 3 / nbv
    w = np.concatenate([rest, np.ones((nbv, 1))], 1)
    M4 = (m * (w.T @ w))[None]
    q0 = np.zeros((1, 4, 3))
    q0[0, :3] = np.eye(3)
    v_rows = np.zeros((1, 4, 3))
    v_rows[0, 3, 2] = v0
    tris = np.concatenate([p["surf_tris"], local[bt] + base])
    edges = np.concatenate([p["surf_edges"], local[be] + base])
    points = np.concatenate([p["surf_points"], np.arange(nbv) + base])
    xa = np.concatenate([p["x0"], p["x_fixed"], rest])
    len2 = ((xa[edges[:, 1]] - xa[edges[:, 0]]) ** 2).sum(1)
    qt = q0.copy()
    p.update(n_bodies=1, body_q0=q0, body_qt=qt, body_M4=M4, body_k=np.array([k_orth]),
             abd_body=np.zeros(nbv, np.int64), abd_rest=rest, bctype=np.zeros(0, np.int32),
             bcidx=np.zeros((0, 4), np.int32), X0=np.concatenate([p["x0"], q0.reshape(-1, 3)]),
             V0=np.concatenate([p["v0"], v_rows.reshape(-1, 3)]), surf_points=points.astype(np.int32),
             surf_edges=edges.astype(np.int32), surf_tris=tris.astype(np.int32), surf_len2=len2,
             name=f"dropbody{nx}x{ny}x{nz}")
    return p
