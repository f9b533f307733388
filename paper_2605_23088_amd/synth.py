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

def _collider_contacts(rng, X, nx, ny, n_pt, n_ee, n_free, dlo=1e-4, dhi=1e-3):
    """PT and EE stencils between the bottom face (z = 0) of a grid block and a
    private fixed feature per stencil placed below it.

    PT: a uniformly chosen bottom triangle and a fixed point at
        centroid - sqrt(d) z, d ~ U(dlo, dhi) (d is a squared distance).
    EE: a uniformly chosen bottom edge and a fixed horizontal edge of length a,
        perpendicular to it, through midpoint - sqrt(d) z.
    Both are interior-type by construction.  Returns (ctype, cidx, x_fixed)."""
    tris = face_triangles(nx, ny, 0)
    edges = face_edges(nx, ny, 0)
    a = X[1, 0] - X[0, 0]
    fixed = []
    ctype, cidx = [], []
    if n_pt:
        t = tris[rng.integers(0, tris.shape[0], size=n_pt)]
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
                  kappa=1e4, dhat=1e-3, random_F=True, name="block"):
    """A Kuhn block [0, nx a] x [0, ny a] x [0, nz a] at its exact grid positions,
    with seeded per-tet rest shapes (so x0 carries random deformation gradients
    with singular values in [0.7, 1.4]) and n_pt + n_ee contact stencils against
    a fixed collider under the bottom face.  All block vertices are free."""
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
    ctype, cidx, x_fixed = _collider_contacts(r_con, X, nx, ny, n_pt, n_ee, n)
    mu, lam = lame(E, nu)
    x_tilde = X + h * h * GRAVITY
    return _pack(n, X, x_fixed, mass, x_tilde, tets, dm_inv, vol, ctype, cidx,
                 mu=mu, lam=lam, h=h, kappa=kappa, dhat=dhat, rho=rho, name=name,
                 grid=(nx, ny, nz), spacing=a)


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
              rho=1000.0, kappa=1e4, dhat=1e-3):
    """Differentiation-form workload: static equilibrium of a 48x48x29-cell block
    (400,896 tets, 72,030 vertices) under gravity, per-tet Young's modulus
    theta log-uniform in [5e4, 2e5], the 4 bottom-corner vertices fixed, and
    300k PT stencils against fixed points under the bottom face.  Also returns
    a seeded target x_tgt = x0 + N(0, 1e-3)."""
    r_pos, r_con, r_theta, r_tgt = _streams(seed)
    X = grid_vertices(nx, ny, nz, a)
    tets = kuhn_tets(nx, ny, nz)
    Ds = _edge_matrix(X, tets)
    dm_inv, vol = np.linalg.inv(Ds), np.abs(np.linalg.det(Ds)) / 6.0
    nv = X.shape[0]
    corners = np.array([grid_vid(nx, ny, i, j, 0) for i in (0, nx) for j in (0, ny)])
    is_fixed = np.zeros(nv, bool)
    is_fixed[corners] = True
    free = np.flatnonzero(~is_fixed)
    n_free = free.size
    new_id = np.empty(nv, np.int64)
    new_id[free] = np.arange(n_free)
    new_id[corners] = n_free + np.arange(4)
    # contacts (vertex ids in the original numbering, fixed partners after the 4 corners)
    ctype, cidx, x_part = _collider_contacts(r_con, X, nx, ny, n_pt, 0, nv)
    cidx = cidx.astype(np.int64)
    part = cidx[:, 0] - nv
    tri = new_id[cidx[:, 1:]]
    cidx = np.concatenate([(n_free + 4 + part)[:, None], tri], 1)
    theta = np.exp(r_theta.uniform(np.log(5e4), np.log(2e5), size=tets.shape[0]))
    mu1, lam1 = lame(1.0, nu)
    mass_all = _lumped_mass(nv, tets, vol, rho)
    x0 = X[free]
    x_tgt = x0 + r_tgt.normal(0.0, 1e-3, size=x0.shape)
    x_fixed = np.concatenate([X[corners], x_part])
    return _pack(n_free, x0, x_fixed, mass_all[free], np.zeros_like(x0), new_id[tets], dm_inv,
                 vol, ctype, cidx, mu_t=theta * mu1, lam_t=theta * lam1, theta=theta,
                 mu1=mu1, lam1=lam1, h=1.0, kappa=kappa, dhat=dhat, rho=rho, static=True,
                 x_tgt=x_tgt, name="C5", grid=(nx, ny, nz), spacing=a)


def small_block(seed=7, nx=5, ny=4, nz=3, n_pt=150, n_ee=150, **kw):
    """A few-hundred-tet version of the metric workload for fast parity runs."""
    return block_problem(nx, ny, nz, 1.0 / max(nx, ny, nz), n_pt, n_ee, seed,
                         name=f"block{nx}x{ny}x{nz}", **kw)
