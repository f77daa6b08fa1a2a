"""Seeded synthetic scenes: meshes, materials, obstacles and contact parameters.

This module only draws inputs.  It holds none of the method's arithmetic
(no assembly, no solve, no contact selection), so both the CPU oracle and the
GPU library consume exactly the same arrays.  Every quantity is a plain numpy
array or Python scalar in SI units.

Scene recipe (the paper's own scene -- "a simple contact scenario" of the
results section -- is not published, so these stand in for it):

* the body is a box of hexahedral cells on a node grid of spacing ``s``, each
  cell split into 6 tetrahedra around its main diagonal (Kuhn split);
* interior nodes are jittered uniformly by up to ``jitter * s`` per axis, and
  nodes on a face only move inside that face, so the box volume is exact;
* linear-elastic material (Young's modulus per tetrahedron, Poisson ratio),
  lumped density, Rayleigh damping coefficients and time step ``h``;
* a kinematic rigid obstacle (tilted plane or sphere) translating at constant
  velocity; its pose at ``t`` and ``t + h`` is derived from ``c0 + vel * t``;
* contact candidates are surface nodes that are not clamped; every step keeps
  the ``n_contacts`` candidates with the smallest signed distance.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

CONFIGS = ("tiny", "medium", "precision", "serving", "stress", "stacked", "stacked_small")


def box_grid(nx: int, ny: int, nz: int, s: float, jitter: float, rng: np.random.Generator):
    """Node positions and Kuhn-split tetrahedra of an ``nx*ny*nz`` node grid.

    Node id = i + nx * (j + ny * k).  Returns (nodes[N,3] f64, tets[T,4] i32,
    ijk[N,3] i32 grid indices).
    """
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ijk = np.zeros((nx * ny * nz, 3), dtype=np.int32)
    ids = (I + nx * (J + ny * K)).ravel()
    ijk[ids, 0] = I.ravel()
    ijk[ids, 1] = J.ravel()
    ijk[ids, 2] = K.ravel()
    dims = np.array([nx, ny, nz])
    nodes = ijk.astype(np.float64) * s
    if jitter > 0:
        movable = (ijk > 0) & (ijk < dims[None, :] - 1)
        shift = rng.uniform(-jitter * s, jitter * s, size=nodes.shape)
        nodes = nodes + np.where(movable, shift, 0.0)

    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()

    def vid(di, dj, dk):
        return (ci + di) + nx * ((cj + dj) + ny * (ck + dk))

    unit = np.eye(3, dtype=np.int64)
    tets = []
    for perm in itertools.permutations(range(3)):
        a, b, _ = perm
        o = np.zeros(3, dtype=np.int64)
        p1 = unit[a]
        p2 = unit[a] + unit[b]
        p3 = np.ones(3, dtype=np.int64)
        v = [vid(*o), vid(*p1), vid(*p2), vid(*p3)]
        # orientation of the undeformed Kuhn tetrahedron: sign of the permutation
        inv = sum(1 for x in range(3) for y in range(x + 1, 3) if perm[x] > perm[y])
        if inv % 2 == 1:
            v[2], v[3] = v[3], v[2]
        tets.append(np.stack(v, axis=1))
    tets = np.concatenate(tets, axis=0).astype(np.int32)
    return nodes, tets, ijk


def stacked_grids(nx: int, ny: int, nz_low: int, nz_up: int, s: float, jitter: float, rng: np.random.Generator):
    """Two bodies stacked along z, each a jittered Kuhn-split node grid.

    The lower body occupies z in [0, (nz_low - 1) s]; the upper body starts at
    its top face.  The two interface layers hold separate nodes at identical
    positions (the upper body's bottom layer copies the lower body's top layer,
    whose jitter is in-face only), so the two meshes touch without sharing a
    node and A is block diagonal.  Returns (nodes, tets, ijk, body, pairs):
    ``body`` is 0 for the lower and 1 for the upper body; ``pairs[i]`` =
    (lower node, upper node) at the same interface position, in grid order.
    """
    lo_nodes, lo_tets, lo_ijk = box_grid(nx, ny, nz_low, s, jitter, rng)
    up_nodes, up_tets, up_ijk = box_grid(nx, ny, nz_up, s, jitter, rng)
    up_nodes = up_nodes + np.array([0.0, 0.0, (nz_low - 1) * s])
    top = np.nonzero(lo_ijk[:, 2] == nz_low - 1)[0]
    bottom = np.nonzero(up_ijk[:, 2] == 0)[0]   # same (i, j) order as ``top``
    up_nodes[bottom] = lo_nodes[top]
    nl = len(lo_nodes)
    nodes = np.concatenate([lo_nodes, up_nodes])
    tets = np.concatenate([lo_tets, up_tets + nl]).astype(np.int32)
    up_ijk = up_ijk + np.array([0, 0, nz_low - 1], dtype=np.int32)
    ijk = np.concatenate([lo_ijk, up_ijk])
    body = np.concatenate([np.zeros(nl, dtype=np.int32), np.ones(len(up_nodes), dtype=np.int32)])
    pairs = np.stack([top, bottom + nl], axis=1).astype(np.int32)
    return nodes, tets, ijk, body, pairs


def interface_edge_points(nx: int, ny: int, pairs: np.ndarray, count: int, rng: np.random.Generator):
    """``count`` points on edges of the interface triangulation (grid edges
    along i and j and the cell diagonals of the Kuhn split), each given on
    both bodies: slots (upper a, upper b, lower a, lower b) with weights
    (w, 1 - w, -w, -(1 - w)), w ~ U[0.1, 0.9].  A point pairs the upper
    body's position with the lower body's, x_1 - x_2 (the upper body is body
    1).  Edges are drawn without replacement while they last, then again."""
    edges = []
    for j in range(ny):
        for i in range(nx):
            a = i + nx * j
            if i + 1 < nx:
                edges.append((a, a + 1))
            if j + 1 < ny:
                edges.append((a, a + nx))
            if i + 1 < nx and j + 1 < ny:
                edges.append((a, a + 1 + nx))
    edges = np.array(edges, dtype=np.int64)
    picks = []
    while len(picks) < count:
        picks.extend(rng.permutation(len(edges))[: count - len(picks)].tolist())
    e = edges[np.array(picks)]
    w = rng.uniform(0.1, 0.9, size=count)
    ids = np.stack([pairs[e[:, 0], 1], pairs[e[:, 1], 1], pairs[e[:, 0], 0], pairs[e[:, 1], 0]], axis=1)
    wts = np.stack([w, 1.0 - w, -w, -(1.0 - w)], axis=1)
    return np.ascontiguousarray(ids.astype(np.int32)), np.ascontiguousarray(wts)


def _signed_volumes(nodes, tets):
    x0 = nodes[tets[:, 0]]
    e = np.stack([nodes[tets[:, 1]] - x0, nodes[tets[:, 2]] - x0, nodes[tets[:, 3]] - x0], axis=2)
    return np.linalg.det(e) / 6.0


def obstacle_pose(obs: dict, t: float) -> np.ndarray:
    """Reference point of the obstacle at time t (sphere centre or plane point)."""
    return np.asarray(obs["c0"], dtype=np.float64) + np.asarray(obs["vel"], dtype=np.float64) * t


def make_scene(config: str, seed: int = 0) -> dict:
    """Draw one scene.  ``config`` is one of CONFIGS."""
    rng = np.random.default_rng(seed)
    s = 0.01
    sc: dict = dict(config=config, seed=seed, rho=1.0e3, alpha=0.1, beta=0.1, h=0.01, nu=0.45,
                    n_newton=5, max_sweeps=200, tol=1e-10, j_inner=8)
    if config == "tiny":
        nx, ny, nz = 4, 4, 16
        nodes, tets, ijk = box_grid(nx, ny, nz, s, 0.0, rng)
        E = np.full(len(tets), 5.0e3)
        fixed = (ijk[:, 2] == 0)
        cand = np.nonzero(ijk[:, 2] == nz - 1)[0]
        theta = math.radians(rng.uniform(0.0, 15.0))
        zmax = (nz - 1) * s
        centre = np.array([(nx - 1) * s / 2, (ny - 1) * s / 2, zmax])
        obs = dict(kind="plane", normal=np.array([0.0, math.sin(theta), -math.cos(theta)]),
                   c0=centre, vel=np.array([0.0, 0.0, -0.05]), radius=0.0)
        mu = np.full(len(cand), 0.3)
        sc.update(gravity=np.array([0.0, 0.0, 9.81]), n_contacts=16, n_steps=1, theta=theta)
    elif config in ("medium", "precision"):
        if config == "medium":
            nx, ny, nz = 15, 15, 14
        else:
            nx, ny, nz = 28, 27, 27
        nodes, tets, ijk = box_grid(nx, ny, nz, s, 0.2, rng)
        if config == "medium":
            E = np.full(len(tets), 5.0e3)
        else:
            E = np.exp(rng.uniform(math.log(1e3), math.log(1e5), size=len(tets)))
        dims = np.array([nx, ny, nz])
        fixed = (ijk[:, 2] == nz - 1)
        surface = np.any((ijk == 0) | (ijk == dims[None, :] - 1), axis=1)
        cand = np.nonzero(surface & ~fixed)[0]
        width = (nx - 1) * s
        R = 0.6 * width
        off = rng.uniform(-0.1, 0.1, size=2) * width
        c0 = np.array([(nx - 1) * s / 2 + off[0], (ny - 1) * s / 2 + off[1], -R + 0.1 * s])
        obs = dict(kind="sphere", normal=np.zeros(3), c0=c0, vel=np.array([0.0, 0.0, 0.05]), radius=R)
        if config == "medium":
            mu = rng.uniform(0.2, 0.6, size=len(cand))
            sc.update(n_contacts=200, n_steps=10)
        else:
            mu = np.full(len(cand), 0.4)
            sc.update(n_contacts=1000, n_steps=20)
        sc.update(gravity=np.array([0.0, 0.0, -9.81]))
    elif config == "serving":
        # one scene of the serving mix: node count log-uniform in [500, 8000],
        # 10-500 contacts, a tilted plane or a sphere rising into the bottom
        # face, mu ~ U[0.1, 0.6] per candidate node
        target = math.exp(rng.uniform(math.log(500.0), math.log(8000.0)))
        nxy = max(4, int(round(target ** (1.0 / 3.0) * rng.uniform(0.85, 1.15))))
        nz = max(4, int(round(target / (nxy * nxy))))
        nx, ny = nxy, nxy
        nodes, tets, ijk = box_grid(nx, ny, nz, s, 0.2, rng)
        E = np.full(len(tets), 5.0e3)
        dims = np.array([nx, ny, nz])
        fixed = (ijk[:, 2] == nz - 1)
        surface = np.any((ijk == 0) | (ijk == dims[None, :] - 1), axis=1)
        cand = np.nonzero(surface & ~fixed)[0]
        width = (nx - 1) * s
        if rng.uniform() < 0.5:
            theta = math.radians(rng.uniform(0.0, 15.0))
            c0 = np.array([(nx - 1) * s / 2, (ny - 1) * s / 2, -0.1 * s])
            obs = dict(kind="plane", normal=np.array([0.0, math.sin(theta), math.cos(theta)]), c0=c0,
                       vel=np.array([0.0, 0.0, 0.05]), radius=0.0)
        else:
            R = 0.6 * width
            off = rng.uniform(-0.1, 0.1, size=2) * width
            c0 = np.array([(nx - 1) * s / 2 + off[0], (ny - 1) * s / 2 + off[1], -R + 0.1 * s])
            obs = dict(kind="sphere", normal=np.zeros(3), c0=c0, vel=np.array([0.0, 0.0, 0.05]), radius=R)
        mu = rng.uniform(0.1, 0.6, size=len(cand))
        n_c = int(min(len(cand), rng.integers(10, 501)))
        sc.update(gravity=np.array([0.0, 0.0, -9.81]), n_contacts=n_c, n_steps=20)
    elif config == "stress":
        # the stress shape on one body: 30x30x28 jittered grid (75 600 DOF),
        # E = 1e4, 3000 contacts (m = 9000) among the surface nodes, mu = 0.5,
        # a sphere pressed into the bottom face and sliding along x at
        # 0.5 m/s; 5 steps x 8 Newton iterations.  (Two stacked bodies with
        # barycentric interface points need a two-body mapping H, which this
        # nodal-contact library does not have.)
        nx, ny, nz = 30, 30, 28
        nodes, tets, ijk = box_grid(nx, ny, nz, s, 0.2, rng)
        E = np.full(len(tets), 1.0e4)
        dims = np.array([nx, ny, nz])
        fixed = (ijk[:, 2] == nz - 1)
        surface = np.any((ijk == 0) | (ijk == dims[None, :] - 1), axis=1)
        cand = np.nonzero(surface & ~fixed)[0]
        width = (nx - 1) * s
        R = 0.6 * width
        off = rng.uniform(-0.1, 0.1, size=2) * width
        c0 = np.array([(nx - 1) * s / 2 + off[0], (ny - 1) * s / 2 + off[1], -R + 0.2 * s])
        obs = dict(kind="sphere", normal=np.zeros(3), c0=c0, vel=np.array([0.5, 0.0, 0.1]), radius=R)
        mu = np.full(len(cand), 0.5)
        sc.update(gravity=np.array([0.0, 0.0, -9.81]), n_contacts=3000, n_steps=5, n_newton=8)
    elif config in ("stacked", "stacked_small"):
        # two deformable bodies stacked along z (the stress configuration:
        # 30x30 node layers, 14 for each body, 75 600 DOF), the lower one
        # clamped at its bottom; 2400 interface points x_1 - x_2 on the
        # interface edges (upper body = body 1), normal +z (the lower body's
        # top surface); a sphere pressed into the upper body's top face and
        # sliding along x at 0.5 m/s; 600 sphere contacts among the top-face
        # nodes; 3000 contacts in all (m = 9000), mu = 0.5, 8 Newton
        # iterations.  stacked_small: 8x8 layers, 5 + 5, 120 points + 16.
        if config == "stacked":
            nx, ny, nzl, nzu, npair, nsph = 30, 30, 14, 14, 2400, 600
        else:
            nx, ny, nzl, nzu, npair, nsph = 8, 8, 5, 5, 120, 16
        nodes, tets, ijk, body, pairs = stacked_grids(nx, ny, nzl, nzu, s, 0.2, rng)
        nz = nzl + nzu
        E = np.full(len(tets), 1.0e4)
        fixed = (ijk[:, 2] == 0) & (body == 0)
        ztop = nzl + nzu - 2
        cand = np.nonzero((ijk[:, 2] == ztop) & (body == 1))[0]
        ids, w = interface_edge_points(nx, ny, pairs, npair, rng)
        width = (nx - 1) * s
        R = 0.6 * width
        off = rng.uniform(-0.1, 0.1, size=2) * width
        c0 = np.array([(nx - 1) * s / 2 + off[0], (ny - 1) * s / 2 + off[1], ztop * s + R - 0.2 * s])
        obs = dict(kind="sphere", normal=np.zeros(3), c0=c0, vel=np.array([0.5, 0.0, -0.1]), radius=R)
        mu = np.full(len(cand), 0.5)
        sc.update(gravity=np.array([0.0, 0.0, -9.81]), n_contacts=npair + nsph, n_steps=5, n_newton=8,
                  body=body, pairs=dict(ids=ids, w=w, normals=np.tile([0.0, 0.0, 1.0], (npair, 1)),
                                        mu=np.full(npair, 0.5)))
    else:
        raise ValueError(f"unknown config {config!r}")

    vol = _signed_volumes(nodes, tets)
    if not np.all(vol > 0):
        raise RuntimeError("generator produced an inverted tetrahedron")
    sc.update(nodes=np.ascontiguousarray(nodes, dtype=np.float64),
              tets=np.ascontiguousarray(tets, dtype=np.int32),
              E=np.ascontiguousarray(E, dtype=np.float64),
              nu_e=np.full(len(tets), sc["nu"]),
              fixed=np.ascontiguousarray(fixed.astype(np.uint8)),
              candidates=np.ascontiguousarray(cand.astype(np.int32)),
              cand_mu=np.ascontiguousarray(mu, dtype=np.float64),
              obstacle=obs, grid=(nx, ny, nz), spacing=s)
    return sc


# ---------------------------------------------------------------------------
# Inputs for the per-call kernels (update_W, solve_contacts, GEMV): random
# numbers only, drawn here so both sides receive identical arrays.
# ---------------------------------------------------------------------------

def random_spd(m: int, rng: np.random.Generator, rank_boost: float = 1.0) -> np.ndarray:
    """Symmetric positive definite m x m matrix with a Delassus-like spectrum."""
    g = rng.standard_normal((m, m)) / math.sqrt(m)
    a = g @ g.T + rank_boost * np.eye(m)
    return np.ascontiguousarray(0.5 * (a + a.T))


def random_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """n random proper rotations, row-major [n, 3, 3]."""
    q, r = np.linalg.qr(rng.standard_normal((n, 3, 3)))
    q = q * np.sign(np.einsum("nii->ni", r))[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 2] *= -1.0
    return np.ascontiguousarray(q)


def random_contact_problem(n_c: int, rng: np.random.Generator, h: float = 0.01):
    """W (SPD), gap d, friction mu and a warm start for one PGS call."""
    m = 3 * n_c
    W = random_spd(m, rng) * 50.0
    d = rng.uniform(-1e-3, 5e-4, size=m)
    mu = rng.uniform(0.1, 0.6, size=n_c)
    lam0 = np.zeros(m)
    return W, d, mu, lam0
