"""Plain FP64 CPU oracle for the constraint-matrix hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  The GPU library never
calls it and shares no code with it.

Every routine follows the paper (Zeng & Courtecuisse, "An efficient implicit
constraint resolution scheme for interactive FE simulations", arXiv 2306.06946)
step by step, in the paper's order and notation, with numpy/scipy primitives
(dense or banded Cholesky, matmul) as the only building blocks.  All values are
IEEE binary64; nothing is blocked, fused or reordered beyond what a formula
states.  Citations name the section, equation, algorithm or table.

Readings where the paper is silent or ambiguous (each is restated in the design
notes of the repository):
  R1  corrective motion carries the factor h:  dv_cor = h A^-1 J^T lambda
      (Eq. 12, which gives the h^2 of Eq. 17/18);
  R2  PGS works on W~ = h^2 W (Eq. 18; Eq. 19 drops the h^2);
  R3  Coulomb's law is the isotropic circular cone |lambda_t| <= mu lambda_n
      (Eq. 9 is written per tangent);
  R4  the tangential gap is the relative tangential displacement over the step,
      T (p - p_start - u_obstacle) (Eq. 10 vanishes for closest points);
  R5  local solver per contact: separate / stick trial / slip fixed point on
      the cone boundary with a shifted (contractive) direction update
      (``local_solve``; Sec. "Constraint resolution" only names the laws);
  R6  Gauss-Seidel order is ascending contact id (= node id), one local solve
      per contact per sweep, no relaxation (Algorithm 1);
  R7  stop after a full sweep when |lam_i - lam_{i-1}|_2 / |lam_i|_2 <= tol
      (Algorithm 1); if |lam_i| = 0 stop iff the change is 0;
  R8  each Newton iteration solves for the TOTAL contact force in frame k,
      warm-started from C_k C_{k-1}^T lam_{k-1}; identical to the increment form
      of Eq. 31 / Algorithm 3 because C_k^T lam'_k = C_k^T lam_k - C_{k-1}^T lam_{k-1};
  R9  the gap right-hand side of Algorithm 3 is
      d_k = delta(p_{k-1}) - C_k (p_{k-1} - p_free);
  R10 fixed Newton count, no convergence test (Sec. "Results": 5 iterations);
  R11 tangent basis: e = unit axis of smallest |n_i| (lowest index on ties),
      t1 = normalize(e - (e.n) n), t2 = n x t1;
  R12 lumped mass rho V / 4 per node; B = alpha M + beta K (Rayleigh);
  R13 clamped DOFs: identity rows/columns of A and zero right-hand side;
  R14 internal force f_t = K (q - q_rest) + B v (linear elasticity, Eq. 4-5);
  R15 W_H is symmetrised once, W_H <- (W_H + W_H^T) / 2;
  R16 warm start across steps: a contact whose node was in contact at the end
      of the previous step starts from that node's world-frame force;
  R17 contacts = the K candidates with smallest signed distance at q_free
      (ties by node id), then ordered by node id;
  R18 directions updated before every local solve (the variant the results
      section proposes, "after the resolution of each constraint"): Gauss-
      Seidel on world-frame forces f; at contact a's turn its frame and gap
      are taken at its current proximity p_a = p_free,a + h^2 sum_b W_H,ab f_b
      and the local problem is R9 applied to that contact alone:
      d_a = delta(p_a) - W~_aa C_a f_a with W~_aa = h^2 C_a W_H,aa C_a^T; the
      stopping rule R7 is taken on f.  With a plane obstacle (constant frames,
      affine gap) this is exactly the PGS of one Newton iteration.
  R19 two deformable bodies: a pair contact is a point of body 1 against the
      same point of body 2, p = x_1 - x_2 = H q with H = [H_1, -H_2] (the
      nodes of body 2 carry negative weights; Eq. 6, 16-17), so its force acts
      as +f on body 1 and -f on body 2 (c_2 = -J_2^T lambda);
  R20 a pair's normal n is the unit normal of body 2's surface at the pair,
      given with the pair and fixed over the step; its gap is the normal
      separation n . p (0 for points that coincide at rest), its tangential
      gap T (p - p_start) (R4 without an obstacle motion), tangents by R11;
  R21 the contacts of a step with pairs are the pairs, in their given
      order, followed by the obstacle contacts of R17 (K = n_contacts - number
      of pairs); pairs warm-start from their own force of the previous step.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, reverse_cuthill_mckee

SEPARATE, STICK, SLIP = 0, 1, 2


# ---------------------------------------------------------------------------
# FE assembly: Sec. "Implicit time integration", Eq. (4)-(5)
# ---------------------------------------------------------------------------

def lame(E, nu):
    """Lame constants of isotropic linear elasticity."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def element_matrices(nodes, tets, E, nu):
    """Linear-tetrahedron stiffness K_e = V B^T D B (12x12 per element) and volume V.

    DOF order inside an element: (node a, axis i) -> 3a + i.  B is the 6x12
    strain-displacement matrix in Voigt order (xx, yy, zz, 2yz, 2xz, 2xy).
    """
    X = nodes[tets]                                   # [T,4,3]
    Dm = np.transpose(X[:, 1:, :] - X[:, :1, :], (0, 2, 1))   # columns x_a - x_0
    vol = np.linalg.det(Dm) / 6.0
    Dinv = np.linalg.inv(Dm)                          # row a-1 = grad of barycentric a
    grads = np.concatenate([-Dinv.sum(axis=1, keepdims=True), Dinv], axis=1)   # [T,4,3]
    T = len(tets)
    B = np.zeros((T, 6, 12))
    for a in range(4):
        bx, by, bz = grads[:, a, 0], grads[:, a, 1], grads[:, a, 2]
        c = 3 * a
        B[:, 0, c + 0] = bx
        B[:, 1, c + 1] = by
        B[:, 2, c + 2] = bz
        B[:, 3, c + 1] = bz
        B[:, 3, c + 2] = by
        B[:, 4, c + 0] = bz
        B[:, 4, c + 2] = bx
        B[:, 5, c + 0] = by
        B[:, 5, c + 1] = bx
    lam, mu = lame(np.asarray(E, dtype=np.float64), np.asarray(nu, dtype=np.float64))
    D = np.zeros((T, 6, 6))
    for i in range(3):
        for j in range(3):
            D[:, i, j] = lam
        D[:, i, i] = lam + 2.0 * mu
        D[:, 3 + i, 3 + i] = mu
    Ke = vol[:, None, None] * np.einsum("tki,tkl,tlj->tij", B, D, B)
    return Ke, vol


def assemble(scene):
    """Mass M (lumped, diagonal), stiffness K, damping B and system matrix A.

    A = M + h B + h^2 K with B = alpha M + beta K (Eq. 5); clamped DOFs get
    identity rows and columns in A (R13).  Returns a dict of scipy CSR
    matrices and vectors, all float64, DOF index = 3 * node + axis.
    """
    nodes, tets = scene["nodes"], scene["tets"]
    N = len(nodes)
    n = 3 * N
    Ke, vol = element_matrices(nodes, tets, scene["E"], scene["nu_e"])
    dofs = (3 * tets[:, :, None] + np.arange(3)[None, None, :]).reshape(len(tets), 12)
    rows = np.repeat(dofs, 12, axis=1).ravel()
    cols = np.tile(dofs, (1, 12)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    mnode = np.zeros(N)
    np.add.at(mnode, tets.ravel(), np.repeat(scene["rho"] * vol / 4.0, 4))
    Mdiag = np.repeat(mnode, 3)
    M = sp.diags(Mdiag).tocsr()
    h, alpha, beta = scene["h"], scene["alpha"], scene["beta"]
    Bd = alpha * M + beta * K
    A = (M + h * Bd + (h * h) * K).tocsr()
    fixed_dofs = np.nonzero(np.repeat(scene["fixed"].astype(bool), 3))[0]
    if len(fixed_dofs):
        keep = np.ones(n)
        keep[fixed_dofs] = 0.0
        S = sp.diags(keep)
        A = (S @ A @ S + sp.diags(1.0 - keep)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return dict(K=K, M=M, Mdiag=Mdiag, B=Bd.tocsr(), A=A, n=n, fixed_dofs=fixed_dofs, vol=vol)


# ---------------------------------------------------------------------------
# Cholesky of A (the factor the multi-RHS solves run against)
# ---------------------------------------------------------------------------

class CholeskyFactor:
    """A = L L^T by LAPACK: dense for small n, banded (after an RCM ordering) else."""

    def __init__(self, A, dense_max: int = 3000):
        A = sp.csr_matrix(A)
        self.n = n = A.shape[0]
        if n <= dense_max:
            self.kind = "dense"
            self.L = np.linalg.cholesky(A.toarray())
        else:
            self.kind = "banded"
            perm = reverse_cuthill_mckee(A, symmetric_mode=True).astype(np.int64)
            Ap = A[perm][:, perm].tocoo()
            low = Ap.row >= Ap.col
            r, c, v = Ap.row[low], Ap.col[low], Ap.data[low]
            bw = int((r - c).max())
            ab = np.zeros((bw + 1, n))
            ab[r - c, c] = v
            self.perm = perm
            self.bandwidth = bw
            self.cb = sla.cholesky_banded(ab, lower=True, overwrite_ab=True, check_finite=False)

    def solve(self, B):
        """X = A^{-1} B for a vector or a dense column block."""
        B = np.asarray(B, dtype=np.float64)
        if self.kind == "dense":
            return sla.cho_solve((self.L, True), B, check_finite=False)
        X = np.empty_like(B)
        X[self.perm] = sla.cho_solve_banded((self.cb, True), B[self.perm], check_finite=False)
        return X


# ---------------------------------------------------------------------------
# Free motion: Eq. (5), Eq. (12), Algorithm 1 (assemble / free solve / q_free)
# ---------------------------------------------------------------------------

def free_motion(asm, factor, scene, q, v, q_rest):
    """b = h M g - h f_t - h^2 K v (Eq. 5, R14); dv_free = A^-1 b; q_free = q + h (v + dv_free)."""
    h = scene["h"]
    g = np.tile(np.asarray(scene["gravity"], dtype=np.float64), len(scene["nodes"]))
    K, Mdiag, B = asm["K"], asm["Mdiag"], asm["B"]
    f_t = K @ (q - q_rest) + B @ v
    b = h * (Mdiag * g) - h * f_t - (h * h) * (K @ v)
    b[asm["fixed_dofs"]] = 0.0
    dv_free = factor.solve(b)
    q_free = q + h * (v + dv_free)
    return dv_free, q_free, b


# ---------------------------------------------------------------------------
# Contact generation stand-in: signed distance to the analytic obstacle
# (Sec. "Contact generation", Eq. 6; R17)
# ---------------------------------------------------------------------------

def obstacle_point(obs, t):
    return np.asarray(obs["c0"], dtype=np.float64) + np.asarray(obs["vel"], dtype=np.float64) * t


def signed_distance(p, obs, t):
    """Signed distance phi and outward normal n of points p[k,3] at time t."""
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    c = obstacle_point(obs, t)
    if obs["kind"] == "sphere":
        r = p - c
        dist = np.sqrt(r[:, 0] * r[:, 0] + r[:, 1] * r[:, 1] + r[:, 2] * r[:, 2])
        nrm = r / dist[:, None]
        return dist - obs["radius"], nrm
    nvec = np.asarray(obs["normal"], dtype=np.float64)
    r = p - c
    phi = r[:, 0] * nvec[0] + r[:, 1] * nvec[1] + r[:, 2] * nvec[2]
    return phi, np.broadcast_to(nvec, p.shape).copy()


def select_contacts(q_free, scene, t1):
    """Node ids of the K candidates closest to the obstacle at q_free (ties by id), ascending (R17)."""
    cand = scene["candidates"]
    phi, _ = signed_distance(q_free.reshape(-1, 3)[cand], scene["obstacle"], t1)
    order = np.lexsort((cand, phi))[: scene["n_contacts"]]
    chosen = np.sort(cand[order])
    return chosen


def contact_margin(q_free, scene, t1):
    """Gap between the K-th and (K+1)-th smallest signed distances at q_free.

    The selection of R17 is decided by this difference: 0 means a tie that the
    node-id rule breaks; a tiny positive value means a near-tie that rounding
    on another machine could flip.
    """
    cand = scene["candidates"]
    phi, _ = signed_distance(q_free.reshape(-1, 3)[cand], scene["obstacle"], t1)
    s = np.sort(phi)
    K = scene["n_contacts"]
    return float(s[K] - s[K - 1]) if K < len(s) else math.inf


def mapping_H(nodes_c, n, weights=None):
    """H: the geometric-mapping Jacobian of the contact points (Eq. 6), m x n sparse.

    Nodal contacts (``weights`` None): contact c selects the three DOFs of node
    nodes_c[c].  Mapped contacts: nodes_c and weights are [n_c, S]; the point
    of contact c is sum_s weights[c, s] x(nodes_c[c, s]) (barycentric weights
    of a surface point), slots with node -1 are unused, and a negative weight
    marks a node of the second body, so that H = [H_1, -H_2] and H q is the
    relative position x_1 - x_2 of the pair (Eq. 6, 16-17; R19).
    """
    nodes_c = np.asarray(nodes_c)
    if weights is None:
        nc = len(nodes_c)
        rows = np.arange(3 * nc)
        cols = (3 * nodes_c[:, None] + np.arange(3)[None, :]).ravel()
        return sp.csr_matrix((np.ones(3 * nc), (rows, cols)), shape=(3 * nc, n))
    weights = np.asarray(weights, dtype=np.float64)
    nc, S = nodes_c.shape
    rows, cols, vals = [], [], []
    for c in range(nc):
        for k in range(S):
            if nodes_c[c, k] < 0:
                continue
            for a in range(3):
                rows.append(3 * c + a)
                cols.append(3 * nodes_c[c, k] + a)
                vals.append(weights[c, k])
    return sp.csr_matrix((vals, (rows, cols)), shape=(3 * nc, n))


# ---------------------------------------------------------------------------
# Mapping compliance W_H = H A^-1 H^T (Eq. 28) and the Delassus operator
# ---------------------------------------------------------------------------

def build_WH(factor, nodes_c, n, columns=None, weights=None):
    """W_H = H A^{-1} H^T, symmetrised (Eq. 28, R15).

    With ``columns`` given, return only those columns of the unsymmetrised
    H A^{-1} H^T (used at sizes where all m solves are too slow).  ``weights``
    as in ``mapping_H``.
    """
    H = mapping_H(nodes_c, n, weights)
    if columns is None:
        Y = factor.solve(H.T.toarray())
        WH = H @ Y
        return 0.5 * (WH + WH.T)
    cols = np.asarray(columns)
    Y = factor.solve(H.T[:, cols].toarray())
    return H @ Y


def build_WH_schur(A, nodes_c):
    """W_H = H A^{-1} H^T for nodal contacts (Eq. 28) as the inverse of a Schur complement.

    For nodal contacts H selects the contact DOFs c, so W_H = (A^{-1})_cc, the
    contact block of the inverse.  Order the DOFs with the contacts last (P A
    P^T = [[A_rr, A_rc], [A_cr, A_cc]]); block elimination gives
    (A^{-1})_cc = S^{-1} with the Schur complement S = A_cc - A_cr A_rr^{-1} A_rc,
    and S = L_cc L_cc^T for the trailing block L_cc of the Cholesky factor of
    P A P^T.  So W_H = L_cc^{-T} L_cc^{-1}, symmetrised (R15).  The remaining
    nodes are ordered by breadth-first levels from the contact set, farthest
    first, which keeps P A P^T banded for LAPACK's banded Cholesky.
    Rows and columns come out in contact order, 3 per contact.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    N = n // 3
    nodes_c = np.asarray(nodes_c, dtype=np.int64)
    Ac = A.tocoo()
    G = sp.csr_matrix((np.ones(len(Ac.row)), (Ac.row // 3, Ac.col // 3)), shape=(N, N))
    k = len(nodes_c)
    link = sp.csr_matrix((np.ones(k), (nodes_c, np.zeros(k, dtype=np.int64))), shape=(N, 1))
    Ge = sp.bmat([[G, link], [link.T, None]]).tocsr()           # node N joins every contact node
    order = breadth_first_order(Ge, N, directed=False, return_predecessors=False)[1:]
    seen = np.zeros(N, dtype=bool)
    seen[order] = True
    is_c = np.zeros(N, dtype=bool)
    is_c[nodes_c] = True
    rest = np.concatenate([np.nonzero(~seen)[0], order[~is_c[order]][::-1]])   # unreached = clamped nodes
    perm = (3 * np.concatenate([rest, nodes_c])[:, None] + np.arange(3)[None, :]).ravel()
    Ap = A[perm][:, perm].tocoo()
    low = Ap.row >= Ap.col
    r, c, v = Ap.row[low], Ap.col[low], Ap.data[low]
    bw = int((r - c).max())
    ab = np.zeros((bw + 1, n))
    ab[r - c, c] = v
    cb = sla.cholesky_banded(ab, lower=True, overwrite_ab=True, check_finite=False)
    m = 3 * k
    r0 = n - m
    Lcc = np.zeros((m, m))
    for d in range(min(bw + 1, m)):
        j = np.arange(r0, n - d)
        Lcc[j - r0 + d, j - r0] = cb[d, j]
    Linv = sla.solve_triangular(Lcc, np.eye(m), lower=True, check_finite=False)
    WH = Linv.T @ Linv
    return 0.5 * (WH + WH.T)


def rotation_blocks_apply(C, x):
    """Block-diagonal C (Eq. 26) times x: y_a = C_a x_a."""
    return np.einsum("aij,aj->ai", C, x.reshape(-1, 3)).ravel()


def rotation_blocks_apply_T(C, x):
    """C^T x blockwise: y_a = C_a^T x_a."""
    return np.einsum("aji,aj->ai", C, x.reshape(-1, 3)).ravel()


def update_W(WH, C):
    """Fast update W = C W_H C^T (Eq. 28; Algorithm 3, second step), 3x3 blocks."""
    nc = C.shape[0]
    Wb = WH.reshape(nc, 3, nc, 3)
    W = np.einsum("aij,ajbk,blk->aibl", C, Wb, C)
    return W.reshape(3 * nc, 3 * nc)


def jacobian(C, nodes_c, n, weights=None):
    """Contact Jacobian J = C H (Eq. 27)."""
    H = mapping_H(nodes_c, n, weights)
    Cbd = sp.block_diag([C[a] for a in range(C.shape[0])], format="csr")
    return Cbd @ H


def delassus_explicit(factor, J):
    """W = J A^{-1} J^T built directly (Eq. 17), the standard rebuild of Algorithm 2."""
    Y = factor.solve(J.T.toarray())
    return J @ Y


# ---------------------------------------------------------------------------
# Constraint directions and gaps (Eq. 7, 10, 26; R4, R9, R11)
# ---------------------------------------------------------------------------

def tangent_basis(nrm):
    """t1, t2 completing the unit normal n into a right-handed orthonormal frame (R11)."""
    nrm = np.asarray(nrm, dtype=np.float64)
    k = nrm.shape[0]
    ax = np.argmin(np.abs(nrm), axis=1)      # first minimum on ties
    e = np.zeros((k, 3))
    e[np.arange(k), ax] = 1.0
    en = (e * nrm).sum(axis=1)
    t1 = e - en[:, None] * nrm
    t1 = t1 / np.sqrt(t1[:, 0] * t1[:, 0] + t1[:, 1] * t1[:, 1] + t1[:, 2] * t1[:, 2])[:, None]
    t2 = np.cross(nrm, t1)
    return t1, t2


def pair_directions(p, p_start, normals):
    """Frames and gaps of pair contacts (R20): fixed normal n, gap n . p,
    tangential gap T (p - p_start)."""
    p = p.reshape(-1, 3)
    nrm = np.asarray(normals, dtype=np.float64).reshape(-1, 3)
    ta, tb = tangent_basis(nrm)
    C = np.stack([nrm, ta, tb], axis=1)
    rel = p - p_start.reshape(-1, 3)
    phi = nrm[:, 0] * p[:, 0] + nrm[:, 1] * p[:, 1] + nrm[:, 2] * p[:, 2]
    delta = np.stack([phi, (ta * rel).sum(axis=1), (tb * rel).sum(axis=1)], axis=1)
    return C, delta.ravel()


def directions(p, p_start, obs, t0, t1, pair_normals=None):
    """Frames C [nc,3,3] (rows n, t1, t2) and gaps delta [m] at proximity p (Algorithm 3, step 1).

    With ``pair_normals`` [P, 3], the first P contacts are pairs (R20) and the
    others obstacle contacts.
    """
    if pair_normals is not None and len(pair_normals):
        P = len(pair_normals)
        Cp, dp = pair_directions(p[:3 * P], p_start[:3 * P], pair_normals)
        if 3 * P == len(p):
            return Cp, dp
        Co, do = directions(p[3 * P:], p_start[3 * P:], obs, t0, t1)
        return np.concatenate([Cp, Co]), np.concatenate([dp, do])
    p = p.reshape(-1, 3)
    phi, nrm = signed_distance(p, obs, t1)
    ta, tb = tangent_basis(nrm)
    C = np.stack([nrm, ta, tb], axis=1)
    u_obs = obstacle_point(obs, t1) - obstacle_point(obs, t0)
    rel = p - p_start.reshape(-1, 3) - u_obs[None, :]
    delta = np.stack([phi, (ta * rel).sum(axis=1), (tb * rel).sum(axis=1)], axis=1)
    return C, delta.ravel()


# ---------------------------------------------------------------------------
# Projected Gauss-Seidel: Eq. (18)-(19), Algorithm 1 (PGS loop)
# ---------------------------------------------------------------------------

def chol3(a):
    """Cholesky of a 3x3 SPD matrix, fixed operation order."""
    l00 = math.sqrt(a[0][0])
    l10 = a[1][0] / l00
    l20 = a[2][0] / l00
    l11 = math.sqrt(a[1][1] - l10 * l10)
    l21 = (a[2][1] - l20 * l10) / l11
    l22 = math.sqrt(a[2][2] - l20 * l20 - l21 * l21)
    return l00, l10, l20, l11, l21, l22


def chol3_solve(L, d):
    l00, l10, l20, l11, l21, l22 = L
    y0 = d[0] / l00
    y1 = (d[1] - l10 * y0) / l11
    y2 = (d[2] - l20 * y0 - l21 * y1) / l22
    x2 = y2 / l22
    x1 = (y1 - l21 * x2) / l11
    x0 = (y0 - l10 * x1 - l20 * x2) / l00
    return x0, x1, x2


def local_solve(Wl, d, mu, j_inner):
    """Per-contact solution of Signorini (Eq. 8) + Coulomb cone (Eq. 9, R3, R5).

    Wl: 3x3 diagonal block of h^2 W in frame (n, t1, t2); d: the contact's
    gap with every other contact's current force (Eq. 19).  Branches:
      separate  d_n >= 0                          -> lambda = 0
      stick     lambda* = -Wl^-1 d inside the cone -> lambda = lambda*
      slip      lambda_t = mu lambda_n u on the cone boundary, with delta_n = 0
                and u opposite to the tangential gap (maximal dissipation).
    The slip direction is a fixed point  u = -r/|r|,
      r = d_t + W_tn lambda_n + mu lambda_n (W_tt - kappa I) u,
    kappa = trace(W_tt)/2: subtracting kappa I from the self term makes the map
    a contraction (factor <= (l_max - l_min)/(l_max + l_min) of W_tt), and it is
    exact after one pass when W_tt is isotropic.  j_inner passes, then lambda
    from the last u.  Returns (lam_n, lam_t1, lam_t2), status.
    """
    if d[0] >= 0.0:
        return (0.0, 0.0, 0.0), SEPARATE
    x = chol3_solve(chol3(Wl), d)
    ln, lt1, lt2 = -x[0], -x[1], -x[2]
    if ln > 0.0 and lt1 * lt1 + lt2 * lt2 <= (mu * ln) * (mu * ln):
        return (ln, lt1, lt2), STICK
    nt = math.sqrt(lt1 * lt1 + lt2 * lt2)
    if nt > 0.0:
        u0, u1 = lt1 / nt, lt2 / nt
    else:
        ndt = math.sqrt(d[1] * d[1] + d[2] * d[2])
        if ndt > 0.0:
            u0, u1 = -d[1] / ndt, -d[2] / ndt
        else:
            u0, u1 = 1.0, 0.0
    kap = 0.5 * (Wl[1][1] + Wl[2][2])

    def force(u0, u1):
        den = Wl[0][0] + mu * (Wl[0][1] * u0 + Wl[0][2] * u1)
        if den <= 0.0:
            den = Wl[0][0]
        lam_n = -d[0] / den
        return lam_n, mu * lam_n * u0, mu * lam_n * u1

    for _ in range(j_inner):
        lam_n, l1, l2 = force(u0, u1)
        r1 = d[1] + Wl[1][0] * lam_n + (Wl[1][1] - kap) * l1 + Wl[1][2] * l2
        r2 = d[2] + Wl[2][0] * lam_n + Wl[2][1] * l1 + (Wl[2][2] - kap) * l2
        nr = math.sqrt(r1 * r1 + r2 * r2)
        if nr > 0.0:
            u0, u1 = -r1 / nr, -r2 / nr
    return force(u0, u1), SLIP


def decision_margins(Wl, d, mu):
    """Relative margins of the two decisions ``local_solve`` takes for one contact.

    sep:  |d_n| / |d|, how far the gap is from the separate/contact switch;
    cone: |mu lam*_n - |lam*_t|| / (mu lam*_n) for the stick trial lam* of a
          contact that is not separate (the stick/slip switch); inf when the
          trial has lam*_n <= 0 or mu = 0 (no cone test is taken then).
    A margin below about 1e-8 marks a decision that rounding on another
    machine could flip (the classification parity of Eq. 8-9).
    """
    nd = math.sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])
    sep = abs(d[0]) / nd if nd > 0.0 else math.inf
    if d[0] >= 0.0:
        return sep, math.inf
    x = chol3_solve(chol3(Wl), d)
    ln, nt = -x[0], math.sqrt(x[1] * x[1] + x[2] * x[2])
    if ln <= 0.0 or mu == 0.0:
        return sep, math.inf
    return sep, abs(mu * ln - nt) / (mu * ln)


def pgs(W, d, mu, h, lam0, max_sweeps, tol, j_inner=8, margins=None):
    """Projected Gauss-Seidel on delta = d + h^2 W lambda (Eq. 18-19, Algorithm 1; R2, R6, R7).

    Returns lambda [m], status [nc] (branch of the last sweep), sweeps, eps.
    With ``margins`` a list, the decision margins (``decision_margins``) of
    every contact's visit in the last sweep are appended to it as an
    [nc, 2] array (columns sep, cone).
    """
    Wt = (h * h) * np.asarray(W, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    nc = len(d) // 3
    lam = np.array(lam0, dtype=np.float64, copy=True)
    status = np.zeros(nc, dtype=np.int8)
    eps = math.inf
    sweeps = 0
    diag = [Wt[3 * a:3 * a + 3, 3 * a:3 * a + 3].tolist() for a in range(nc)]
    marg = np.full((nc, 2), math.inf) if margins is not None else None
    for sweep in range(max_sweeps):
        prev = lam.copy()
        for a in range(nc):
            r0, r1 = 3 * a, 3 * a + 3
            rows = Wt[r0:r1]
            da = d[r0:r1] + rows[:, :r0] @ lam[:r0] + rows[:, r1:] @ lam[r1:]
            if marg is not None:
                marg[a] = decision_margins(diag[a], da.tolist(), float(mu[a]))
            (l0, l1, l2), st = local_solve(diag[a], da.tolist(), float(mu[a]), j_inner)
            lam[r0], lam[r0 + 1], lam[r0 + 2] = l0, l1, l2
            status[a] = st
        sweeps = sweep + 1
        diff = float(np.sqrt(np.dot(lam - prev, lam - prev)))
        nl = float(np.sqrt(np.dot(lam, lam)))
        eps = diff / nl if nl > 0.0 else (0.0 if diff == 0.0 else math.inf)
        if eps <= tol:
            break
    if margins is not None:
        margins.append(marg)
    return lam, status, sweeps, eps


# ---------------------------------------------------------------------------
# Recursive corrective motion with the fast update: Algorithm 3, Eq. (28)-(31)
# ---------------------------------------------------------------------------

def newton_fast(WH, p_free, p_start, obs, t0, t1, mu, h, f_init, n_newton, max_sweeps, tol, j_inner,
                record=None, margins=False, pair_normals=None):
    """Algorithm 3 with readings R8-R10.  Returns (f world force [nc,3], p, last C, lambda, info).

    With ``margins``, each entry of ``info`` (and of ``record``) also holds the
    decision margins of that iteration's last PGS sweep (``pgs``).
    """
    nc = len(p_free) // 3
    p = p_free.copy()
    f = f_init.reshape(-1, 3).copy()
    info = []
    lam = np.zeros(3 * nc)
    C = None
    for k in range(n_newton):
        C, delta = directions(p, p_start, obs, t0, t1, pair_normals)   # step 1
        W = update_W(WH, C)                                            # step 2
        dk = delta - rotation_blocks_apply(C, p - p_free)              # R9
        lam0 = rotation_blocks_apply(C, f.ravel())                     # R8 warm start
        marg = [] if margins else None
        lam, status, sweeps, eps = pgs(W, dk, mu, h, lam0, max_sweeps, tol, j_inner, marg)   # step 3
        f = rotation_blocks_apply_T(C, lam).reshape(-1, 3)
        p = p_free + (h * h) * (WH @ f.ravel())                        # step 4 (Eq. 31)
        info.append(dict(sweeps=sweeps, eps=eps, status=status.copy()))
        if margins:
            info[-1]["margins"] = marg[0]
        if record is not None:
            record.append(dict(C=C, W=W, d=dk, lam0=lam0, lam=lam.copy(), status=status.copy(), p=p.copy(),
                               sweeps=sweeps, eps=eps))
            if margins:
                record[-1]["margins"] = marg[0]
    return f, p, C, lam, info


def pgs_per_constraint(WH, p_free, p_start, obs, t0, t1, mu, h, f_init, max_sweeps, tol, j_inner=8):
    """Gauss-Seidel with the directions updated before every local solve (R18).

    Returns (f world force [nc,3], C last frames [nc,3,3], lambda [m] in those
    frames, status [nc], sweeps, eps).
    """
    nc = len(p_free) // 3
    WH = np.asarray(WH, dtype=np.float64)
    f = np.array(f_init, dtype=np.float64).reshape(nc, 3)
    C = np.zeros((nc, 3, 3))
    lam = np.zeros(3 * nc)
    status = np.zeros(nc, dtype=np.int8)
    eps = math.inf
    sweeps = 0
    h2 = h * h
    for sweep in range(max_sweeps):
        prev = f.copy()
        for a in range(nc):
            r0, r1 = 3 * a, 3 * a + 3
            pa = p_free[r0:r1] + h2 * (WH[r0:r1] @ f.ravel())          # current proximity of contact a
            Ca, delta = directions(pa, p_start[r0:r1], obs, t0, t1)      # its frame and gap there
            Ca = Ca[0]
            Wl = h2 * (Ca @ WH[r0:r1, r0:r1] @ Ca.T)
            da = delta - Wl @ (Ca @ f[a])                               # R9 for this contact alone
            (l0, l1, l2), st = local_solve(Wl.tolist(), da.tolist(), float(mu[a]), j_inner)
            la = np.array([l0, l1, l2])
            f[a] = Ca.T @ la
            C[a] = Ca
            lam[r0:r1] = la
            status[a] = st
        sweeps = sweep + 1
        diff = float(np.sqrt(np.sum((f - prev) ** 2)))
        nf = float(np.sqrt(np.sum(f * f)))
        eps = diff / nf if nf > 0.0 else (0.0 if diff == 0.0 else math.inf)
        if eps <= tol:
            break
    return f, C, lam, status, sweeps, eps


def newton_per_constraint(WH, p_free, p_start, obs, t0, t1, mu, h, f_init, n_newton, max_sweeps, tol, j_inner,
                          record=None):
    """Algorithm 3's loop with the per-constraint direction update (R18) in place
    of steps 1-3: n_newton calls of max_sweeps sweeps, each followed by the
    proximity update of Eq. 31."""
    f = np.array(f_init, dtype=np.float64).reshape(-1, 3)
    p = p_free + (h * h) * (WH @ f.ravel())
    info = []
    C = lam = None
    for k in range(n_newton):
        f, C, lam, status, sweeps, eps = pgs_per_constraint(WH, p_free, p_start, obs, t0, t1, mu, h, f, max_sweeps,
                                                           tol, j_inner)
        p = p_free + (h * h) * (WH @ f.ravel())
        info.append(dict(sweeps=sweeps, eps=eps, status=status.copy()))
        if record is not None:
            record.append(dict(C=C, lam=lam.copy(), status=status.copy(), p=p.copy(), sweeps=sweeps, eps=eps))
    return f, p, C, lam, info


def newton_standard(factor, nodes_c, n, q_free, p_start, obs, t0, t1, mu, h, f_init, n_newton, max_sweeps,
                    tol, j_inner, record=None):
    """Algorithm 2: re-linearise, rebuild W_k = J_k A^-1 J_k^T, PGS, correct, integrate, remap."""
    H = mapping_H(nodes_c, n)
    p_free = H @ q_free
    p = p_free.copy()
    f = f_init.reshape(-1, 3).copy()
    q = q_free.copy()
    lam = None
    for k in range(n_newton):
        C, delta = directions(p, p_start, obs, t0, t1)
        J = jacobian(C, nodes_c, n)
        W = delassus_explicit(factor, J)
        W = 0.5 * (W + W.T)
        dk = delta - rotation_blocks_apply(C, p - p_free)
        lam0 = rotation_blocks_apply(C, f.ravel())
        lam, status, sweeps, eps = pgs(W, dk, mu, h, lam0, max_sweeps, tol, j_inner)
        f = rotation_blocks_apply_T(C, lam).reshape(-1, 3)
        q = q_free + (h * h) * factor.solve(J.T @ lam)                 # Eq. 22-23, total force (R8)
        p = H @ q
        if record is not None:
            record.append(dict(C=C, W=W, d=dk, lam=lam.copy(), status=status.copy(), p=p.copy(),
                               sweeps=sweeps, eps=eps))
    return f, p, q, lam


# ---------------------------------------------------------------------------
# One time step (Algorithm 1 outer loop with Algorithm 3 inside)
# ---------------------------------------------------------------------------

class Simulation:
    """Scene state and the full time step of the fast scheme, on the CPU."""

    def __init__(self, scene, dense_max=3000):
        self.scene = scene
        self.asm = assemble(scene)
        self.factor = CholeskyFactor(self.asm["A"], dense_max=dense_max)
        self.n = self.asm["n"]
        self.q_rest = scene["nodes"].ravel().copy()
        self.q = self.q_rest.copy()
        self.v = np.zeros(self.n)
        self.t = 0.0
        self.node_force = np.zeros((len(scene["nodes"]), 3))   # R16
        cand = scene["candidates"]
        self.mu_of_node = np.zeros(len(scene["nodes"]))
        self.mu_of_node[cand] = scene["cand_mu"]
        pr = scene.get("pairs")
        self.pairs = pr
        self.pair_force = np.zeros((len(pr["ids"]), 3)) if pr is not None else None   # R21

    def step(self, standard=False, record=None, max_sweeps=None, tol=None, per_constraint=False, margins=False,
             wh="solve"):
        """One time step.  ``wh`` = "solve" builds W_H by A^-1 H^T solves
        (``build_WH``), "schur" by the Schur complement (``build_WH_schur``)."""
        sc = self.scene
        h = sc["h"]
        t0, t1 = self.t, self.t + h
        ms = sc["max_sweeps"] if max_sweeps is None else max_sweeps
        tl = sc["tol"] if tol is None else tol
        dv_free, q_free, _ = free_motion(self.asm, self.factor, sc, self.q, self.v, self.q_rest)
        pr = self.pairs
        P = 0 if pr is None else len(pr["ids"])
        if P and (standard or per_constraint):
            raise ValueError("pair contacts run in the fast scheme (Algorithm 3) only")
        nodes_c = select_contacts(q_free, dict(sc, n_contacts=sc["n_contacts"] - P), t1) \
            if sc["n_contacts"] > P else np.zeros(0, dtype=np.int64)
        if P:
            # R21: the pairs, then the obstacle contacts as one-slot points
            ids = np.full((P + len(nodes_c), 4), -1, dtype=np.int64)
            w = np.zeros((P + len(nodes_c), 4))
            ids[:P], w[:P] = pr["ids"], pr["w"]
            ids[P:, 0], w[P:, 0] = nodes_c, 1.0
            H = mapping_H(ids, self.n, w)
            mu = np.concatenate([pr["mu"], self.mu_of_node[nodes_c]])
            f_init = np.concatenate([self.pair_force, self.node_force[nodes_c]])
            normals = pr["normals"]
        else:
            ids = w = None
            H = mapping_H(nodes_c, self.n)
            mu = self.mu_of_node[nodes_c]
            f_init = self.node_force[nodes_c]
            normals = None
        p_free = H @ q_free
        p_start = H @ self.q
        out = dict(nodes_c=nodes_c, q_free=q_free, dv_free=dv_free, p_free=p_free)
        if standard:
            f, p, q_new, lam = newton_standard(self.factor, nodes_c, self.n, q_free, p_start, sc["obstacle"],
                                               t0, t1, mu, h, f_init, sc["n_newton"], ms, tl, sc["j_inner"],
                                               record)
        else:
            if P:
                WH = build_WH(self.factor, ids, self.n, weights=w)
            elif wh == "schur":
                WH = build_WH_schur(self.asm["A"], nodes_c)
            else:
                WH = build_WH(self.factor, nodes_c, self.n)
            out["WH"] = WH
            if per_constraint:
                f, p, C, lam, info = newton_per_constraint(WH, p_free, p_start, sc["obstacle"], t0, t1, mu, h,
                                                           f_init, sc["n_newton"], ms, tl, sc["j_inner"], record)
            else:
                f, p, C, lam, info = newton_fast(WH, p_free, p_start, sc["obstacle"], t0, t1, mu, h, f_init,
                                                 sc["n_newton"], ms, tl, sc["j_inner"], record, margins, normals)
            out["info"] = info
            out["C"] = C
        # corrective motion and integration (Eq. 20, Algorithm 1 last loop, R1)
        dv = dv_free + h * self.factor.solve(H.T @ f.ravel())
        self.v = self.v + dv
        self.q = self.q + h * self.v
        self.node_force[:] = 0.0
        self.node_force[nodes_c] = f[P:]
        if P:
            self.pair_force = f[:P].copy()
        self.t = t1
        out.update(f=f, p=p, lam=lam, q=self.q.copy(), v=self.v.copy())
        return out
