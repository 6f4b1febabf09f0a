"""GLS-stabilised finite elements for the model problem (Section 2).

The discrete problem is a(u, v) = b(u, v) + z(u, v) = g(v) with
  b(u, v) = int nu grad u . grad v + C(x) Lu Lv + ctilde u v
  z(u, v) = 1/2 int (a . grad u) v - (a . grad v) u
  g(v)    = int f v + C(x) f Lv
  L u     = -div(nu grad u) + a . grad u + c u,  ctilde = c - div(a) / 2
and the element parameter C_K of the Peclet-number switch with tau (Section 2,
definition of P_K and C(x)).  Two element families on the box grid:

  * "q1": trilinear boxes (the synthetic workloads), on which -div(nu grad u)
    vanishes inside an element for constant nu_K, so L u = a . grad u + c u
    elementwise; affine velocity, 3x3x3 Gauss quadrature.
  * "p1": the paper's linear tetrahedra, six per box (the Kuhn split used by
    the numerical examples of Section 4), viscosity per tetrahedron, the
    velocity interpolated linearly from nodal values on each tetrahedron
    (|a|_K is then the largest vertex speed and div a is constant on K),
    4-point degree-2 quadrature, exact for every integrand with linear a and f.

Entry A_K[i, j] = a(phi_j, phi_i): row = test function, column = trial.
Box-local corner (p, q, r) in {0,1}^3 has index p + 2 q + 4 r; a "p1" box
matrix is the sum of its six tetrahedra's 4x4 matrices on those corners.

Nonzero Dirichlet data (Section 4's example) enter by lifting: u_h = u_0 + w
with u_0 the nodal data on the boundary and w in the space with zero trace,
so the load of a free node i becomes g(phi_i) - a(u_0, phi_i).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def gauss01(npts):
    """Gauss-Legendre points and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(npts)
    return 0.5 * (x + 1.0), 0.5 * w


def _corner_bits():
    idx = np.arange(8)
    return idx & 1, (idx >> 1) & 1, (idx >> 2) & 1


def velocity(problem, pts):
    """a(x) = beta0 + beta1 x at points pts (..., 3)."""
    return problem["beta0"] + pts @ problem["beta1"].T


def origin(problem):
    return np.asarray(problem.get("origin", (0.0, 0.0, 0.0)), dtype=np.float64)


def element_geometry(problem, topo):
    """Lower corners (ne, 3) and sizes (3,) of all elements (x-fastest)."""
    L = problem["length"]
    h = np.array([L[a] / topo.ne_axis[a] for a in range(3)])
    e = np.arange(topo.n_elem)
    ex = e % topo.ne_axis[0]
    ey = (e // topo.ne_axis[0]) % topo.ne_axis[1]
    ez = e // (topo.ne_axis[0] * topo.ne_axis[1])
    x0 = origin(problem) + np.stack([ex * h[0], ey * h[1], ez * h[2]], axis=1)
    return x0, h, (ex, ey, ez)


def node_coordinates(problem, topo):
    """Coordinates (n_nodes, 3) of every grid node, node-id order."""
    L = problem["length"]
    h = np.array([L[a] / topo.ne_axis[a] for a in range(3)])
    ix, iy, iz = topo.node_coords(np.arange(topo.n_nodes))
    return origin(problem) + np.stack([ix * h[0], iy * h[1], iz * h[2]], axis=1)


def kuhn_tetrahedra():
    """Corner indices (6, 4) of the six tetrahedra of a box: the monotone
    corner paths from corner 0 to corner 7, one per ordering of the three
    axes, orderings in lexicographic order (xyz, xzy, yxz, yzx, zxy, zyx)."""
    out = []
    for perm in itertools.permutations(range(3)):
        v, cur = [0], 0
        for a in perm:
            cur += 1 << a
            v.append(cur)
        out.append(v)
    return np.array(out, dtype=np.int64)


def tet_quadrature():
    """Symmetric 4-point rule on a tetrahedron, exact for polynomials of
    degree 2: barycentric points (alpha, beta, beta, beta) and permutations,
    alpha = (5 + 3 sqrt 5) / 20, beta = (5 - sqrt 5) / 20, weights 1/4 of the
    volume."""
    al = (5.0 + 3.0 * np.sqrt(5.0)) / 20.0
    be = (5.0 - np.sqrt(5.0)) / 20.0
    lam = np.full((4, 4), be)
    np.fill_diagonal(lam, al)
    return lam, np.full(4, 0.25)


def element_kind(problem):
    return problem.get("element", "q1")


def element_node_ids(topo, ex, ey, ez):
    px, py, pz = _corner_bits()
    return topo.node_id(ex[:, None] + px[None, :], ey[:, None] + py[None, :], ez[:, None] + pz[None, :])


def stabilisation(problem, x0, h, nu):
    """C_K of Section 2: tau h_K / (2 |a|_K) if P_K >= 1, else tau h_K^2 / (4 nu).

    h_K is the box diameter; |a|_K = sup over K of |a|, attained at a vertex
    because |a(x)| is convex for affine a."""
    tau = problem["tau"]
    hK = float(np.sqrt(np.sum(h ** 2)))
    px, py, pz = _corner_bits()
    corners = x0[:, None, :] + np.stack([px, py, pz], axis=1)[None, :, :] * h[None, None, :]
    amax = np.linalg.norm(velocity(problem, corners), axis=2).max(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        peclet = hK * amax / (2.0 * nu)
        c_adv = tau * hK / (2.0 * amax)
    c_diff = tau * hK ** 2 / (4.0 * nu)
    return np.where(peclet >= 1.0, c_adv, c_diff), peclet


def element_matrices(problem, topo, npts=3):
    """Box matrices A_K (ne, 8, 8) and loads F_K (ne, 8) of the problem's
    element family, with the Dirichlet lifting applied to the loads, and the
    corner node ids (ne, 8)."""
    if element_kind(problem) == "p1":
        A, F, nodes = p1_element_matrices(problem, topo)
    else:
        A, F, nodes = q1_element_matrices(problem, topo, npts)
    u0 = problem.get("u_dirichlet")
    if u0 is not None:
        # g(phi_i) - a(u_0, phi_i): u_0 is the data on Dirichlet corners, zero
        # on free ones
        ub = np.where(topo.dof_of_node[nodes] < 0, np.asarray(u0)[nodes], 0.0)
        F = F - np.einsum("eij,ej->ei", A, ub)
    return A, F, nodes


def p1_element_matrices(problem, topo):
    """Box matrices (ne, 8, 8) and loads (ne, 8) as sums over the six Kuhn
    tetrahedra of each box (Section 2's linear elements), without lifting.

    On a tetrahedron with vertices P_k and barycentric coordinates lambda_k:
    phi_k = lambda_k, grad phi_k constant; a_h = sum_k a(P_k) lambda_k;
    ctilde = c - div(a_h) / 2; |a|_K = max_k |a(P_k)|; h_K = the longest
    edge (the box diagonal); C_K by the Peclet switch with the tetrahedron's
    nu; L phi_k = a_h . grad phi_k + c phi_k."""
    x0, h, (ex, ey, ez) = element_geometry(problem, topo)
    ne = topo.n_elem
    nodes = element_node_ids(topo, ex, ey, ez)
    c = problem["c"]
    tau = problem["tau"]
    nu = np.asarray(problem["nu"], dtype=np.float64).reshape(ne, 6)
    px, py, pz = _corner_bits()
    rel = np.stack([px, py, pz], axis=1) * h[None, :]                    # (8, 3) corner offsets
    if problem.get("a_nodal") is not None:
        anod = np.asarray(problem["a_nodal"], dtype=np.float64).reshape(-1, 3)[nodes]   # (ne, 8, 3)
    else:
        anod = velocity(problem, x0[:, None, :] + rel[None, :, :])
    fnod = problem.get("f_nodal")
    fcor = np.full((ne, 8), problem["f_const"]) if fnod is None else np.asarray(fnod)[nodes]
    hK = float(np.sqrt(np.sum(h ** 2)))
    lam, qw = tet_quadrature()
    A = np.zeros((ne, 8, 8))
    F = np.zeros((ne, 8))
    for t, v in enumerate(kuhn_tetrahedra()):
        P = rel[v]                                                         # (4, 3)
        J = (P[1:] - P[0]).T                                               # columns P_k - P_0
        vol = abs(np.linalg.det(J)) / 6.0
        Ji = np.linalg.inv(J)                                              # rows: grad lambda_1..3
        G = np.vstack([-Ji.sum(axis=0), Ji])                               # (4, 3) grad lambda_k
        av = anod[:, v, :]                                                 # (ne, 4, 3)
        diva = np.einsum("eka,ka->e", av, G)
        ctil = c - 0.5 * diva
        amax = np.linalg.norm(av, axis=2).max(axis=1)
        nut = nu[:, t]
        with np.errstate(divide="ignore", invalid="ignore"):
            peclet = hK * amax / (2.0 * nut)
            c_adv = tau * hK / (2.0 * amax)
        CK = np.where(peclet >= 1.0, c_adv, tau * hK ** 2 / (4.0 * nut))
        diff = G @ G.T
        At = np.zeros((ne, 4, 4))
        Ft = np.zeros((ne, 4))
        for q in range(4):
            phi = lam[q]                                                   # (4,)
            w = qw[q] * vol
            aq = np.einsum("k,eka->ea", phi, av)
            agrad = aq @ G.T                                               # (ne, 4) a . grad phi_k
            Lphi = agrad + c * phi[None, :]
            At += w * (nut[:, None, None] * diff[None]
                       + CK[:, None, None] * Lphi[:, :, None] * Lphi[:, None, :]
                       + ctil[:, None, None] * np.outer(phi, phi)[None]
                       + 0.5 * (agrad[:, None, :] * phi[None, :, None]
                                - agrad[:, :, None] * phi[None, None, :]))
            fq = fcor[:, v] @ phi
            Ft += w * (fq[:, None] * phi[None, :] + CK[:, None] * fq[:, None] * Lphi)
        A[:, v[:, None], v[None, :]] += At
        F[:, v] += Ft
    return A, F, nodes


def q1_element_matrices(problem, topo, npts=3):
    """Trilinear box matrices A_K (ne, 8, 8) and loads F_K (ne, 8) by tensor
    Gauss quadrature with npts points per axis (3 is exact for affine a and
    trilinear f), without lifting."""
    x0, h, (ex, ey, ez) = element_geometry(problem, topo)
    nu = problem["nu"]
    c = problem["c"]
    ctil = c - 0.5 * np.trace(problem["beta1"])
    CK, _ = stabilisation(problem, x0, h, nu)
    nodes = element_node_ids(topo, ex, ey, ez)
    fnod = problem["f_nodal"]
    px, py, pz = _corner_bits()
    qp, qw = gauss01(npts)
    vol = float(np.prod(h))
    ne = topo.n_elem
    A = np.zeros((ne, 8, 8))
    F = np.zeros((ne, 8))
    for i, s in enumerate(qp):
        for j, t in enumerate(qp):
            for k, u in enumerate(qp):
                w = qw[i] * qw[j] * qw[k] * vol
                fs = np.where(px == 1, s, 1 - s)
                ft = np.where(py == 1, t, 1 - t)
                fu = np.where(pz == 1, u, 1 - u)
                phi = fs * ft * fu                                   # (8,)
                grad = np.stack([(2 * px - 1) / h[0] * ft * fu,
                                 fs * (2 * py - 1) / h[1] * fu,
                                 fs * ft * (2 * pz - 1) / h[2]], axis=1)  # (8, 3)
                xq = x0 + np.array([s, t, u]) * h                     # (ne, 3)
                aq = velocity(problem, xq)                           # (ne, 3)
                agrad = aq @ grad.T                                  # (ne, 8)
                Lphi = agrad + c * phi[None, :]
                diff = grad @ grad.T                                 # (8, 8)
                A += w * (nu[:, None, None] * diff[None]
                          + CK[:, None, None] * Lphi[:, :, None] * Lphi[:, None, :]
                          + ctil * np.outer(phi, phi)[None]
                          + 0.5 * (agrad[:, None, :] * phi[None, :, None]
                                   - agrad[:, :, None] * phi[None, None, :]))
                if fnod is None:
                    fq = np.full(ne, problem["f_const"])
                else:
                    fq = fnod[nodes] @ phi
                F += w * (fq[:, None] * phi[None, :] + CK[:, None] * fq[:, None] * Lphi)
    return A, F, nodes


def assemble_global(problem, topo, npts=3):
    """Global sparse matrix and load over the free dofs (free-node order)."""
    A, F, nodes = element_matrices(problem, topo, npts)
    dof = topo.dof_of_node[nodes]                                    # (ne, 8)
    rows = np.repeat(dof[:, :, None], 8, axis=2)
    cols = np.repeat(dof[:, None, :], 8, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    M = sp.coo_matrix((A[keep], (rows[keep], cols[keep])), shape=(topo.n_dof, topo.n_dof)).tocsr()
    b = np.zeros(topo.n_dof)
    kf = dof >= 0
    np.add.at(b, dof[kf], F[kf])
    return M, b


def assemble_subdomains(problem, topo, npts=3, elem=None, subs=None):
    """Dense local matrices A^(i) and loads f^(i) in local order [I; Gamma_i]
    (for the subdomains in ``subs``, default all).

    Section 3: A^(i), f^(i) come from a_i(., .) and g(.) restricted to the
    elements of subdomain i; Dirichlet nodes are dropped."""
    if elem is None:
        elem = element_matrices(problem, topo, npts)
    A, F, nodes = elem
    out = []
    for s in (range(topo.n_sub) if subs is None else subs):
        eids = topo.elements_of(s)
        lnodes = topo.local_nodes(s)
        lmap = -np.ones(topo.n_nodes, dtype=np.int64)
        lmap[lnodes] = np.arange(lnodes.size)
        n = lnodes.size
        loc = lmap[nodes[eids]]                                      # (nel, 8)
        Al = np.zeros((n, n))
        fl = np.zeros(n)
        rows = np.repeat(loc[:, :, None], 8, axis=2)
        cols = np.repeat(loc[:, None, :], 8, axis=1)
        keep = (rows >= 0) & (cols >= 0)
        np.add.at(Al, (rows[keep], cols[keep]), A[eids][keep])
        kf = loc >= 0
        np.add.at(fl, loc[kf], F[eids][kf])
        out.append((Al, fl))
    return out
