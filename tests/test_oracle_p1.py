"""Pins of the oracle's linear-tetrahedron discretisation (Section 2's P1
space on the Kuhn split of each box, used by Section 4's example) against
closed forms, a textbook stencil, exact reproduction of linear solutions and
the positivity the paper states for b(., .)."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2501_01676_amd import workloads as W
from oracle import Topology, fem


def _one_box(h, nu, b, c, tau=0.7, f=1.0, nodal=False, origin=(0.0, 0.0, 0.0)):
    """A 2x2x2-box problem (one free node) with constant velocity b."""
    widths = [[1, 1]] * 3
    L = (2 * h[0], 2 * h[1], 2 * h[2])
    kw = {}
    if nodal:
        X, Y, Z = W.grid_nodes(widths, L, origin)
        kw["a_nodal"] = np.tile(np.asarray(b, dtype=float), (X.size, 1))
        beta0 = (0.0, 0.0, 0.0)
    else:
        beta0 = b
    nu_t = np.full(6 * 8, float(nu))
    return W._problem((1, 1, 1), [[2]] * 3, nu_t, beta0, c=c, f_const=f, tau=tau, length=L,
                      element="p1", origin=origin, **kw)


def _kuhn_by_inequalities():
    """The six tetrahedra {x in [0,1]^3 : x_p >= x_q >= x_r} of the unit box,
    one per ordering (p, q, r), as the 4 box corners in each region."""
    corners = [(i & 1, (i >> 1) & 1, (i >> 2) & 1) for i in range(8)]
    tets = []
    for p, q, r in itertools.permutations(range(3)):
        tets.append([i for i, x in enumerate(corners) if x[p] >= x[q] >= x[r]])
    return tets


def _closed_form_box(h, nu, b, c, tau, f):
    """Box matrix and load of the GLS form from per-tetrahedron closed forms:
    barycentric gradients from the 4x4 vertex system, mass V/20 (1 + delta),
    int phi = V/4, constant velocity (div a = 0, |a|_K = |b|)."""
    b = np.asarray(b, dtype=float)
    corners = np.array([[(i & 1) * h[0], ((i >> 1) & 1) * h[1], ((i >> 2) & 1) * h[2]] for i in range(8)])
    A = np.zeros((8, 8))
    F = np.zeros(8)
    for v in _kuhn_by_inequalities():
        P = corners[v]
        Cm = np.hstack([np.ones((4, 1)), P])
        coef = np.linalg.inv(Cm)            # column k: coefficients of lambda_k
        G = coef[1:, :].T                   # (4, 3)
        V = abs(np.linalg.det(Cm)) / 6.0
        hK = max(np.linalg.norm(P[i] - P[j]) for i in range(4) for j in range(4))
        an = np.linalg.norm(b)
        Pk = hK * an / (2 * nu)
        CK = tau * hK / (2 * an) if Pk >= 1 else tau * hK ** 2 / (4 * nu)
        bg = G @ b
        M = V / 20.0 * (np.ones((4, 4)) + np.eye(4))
        for i in range(4):
            for j in range(4):
                gls = V * bg[i] * bg[j] + c * V / 4 * (bg[i] + bg[j]) + c * c * M[i, j]
                A[v[i], v[j]] += nu * V * G[i] @ G[j] + CK * gls + c * M[i, j] + 0.5 * V / 4 * (bg[j] - bg[i])
            F[v[i]] += f * V / 4 + CK * f * (V * bg[i] + c * V / 4)
    return A, F


@pytest.mark.parametrize("nodal", [False, True])
@pytest.mark.parametrize("nu,b,c", [(1.0, (0.0, 0.0, 0.0), 0.0), (0.3, (1.0, -2.0, 0.5), 1.0),
                                    (1e-3, (3.0, 1.0, -1.0), 0.5), (2.0, (0.2, 0.1, 0.0), 2.0)])
def test_p1_box_matches_closed_form(nu, b, c, nodal):
    h = np.array([0.5, 0.25, 0.4])
    p = _one_box(h, nu, b, c, f=1.7, nodal=nodal, origin=(-0.3, 0.2, 1.0))
    topo = Topology(p["nsub"], p["widths"])
    A, F, _ = fem.element_matrices(p, topo)
    Ac, Fc = _closed_form_box(h, nu, b, c, 0.7, 1.7)
    for e in range(topo.n_elem):
        np.testing.assert_allclose(A[e], Ac, rtol=1e-12, atol=1e-14 * np.abs(Ac).max())
        np.testing.assert_allclose(F[e], Fc, rtol=1e-12, atol=1e-14 * np.abs(Fc).max())


def _duffy_rule(n=4):
    """Conical-product Gauss rule on the reference tetrahedron (collapsed
    cube), exact far beyond the degree-2 integrands used here."""
    x, w = np.polynomial.legendre.leggauss(n)
    x, w = 0.5 * (x + 1), 0.5 * w
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                u, v, t = x[i], x[j], x[k]
                pts.append((u, (1 - u) * v, (1 - u) * (1 - v) * t))
                wts.append(w[i] * w[j] * w[k] * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def _sampled_box(h, nu6, a_corner, c, tau, f):
    """Box matrix and load with a velocity interpolated from its 8 corner
    values: each tetrahedron integrated by the collapsed-cube rule, |a|_K as
    the largest speed over a dense barycentric sample of K (vertices
    included), div a from the linear fit through the vertices."""
    corners = np.array([[(i & 1) * h[0], ((i >> 1) & 1) * h[1], ((i >> 2) & 1) * h[2]] for i in range(8)])
    qp, qw = _duffy_rule()
    grid = np.array([(i, j, k) for i in range(7) for j in range(7) for k in range(7) if i + j + k <= 6]) / 6.0
    A = np.zeros((8, 8))
    F = np.zeros(8)
    for t, v in enumerate(_kuhn_by_inequalities()):
        # the inequality regions come out in the same permutation order as
        # the viscosity layout (xyz, xzy, yxz, yzx, zxy, zyx); the vertex
        # order inside a region does not matter
        P = corners[v]
        Cm = np.hstack([np.ones((4, 1)), P])
        coef = np.linalg.inv(Cm)
        G = coef[1:, :].T
        V = abs(np.linalg.det(Cm)) / 6.0
        av = a_corner[v]                                  # (4, 3)
        bary = np.hstack([1 - grid.sum(1, keepdims=True), grid])
        amax = np.linalg.norm(bary @ av, axis=1).max()
        hK = max(np.linalg.norm(P[i] - P[j]) for i in range(4) for j in range(4))
        Pk = hK * amax / (2 * nu6[t])
        CK = tau * hK / (2 * amax) if Pk >= 1 else tau * hK ** 2 / (4 * nu6[t])
        diva = sum(av[k] @ G[k] for k in range(4))
        for xi, wq in zip(qp, qw):
            lam = np.array([1 - xi.sum(), xi[0], xi[1], xi[2]])
            w = wq * 6 * V                                # reference volume 1/6
            aq = lam @ av
            ag = G @ aq
            L = ag + c * lam
            for i in range(4):
                for j in range(4):
                    A[v[i], v[j]] += w * (nu6[t] * G[i] @ G[j] + CK * L[i] * L[j]
                                          + (c - 0.5 * diva) * lam[i] * lam[j]
                                          + 0.5 * (ag[j] * lam[i] - ag[i] * lam[j]))
                F[v[i]] += w * (f * lam[i] + CK * f * L[i])
    return A, F


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p1_box_with_varying_velocity_and_viscosity(seed):
    """A single box (the middle of a 1x1x1 grid has no free node, so compare
    the box matrix itself) with corner velocities drawn at random and six
    different tetrahedron viscosities, against an independent rule."""
    rng = np.random.default_rng(seed)
    h = np.array([0.3, 0.5, 0.2])
    a_corner = rng.uniform(-3, 3, (8, 3))
    nu6 = 10.0 ** rng.uniform(-3, 0, 6)
    c = 0.7
    widths = [[1]] * 3
    nodes_a = np.zeros((8, 3))
    for i in range(8):
        nodes_a[(i & 1) + 2 * ((i >> 1) & 1) + 4 * ((i >> 2) & 1)] = a_corner[i]
    p = W._problem((1, 1, 1), widths, nu6, (0.0, 0.0, 0.0), c=c, f_const=1.3, length=tuple(h),
                   element="p1", a_nodal=nodes_a)
    topo = Topology.__new__(Topology)   # a one-box grid has no interior node; build the ids only
    topo.ne_axis = [1, 1, 1]
    topo.nn_axis = [2, 2, 2]
    topo.n_elem = 1
    topo.n_nodes = 8
    A, F, _ = fem.p1_element_matrices(p, topo)
    Ar, Fr = _sampled_box(h, nu6, a_corner, c, 0.7, 1.3)
    np.testing.assert_allclose(A[0], Ar, rtol=1e-11, atol=1e-12 * np.abs(Ar).max())
    np.testing.assert_allclose(F[0], Fr, rtol=1e-11, atol=1e-12 * np.abs(Fr).max())


def test_p1_kuhn_split_tiles_the_box():
    """The six tetrahedra are the oracle's and each has volume 1/6."""
    mine = sorted(tuple(sorted(v)) for v in fem.kuhn_tetrahedra())
    ref = sorted(tuple(sorted(v)) for v in _kuhn_by_inequalities())
    assert mine == ref
    corners = np.array([[(i & 1), (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], dtype=float)
    for v in fem.kuhn_tetrahedra():
        P = corners[v]
        assert abs(abs(np.linalg.det(P[1:] - P[0])) / 6 - 1 / 6) < 1e-15


def test_p1_laplacian_is_seven_point_stencil():
    """On a uniform cubic grid the P1 stiffness of the Kuhn split is h times
    the 7-point Laplacian (the diagonal couplings cancel)."""
    n = 6
    h = 1.0 / n
    p = W._problem((2, 2, 2), [[3, 3]] * 3, 1.0, (0.0, 0.0, 0.0), c=0.0, element="p1")
    topo = Topology(p["nsub"], p["widths"])
    M, _ = fem.assemble_global(p, topo)
    k = n - 1
    I = np.eye(k)
    T = 2 * I - np.eye(k, k=1) - np.eye(k, k=-1)
    lap = np.kron(np.kron(T, I), I) + np.kron(np.kron(I, T), I) + np.kron(np.kron(I, I), T)
    np.testing.assert_allclose(M.toarray(), h * lap, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_p1_reproduces_linear_solutions(seed):
    """For u linear, constant nu, affine a and f = a . grad u + c u, the GLS
    form is consistent and u lies in the space, so the lifted discrete
    solution equals u at every free node (pins the skew part, ctilde with
    div a != 0, the load's stabilisation term and the lifting)."""
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(-1, 1)
    beta = rng.uniform(-1, 1, 3)
    b0 = rng.uniform(-2, 2, 3)
    b1 = rng.uniform(-2, 2, (3, 3))
    c = 2.0 + abs(np.trace(b1))     # keeps ctilde = c - div(a)/2 > 0
    widths = [[2, 3], [3, 2], [2, 2]]
    org = (-0.5, -0.5, 0.0)
    X, Y, Z = W.grid_nodes(widths, origin=org)
    xyz = np.stack([X, Y, Z], axis=1)
    u = alpha + xyz @ beta
    a = b0 + xyz @ b1.T
    f = a @ beta + c * u
    nu_t = np.full(6 * 5 * 5 * 4, 0.05)
    p = W._problem((2, 2, 2), widths, nu_t, (0.0, 0.0, 0.0), c=c, f_nodal=f, element="p1",
                   origin=org, a_nodal=a, u_dirichlet=u)
    topo = Topology(p["nsub"], p["widths"])
    M, rhs = fem.assemble_global(p, topo)
    sol = spla.spsolve(M.tocsc(), rhs)
    free = np.flatnonzero(topo.dof_of_node >= 0)
    np.testing.assert_allclose(sol, u[free], rtol=0, atol=1e-11)


def test_p1_example_symmetric_part_positive_definite():
    """Section 2: b(., .) is SPD when ctilde > 0; the example's nodal field is
    divergence-free on the Kuhn split, so sym(A) must be SPD."""
    p = W.example_helicoid(3, 1.0, 1e-7, 2)
    topo = Topology(p["nsub"], p["widths"])
    M, _ = fem.assemble_global(p, topo)
    S = M.toarray()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0
    skew = 0.5 * (S - S.T)
    assert np.abs(skew).max() > 1e-3


def test_example_patterns():
    """The helicoidal numbering and the tests' viscosity groups as stated in
    Section 4 (Test 1 groups the x < 0 half)."""
    p = W.example_helicoid(1, 1.0, 1e-7, 2)
    X, Y, Z = W.element_centres(p["widths"], p["length"])
    nu_box = p["nu"].reshape(-1, 6)[:, 0]
    assert np.all((nu_box == 1.0) == (X < 0.5))          # element centres measured from the origin corner
    assert np.all(p["nu"].reshape(-1, 6) == nu_box[:, None])
    X, Y, Z = W.grid_nodes(p["widths"], p["length"], p["origin"])
    assert np.all((p["u_dirichlet"] == 1.0) == (Z == 0.0))
