"""Pins of the oracle's discretisation (Section 2) against closed forms,
exactness, structure and the textbook convergence rate."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2501_01676_amd import workloads as W
from oracle import Topology, fem


# ------------------------------------------------------------ closed forms
def _closed_form_element(h, nu, b, c, tau, f):
    """Element matrix and load of the GLS form on one box with constant
    velocity b, written from tensor products of 1D integrals (independent of
    the quadrature code).  Row i = test function, column j = trial."""
    M = [hd / 6.0 * np.array([[2.0, 1.0], [1.0, 2.0]]) for hd in h]
    K = [1.0 / hd * np.array([[1.0, -1.0], [-1.0, 1.0]]) for hd in h]
    G = np.array([[-0.5, 0.5], [-0.5, 0.5]])   # G[a][a'] = int psi_a psi'_a'
    bits = [(i & 1, (i >> 1) & 1, (i >> 2) & 1) for i in range(8)]

    def prod(fac, i, j):
        return np.prod([fac[d](bits[i][d], bits[j][d]) for d in range(3)])

    def mass(i, j):
        return prod([lambda x, y, d=d: M[d][x][y] for d in range(3)], i, j)

    def dd(d, i, j):       # int d_d phi_j d_d phi_i
        return prod([(lambda x, y, e=e: K[e][x][y]) if e == d else (lambda x, y, e=e: M[e][x][y])
                     for e in range(3)], i, j)

    def cross(d, e, i, j):  # int d_d phi_j d_e phi_i, d != e
        fac = []
        for a in range(3):
            if a == d:
                fac.append(lambda x, y: G[x][y])          # int psi'_{j} psi_{i}: G[i][j]
            elif a == e:
                fac.append(lambda x, y: G[y][x])          # int psi_{j} psi'_{i}: G[j][i]
            else:
                fac.append(lambda x, y, a=a: M[a][x][y])
        return prod(fac, i, j)

    def vd(d, i, j):        # int d_d phi_j phi_i
        return prod([(lambda x, y: G[x][y]) if a == d else (lambda x, y, a=a: M[a][x][y])
                     for a in range(3)], i, j)

    hK = np.sqrt(np.sum(np.square(h)))
    an = np.linalg.norm(b)
    P = hK * an / (2 * nu)
    CK = tau * hK / (2 * an) if P >= 1 else tau * hK ** 2 / (4 * nu)
    A = np.zeros((8, 8))
    for i in range(8):
        for j in range(8):
            diff = sum(dd(d, i, j) for d in range(3))
            gls = sum(b[d] ** 2 * dd(d, i, j) for d in range(3))
            gls += sum(b[d] * b[e] * cross(d, e, i, j) for d in range(3) for e in range(3) if d != e)
            gls += c * sum(b[d] * (vd(d, i, j) + vd(d, j, i)) for d in range(3)) + c * c * mass(i, j)
            skew = 0.5 * sum(b[d] * (vd(d, i, j) - vd(d, j, i)) for d in range(3))
            A[i, j] = nu * diff + CK * gls + c * mass(i, j) + skew
    vol = np.prod(h)
    F = np.zeros(8)
    for i in range(8):
        intphi = vol / 8.0
        intgrad = [(2 * bits[i][d] - 1) * vol / h[d] / 4.0 for d in range(3)]
        F[i] = f * intphi + CK * f * (sum(b[d] * intgrad[d] for d in range(3)) + c * intphi)
    return A, F, CK


def test_q1_laplace_closed_form():
    """Q1 cube stiffness = h * {1/3, 0, -1/12, -1/12} by Hamming distance."""
    p = W.uniform(2, 2, beta=(0.0, 0.0, 0.0))
    topo = Topology(p["nsub"], p["widths"])
    A, F, _ = fem.element_matrices(p, topo)
    h = 0.25
    table = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}
    ref = np.array([[h * table[bin(i ^ j).count("1")] for j in range(8)] for i in range(8)])
    assert np.allclose(A[5], ref, rtol=0, atol=1e-15)
    assert np.allclose(A[5].sum(axis=1), 0, atol=1e-15)
    assert np.allclose(F[5], h ** 3 / 8, rtol=1e-14)


@pytest.mark.parametrize("nu,b,c", [(1.0, (1.0, 0.5, 0.25), 0.0),      # P_K < 1
                                    (1e-3, (10.0, -3.0, 2.0), 0.0),    # P_K >= 1
                                    (0.05, (2.0, 1.0, -1.0), 1.5)])    # reaction
def test_element_matches_tensor_closed_form(nu, b, c):
    widths = [[2, 3], [3, 2], [2, 2]]   # anisotropic boxes
    p = W._problem((2, 2, 2), widths, nu, b, c=c, f_const=1.7)
    topo = Topology(p["nsub"], p["widths"])
    A, F, _ = fem.element_matrices(p, topo)
    h = np.array([1 / 5, 1 / 5, 1 / 4])
    Aref, Fref, _ = _closed_form_element(h, nu, np.array(b), c, 0.7, 1.7)
    scale = np.abs(Aref).max()
    assert np.abs(A[7] - Aref).max() <= 1e-13 * scale
    assert np.abs(F[7] - Fref).max() <= 1e-13 * np.abs(Fref).max()


def test_quadrature_exact_for_affine_velocity():
    """3x3x3 Gauss is exact: equals 5x5x5 for rotating affine a and nodal f."""
    p = W.config4(1)
    small = W._problem((2, 2, 2), [[2, 3], [3, 2], [2, 2]], np.linspace(0.1, 2.0, 100),
                       p["beta0"] * 0.1, p["beta1"] * 0.1, c=0.3,
                       f_nodal=np.random.default_rng(0).standard_normal(6 * 6 * 5))
    topo = Topology(small["nsub"], small["widths"])
    A3, F3, _ = fem.element_matrices(small, topo, 3)
    A5, F5, _ = fem.element_matrices(small, topo, 5)
    assert np.abs(A3 - A5).max() <= 1e-14 * np.abs(A5).max()
    assert np.abs(F3 - F5).max() <= 1e-14 * np.abs(F5).max()


def test_structure_skew_and_symmetric_parts():
    """b(., .) symmetric PSD with constants in its kernel when c = 0 and
    div a = 0; z(., .) skew; the stabilisation switch is continuous."""
    p = W.config2()
    topo = Topology(p["nsub"], p["widths"])
    A, _, _ = fem.element_matrices(p, topo)
    Asym = 0.5 * (A + A.transpose(0, 2, 1))
    Askw = 0.5 * (A - A.transpose(0, 2, 1))
    assert np.abs(Asym @ np.ones(8)).max() <= 1e-14 * np.abs(A).max()
    ev = np.linalg.eigvalsh(Asym[:200])
    assert ev.min() >= -1e-14 * np.abs(A).max()
    # skew part of a single element equals the convection form alone
    q = dict(p, nu=np.zeros_like(p["nu"]) + 1.0)
    q["beta0"] = np.zeros(3)
    Anob, _, _ = fem.element_matrices(q, topo)
    assert np.abs(0.5 * (Anob - Anob.transpose(0, 2, 1))).max() == 0.0
    assert np.abs(Askw).max() > 0
    # continuity of C_K at P_K = 1
    x0 = np.zeros((1, 3))
    h = np.array([0.1, 0.1, 0.1])
    hK = np.sqrt(0.03)
    an = np.linalg.norm(p["beta0"])
    nu1 = hK * an / 2
    c_lo, _ = fem.stabilisation(p, x0, h, np.array([nu1 * (1 + 1e-12)]))
    c_hi, _ = fem.stabilisation(p, x0, h, np.array([nu1 * (1 - 1e-12)]))
    assert abs(c_lo[0] - c_hi[0]) <= 1e-10 * c_hi[0]


def test_subassembly_equals_global_and_positive_real():
    p = W._problem((2, 3, 2), [[2, 3], [2, 2, 3], [3, 2]], np.linspace(0.01, 1, 5 * 7 * 5),
                   (3.0, -1.0, 2.0))
    topo = Topology(p["nsub"], p["widths"])
    Ag, bg = fem.assemble_global(p, topo)
    Ag = Ag.toarray()
    loc = fem.assemble_subdomains(p, topo)
    As = np.zeros_like(Ag)
    bs = np.zeros_like(bg)
    for s, (Al, fl) in enumerate(loc):
        dofs = topo.dof_of_node[topo.local_nodes(s)]
        As[np.ix_(dofs, dofs)] += Al
        bs[dofs] += fl
    assert np.abs(As - Ag).max() <= 1e-14 * np.abs(Ag).max()
    assert np.abs(bs - bg).max() <= 1e-14 * np.abs(bg).max()
    assert np.linalg.eigvalsh(Ag + Ag.T).min() > 0


def _l2_error(p, topo, u):
    """L2 norm of u_h - u* with u* = sin(pi x) sin(pi y) sin(pi z)."""
    x0, h, (ex, ey, ez) = fem.element_geometry(p, topo)
    nodes = fem.element_node_ids(topo, ex, ey, ez)
    full = np.zeros(topo.n_nodes)
    full[topo.free_nodes] = u
    ue = full[nodes]
    qp, qw = fem.gauss01(4)
    err = 0.0
    bits = np.arange(8)
    for i, s in enumerate(qp):
        for j, t in enumerate(qp):
            for k, r in enumerate(qp):
                phi = np.where(bits & 1, s, 1 - s) * np.where(bits & 2, t, 1 - t) * np.where(bits & 4, r, 1 - r)
                xq = x0 + np.array([s, t, r]) * h
                ex_ = np.prod(np.sin(np.pi * xq), axis=1)
                err += qw[i] * qw[j] * qw[k] * np.prod(h) * np.sum((ue @ phi - ex_) ** 2)
    return np.sqrt(err)


def test_manufactured_solution_rate():
    """L2 error of the stabilised Q1 solution decays like h^2 (diffusion
    dominated, C_K = tau h^2 / (4 nu))."""
    errs = []
    for hh in (2, 4, 8):
        p = W.manufactured(hh)
        topo = Topology(p["nsub"], p["widths"])
        A, b = fem.assemble_global(p, topo)
        u = spla.spsolve(A.tocsc(), b)
        errs.append(_l2_error(p, topo, u))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 1.8 <= rates[-1] <= 2.2, (errs, rates)
    assert np.all(rates > 1.6), (errs, rates)
