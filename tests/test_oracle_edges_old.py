"""Pins of the oracle's earlier edge eigenproblem (Section 3, eq. equ-4-8-E,
primal-constraints-E, Lemma lemma-E-1) against the mathematics: the parallel
sum of several matrices, the metric B_E dominating each of its terms, the
eigenproblem against a library solver, the constrained Rayleigh bound, the
estimate the lemma's proof establishes (with the constant the proof's
steps give), exactness when every dof is primal, brute force, and the
textbook lower bound in the symmetric case."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.linalg import eigh

from paper_2501_01676_amd import workloads as W
from oracle import bddc, fem

LOOSE_OLD = {"theta_face": 2.0, "theta_edge": 2.0, "edge_variant": "old"}


def _setup(p, opts):
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space(opts)
    return o


def _layered():
    p = W.uniform(2, 5, beta=(0.7, -0.4, 1.1))
    sx, sy, sz = W.element_subdomain(p["widths"])
    p["nu"] = np.where(sx == 0, 1.0, 1e-3) * np.where(sz == 0, 1.0, 0.1)
    return p


@pytest.fixture(scope="module")
def old_cases():
    """A layered 2x2x2 problem and a 3x3x3 one with a floating subdomain,
    both with low thresholds so edges select constraints and some do not."""
    return [_setup(_layered(), {**LOOSE_OLD, "theta_edge": 30.0}),
            _setup(W.random_field(3, 2, 7, beta=(2.0, -1.0, 0.5)), {**LOOSE_OLD, "theta_edge": 6.0})]


def test_parallel_sum_of_several():
    """A_1 : ... : A_m = (sum A_i^{-1})^{-1} for SPD A_i, independent of the
    order of the fold, below every A_i; with a common null vector the sum
    keeps it in its kernel."""
    rng = np.random.default_rng(11)
    n = 7
    mats = []
    for _ in range(4):
        X = rng.standard_normal((n, n))
        mats.append(X @ X.T + 0.2 * np.eye(n))
    P = bddc.parallel_sum_all(mats, 1e-13)
    ref = np.linalg.inv(sum(np.linalg.inv(A) for A in mats))
    assert np.abs(P - ref).max() <= 1e-11 * np.abs(ref).max()
    for perm in itertools.permutations(range(4)):
        Q = bddc.parallel_sum_all([mats[i] for i in perm], 1e-13)
        assert np.abs(Q - P).max() <= 1e-11 * np.abs(P).max()
    for A in mats:
        assert np.linalg.eigvalsh(A - P).min() >= -1e-11 * np.abs(P).max()
    # singular members with the constant vector in their kernel
    c = np.ones(n) / np.sqrt(n)
    Pc = np.eye(n) - np.outer(c, c)
    sing = [Pc @ A @ Pc for A in mats]
    S = bddc.parallel_sum_all(sing, 1e-10)
    assert np.linalg.norm(S @ c) <= 1e-10 * np.abs(S).max()
    # on the complement of c it is the parallel sum of the restrictions
    B = np.linalg.qr(np.column_stack([c, rng.standard_normal((n, n - 1))]))[0][:, 1:]
    red = np.linalg.inv(sum(np.linalg.inv(B.T @ A @ B) for A in sing))
    assert np.abs(B.T @ S @ B - red).max() <= 1e-9 * np.abs(red).max()


def test_metric_dominates_each_term(old_cases):
    """B_E is SPD and B_E - D_E^(k)^T B_E^(i) D_E^(k) is positive
    semidefinite for every ordered pair i != k of n(E) (B_E sums exactly
    those terms); Btilde_E lies below every member's Schur complement."""
    for o in old_cases:
        for k in o.topo.edges:
            aux = o.edge_aux[k]
            BE, subs = aux["BE"], aux["subs"]
            assert np.linalg.eigvalsh(BE).min() > 0
            scale = np.abs(BE).max()
            for i in subs:
                for kk in subs:
                    if kk == i:
                        continue
                    t = o.D[(k, kk)].T @ aux["BEi"][i] @ o.D[(k, kk)]
                    assert np.linalg.eigvalsh(BE - bddc.sym(t)).min() >= -1e-10 * scale
            for Bts in aux["Bts"]:
                assert np.linalg.eigvalsh(Bts - aux["Bt"]).min() >= -1e-10 * np.abs(Bts).max()


def test_eigenproblem_against_library(old_cases):
    """mu (reciprocal eigenvalues) equal scipy's for the pencil
    (Btilde_E, B_E); v^T B_E v = I; residual; Btilde_E-orthogonality across
    the selected / rejected split."""
    for o in old_cases:
        for k in o.topo.edges:
            aux = o.edge_aux[k]
            BE, Bt, X, mu = aux["BE"], aux["Bt"], aux["X"], o.edge_mu[k]
            ref = eigh(Bt, BE, eigvals_only=True)
            assert np.abs(np.sort(mu) - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
            V = np.linalg.solve(BE, X)
            assert np.abs(V.T @ BE @ V - np.eye(V.shape[1])).max() <= 1e-9
            assert np.abs(Bt @ V - BE @ V * mu).max() <= 1e-9 * np.abs(BE).max()
            sel = aux["sel"]
            cross = (Bt @ V[:, sel]).T @ V[:, ~sel]
            if cross.size:
                assert np.abs(cross).max() <= 1e-9 * np.abs(Bt).max()


def _constrained_edge_values(o, k, rng):
    """Edge values w_i,E (i in n(E)) satisfying eq. primal-constraints-E:
    a common part plus differences in range(Q_E^perp)."""
    T, p = o.edge_T[k], o.edge_r[k]
    n = T.shape[0]
    c = rng.standard_normal(n)
    return {s: c + T[:, p:] @ rng.standard_normal(n - p) for s in o.topo.objects[k]["subs"]}


def test_constrained_rayleigh_and_key_estimate(old_cases):
    """On the constrained differences x in range(Q_E^perp),
    x^T B_E x <= Theta_E x^T Btilde_E x; for constrained edge values the
    double sum of the proof of Lemma E-1 is at most 4 Theta_E
    sum_i w_i,E^T Btilde_E w_i,E, and the lemma's left-hand side is at most
    (|n(E)| - 1) 4 Theta_E sum_i w_i^T B^(i) w_i.  (The printed lemma states
    2 Theta_E: its proof drops the (|n(E)| - 1) of the Cauchy-Schwarz step and
    bounds two sums of the form sum_i sum_{k != i} by one B_E each.)"""
    rng = np.random.default_rng(12)
    checked = 0
    for o in old_cases:
        th = o.opt["theta_edge"]
        for k in o.topo.edges:
            aux = o.edge_aux[k]
            BE, Bt, subs = aux["BE"], aux["Bt"], aux["subs"]
            T, p = o.edge_T[k], o.edge_r[k]
            Qp = T[:, p:]
            if Qp.shape[1]:
                mu = eigh(Qp.T @ Bt @ Qp, Qp.T @ BE @ Qp, eigvals_only=True)
                assert mu.min() >= (1.0 / th) * (1 - 1e-9)
            m = len(subs)
            for _ in range(4):
                wE = _constrained_edge_values(o, k, rng)
                dbl = sum((wE[i] - wE[kk]) @ o.D[(k, kk)].T @ aux["BEi"][i] @ o.D[(k, kk)] @ (wE[i] - wE[kk])
                          for i in subs for kk in subs if kk != i)
                assert dbl <= 4 * th * sum(wE[i] @ Bt @ wE[i] for i in subs) * (1 + 1e-10) + 1e-14
                # full local vectors with these edge values
                w = {}
                for s in subs:
                    ws = rng.standard_normal(o.topo.sub[s]["nB"])
                    ws[o.topo.sub[s]["obj_local"][k]] = wE[s]
                    w[s] = ws
                lhs = 0.0
                for i in subs:
                    v = sum(o.D[(k, j)] @ (wE[i] - wE[j]) for j in subs)
                    lhs += v @ aux["BEi"][i] @ v
                rhs = (m - 1) * 4 * th * sum(w[s] @ o.B[s] @ w[s] for s in subs)
                assert lhs <= rhs * (1 + 1e-10)
                checked += 1
    assert checked > 0
    assert any(o.counts["pnum_edge"] > 0 for o in old_cases)
    assert any(0 < o.edge_r[k] < o.topo.objects[k]["nodes"].size for o in old_cases for k in o.topo.edges)


def test_faces_are_shared_with_the_new_variant():
    """The face stage does not depend on the edge variant: identical face
    counts and face bases (the printed tables give the same pnumF for both
    methods)."""
    p = _layered()
    o_old = _setup(p, LOOSE_OLD)
    o_new = _setup(p, {**LOOSE_OLD, "edge_variant": "new"})
    assert o_old.counts["pnum_face"] == o_new.counts["pnum_face"]
    for k in o_old.topo.faces:
        assert np.array_equal(o_old.face_T[k], o_new.face_T[k])


def test_all_primal_is_exact_old():
    """Theta -> 0+ with the earlier edge eigenproblem: every edge dof primal
    (one constraint per eigenvector), M^{-1} = Shat^{-1}, one step."""
    o = _setup(W.random_field(3, 2, 7, beta=(2.0, -1.0, 0.5)),
               {"theta_face": 1e-12, "theta_edge": 1e-12, "edge_variant": "old"})
    assert o.counts["pnum_edge"] == sum(o.topo.objects[k]["nodes"].size for k in o.topo.edges)
    assert o.counts["n_primal"] == o.topo.n_gamma
    _, info = o.gmres_solve(rtol=1e-12)
    assert info["iters"] == 1


@pytest.mark.parametrize("name", ["config1b", "floating"])
def test_solution_matches_direct_solve_old(name):
    p = W.random_field(3, 2, 7, beta=(2.0, -1.0, 0.5)) if name == "floating" else W.get(name)
    o, info = bddc.solve(p, {"edge_variant": "old", "theta_edge": 3.0}, rtol=1e-13, maxit=300)
    A, b = fem.assemble_global(p, o.topo)
    u = spla.spsolve(A.tocsc(), b)
    assert info["relres_true"] <= 1e-13
    assert np.linalg.norm(o.u - u) <= 1e-10 * np.linalg.norm(u)


def test_spd_case_lower_bound_old():
    """a = 0 (SPD): lambda_min(M^{-1} Shat) >= 1 and a real spectrum with the
    earlier edge constraints too."""
    p = W.random_field(3, 2, 3, lo=-2, hi=1, beta=(0.0, 0.0, 0.0))
    o = _setup(p, {"theta_face": 3.0, "theta_edge": 3.0, "edge_variant": "old"})
    n = o.topo.n_gamma
    S = np.stack([o.apply_schur(e) for e in np.eye(n)], 1)
    M = np.stack([o.apply_bddc(e) for e in np.eye(n)], 1)
    ev = np.linalg.eigvals(M @ S)
    assert np.abs(ev.imag).max() <= 1e-8
    assert ev.real.min() >= 1 - 1e-10


def test_metric_from_the_lemma_quadratic_form(old_cases):
    """The quadratic form of the proof of Lemma E-1,
    Q(w) = sum_i sum_{k != i} (w_i - w_k)^T D^(k)^T B_E^(i) D^(k) (w_i - w_k),
    evaluated on the unit jumps (x on subdomain a, 0 on the others) and
    summed over a, is 2 x^T B_E x."""
    rng = np.random.default_rng(13)
    for o in old_cases:
        for k in o.topo.edges[:6]:
            aux = o.edge_aux[k]
            subs, BE = aux["subs"], aux["BE"]
            for _ in range(3):
                x = rng.standard_normal(BE.shape[0])
                tot = 0.0
                for a in subs:
                    w = {s: (x if s == a else np.zeros_like(x)) for s in subs}
                    tot += sum((w[i] - w[kk]) @ o.D[(k, kk)].T @ aux["BEi"][i] @ o.D[(k, kk)] @ (w[i] - w[kk])
                               for i in subs for kk in subs if kk != i)
                assert abs(tot - 2 * x @ BE @ x) <= 1e-11 * abs(tot)


def test_member_schur_is_minimum_energy(old_cases):
    """Btilde_E^(nu) is the minimum of w^T B^(nu) w over the local vectors
    with w_E fixed, found here by a least-squares solve on a Cholesky factor
    of B^(nu) over the free coordinates."""
    rng = np.random.default_rng(14)
    for o in old_cases:
        for k in o.topo.edges[:4]:
            aux = o.edge_aux[k]
            for s, Bts in zip(aux["subs"], aux["Bts"]):
                B = o.B[s]
                n = B.shape[0]
                loc = o.topo.sub[s]["obj_local"][k]
                free = np.setdiff1d(np.arange(n), loc)
                ev, U = np.linalg.eigh(B)
                R = (U * np.sqrt(np.maximum(ev, 0.0))).T          # B = R^T R
                for _ in range(2):
                    x = rng.standard_normal(loc.size)
                    y, *_ = np.linalg.lstsq(R[:, free], -R[:, loc] @ x, rcond=None)
                    w = np.zeros(n)
                    w[loc], w[free] = x, y
                    assert abs(w @ B @ w - x @ Bts @ x) <= 1e-8 * abs(w @ B @ w)


def test_constraints_are_the_metric_images(old_cases):
    """Q_E spans {B_E v_l : l selected}: those vectors lie in range(Q_E),
    and range(Q_E) is orthogonal to every rejected eigenvector v_m (the
    paper's (B_E v_l)^T v_m = 0 for l != m)."""
    for o in old_cases:
        for k in o.topo.edges:
            aux = o.edge_aux[k]
            BE, X, sel = aux["BE"], aux["X"], aux["sel"]
            T, p = o.edge_T[k], o.edge_r[k]
            assert p == int(sel.sum())
            V = np.linalg.solve(BE, X)
            Q = T[:, :p]
            if p:
                C = X[:, sel]
                assert np.abs(C - Q @ (Q.T @ C)).max() <= 1e-10 * np.abs(C).max()
                if (~sel).any():
                    assert np.abs(Q.T @ V[:, ~sel]).max() <= 1e-9 * np.abs(V).max()
