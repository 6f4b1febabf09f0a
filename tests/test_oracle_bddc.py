"""Pins of the oracle's BDDC machinery (Section 3) against brute force,
degenerate special cases, textbook properties, the paper's identities and
inequalities, and invariances."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.linalg import eigh

from paper_2501_01676_amd import workloads as W
from oracle import bddc, fem

LOOSE = {"theta_face": 2.0, "theta_edge": 2.0}


def _setup(p, opts=None):
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space(opts)
    return o


@pytest.fixture(scope="module")
def small_loose():
    """2x2x2, H/h = 5, with low thresholds so faces and edges select modes."""
    p = W.uniform(2, 5, beta=(0.7, -0.4, 1.1))
    sx, sy, sz = W.element_subdomain(p["widths"])
    p["nu"] = np.where(sx == 0, 1.0, 1e-3) * np.where(sz == 0, 1.0, 0.1)
    return _setup(p, LOOSE)


@pytest.fixture(scope="module")
def floating():
    """3x3x3, H/h = 2 (one floating subdomain), random viscosity."""
    return _setup(W.random_field(3, 2, 7, beta=(2.0, -1.0, 0.5)), LOOSE)


# ------------------------------------------------------- end-to-end brute force
@pytest.mark.parametrize("name", ["config1a", "config1b", "floating"])
def test_solution_matches_direct_solve(name):
    p = W.random_field(3, 2, 7, beta=(2.0, -1.0, 0.5)) if name == "floating" else W.get(name)
    o, info = bddc.solve(p, rtol=1e-13, maxit=300)
    A, b = fem.assemble_global(p, o.topo)
    u = spla.spsolve(A.tocsc(), b)
    assert info["relres_true"] <= 1e-13
    assert np.linalg.norm(o.u - u) <= 1e-10 * np.linalg.norm(u)


def test_all_primal_is_exact():
    """Theta -> 0+: every eigenvector selected, every interface dof primal,
    Wtilde = What and M^{-1} = Shat^{-1}: GMRES converges in one step."""
    o = _setup(W.config1a(), {"theta_face": 1e-12, "theta_edge": 1e-12})
    assert o.counts["n_primal"] == o.topo.n_gamma
    r = np.random.default_rng(1).standard_normal(o.topo.n_gamma)
    assert np.linalg.norm(o.apply_schur(o.apply_bddc(r)) - r) <= 1e-12 * np.linalg.norm(r)
    _, info = o.gmres_solve(rtol=1e-12)
    assert info["iters"] == 1


@pytest.mark.parametrize("nsub,hh", [(3, 2), (2, 3)])
def test_spd_case_lower_bound(nsub, hh):
    """a = 0 (SPD): BDDC with any partition-of-unity scaling has
    lambda_min(M^{-1} Shat) >= 1 and a real spectrum."""
    p = W.random_field(nsub, hh, 3, lo=-2, hi=1, beta=(0.0, 0.0, 0.0))
    o = _setup(p, {"theta_face": 3.0, "theta_edge": 3.0})
    n = o.topo.n_gamma
    S = np.stack([o.apply_schur(e) for e in np.eye(n)], 1)
    M = np.stack([o.apply_bddc(e) for e in np.eye(n)], 1)
    ev = np.linalg.eigvals(M @ S)
    assert np.abs(ev.imag).max() <= 1e-8
    assert ev.real.min() >= 1 - 1e-10


def test_explicit_partially_assembled_space(small_loose):
    """M^{-1} r from block elimination equals Rtilde^T Dtilde Stilde^{-1}
    Dtilde^T Rtilde r built with dense matrices on the explicit space Wtilde
    (local dual coordinates, shared primal coordinates)."""
    o = small_loose
    topo = o.topo
    nB = [topo.sub[s]["nB"] for s in range(topo.n_sub)]
    offs = np.concatenate([[0], np.cumsum(nB)])
    nD = [o.Delta_loc[s].size for s in range(topo.n_sub)]
    doffs = np.concatenate([[0], np.cumsum(nD)])
    ncoord = doffs[-1] + o.n_primal
    N = np.zeros((offs[-1], ncoord))
    Rst = np.zeros((offs[-1], topo.n_gamma))
    Sst = np.zeros((offs[-1], offs[-1]))
    Dst = np.zeros((offs[-1], offs[-1]))
    for s in range(topo.n_sub):
        T = o.T[s]
        rows = slice(offs[s], offs[s + 1])
        N[rows, doffs[s]:doffs[s + 1]] = T[:, o.Delta_loc[s]]
        N[rows, doffs[-1] + o.Pi_gid[s]] += T[:, o.Pi_loc[s]]
        Rst[np.arange(offs[s], offs[s + 1]), topo.sub[s]["gamma"]] = 1.0
        Sst[rows, rows] = o.S[s]
        Dst[rows, rows] = o.Dmat[s]
    Rt = np.linalg.lstsq(N, Rst, rcond=None)[0]
    assert np.abs(N @ Rt - Rst).max() <= 1e-12
    St = N.T @ Sst @ N
    Dt = N.T @ Dst @ N
    Minv = Rt.T @ Dt @ np.linalg.solve(St, Dt.T @ Rt)
    r = np.random.default_rng(2).standard_normal(topo.n_gamma)
    z = o.apply_bddc(r)
    assert np.linalg.norm(z - Minv @ r) <= 1e-11 * np.linalg.norm(z)


# ------------------------------------------------------------ paper identities
def test_partition_of_unity(small_loose, floating):
    for o in (small_loose, floating):
        for k, obj in enumerate(o.topo.objects):
            tot = sum(o.D[(k, s)] for s in obj["subs"])
            assert np.abs(tot - np.eye(tot.shape[0])).max() <= 1e-12


def test_face_jump_identity(small_loose):
    """sum_i (w_i - sum_k D_k w_k)^T B_F^(i) (...) = (w_i - w_j)^T B_F (w_i - w_j)."""
    o = small_loose
    rng = np.random.default_rng(3)
    for k in o.topo.faces:
        i, j = o.topo.objects[k]["subs"]
        Di, Dj = o.D[(k, i)], o.D[(k, j)]
        BFi, BFj = o._block(o.B[i], i, k), o._block(o.B[j], j, k)
        wi, wj = rng.standard_normal((2, Di.shape[0]))
        avg = Di @ wi + Dj @ wj
        lhs = (wi - avg) @ BFi @ (wi - avg) + (wj - avg) @ BFj @ (wj - avg)
        d = wi - wj
        rhs = d @ o.face_aux[k]["BF"] @ d
        assert abs(lhs - rhs) <= 1e-11 * abs(rhs)


def test_edge_change_of_unknowns_identities(small_loose):
    """w_1 = -sum_{k>=2} D_k wcheck_k + what, w_k - what = That_k wcheck and
    sum_k (w_k - what)^T B_E^(k) (w_k - what) = wcheck^T M_E wcheck."""
    o = small_loose
    rng = np.random.default_rng(4)
    for k in o.topo.edges:
        a = o.edge_aux[k]
        m, nE, Ds = a["m"], a["nE"], a["Ds"]
        w = rng.standard_normal((m, nE))
        what = sum(Ds[q] @ w[q] for q in range(m))
        wch = np.concatenate([w[q] - w[0] for q in range(1, m)])
        w1 = -sum(Ds[q] @ (w[q] - w[0]) for q in range(1, m)) + what
        assert np.abs(w1 - w[0]).max() <= 1e-12 * np.abs(w).max()
        for q in range(m):
            assert np.abs(a["That"][q] @ wch - (w[q] - what)).max() <= 1e-12 * np.abs(w).max()
        lhs = sum((w[q] - what) @ a["BE"][q] @ (w[q] - what) for q in range(m))
        assert abs(lhs - wch @ a["ME"] @ wch) <= 1e-11 * abs(lhs)


def test_parallel_sum_and_schur_minimum_energy(small_loose):
    rng = np.random.default_rng(5)
    n = 6
    X, Y = rng.standard_normal((2, n, n))
    A, B = X @ X.T + 0.1 * np.eye(n), Y @ Y.T + 0.1 * np.eye(n)
    P = bddc.parallel_sum(A, B, 1e-12)
    assert np.abs(P - np.linalg.inv(np.linalg.inv(A) + np.linalg.inv(B))).max() <= 1e-12 * np.abs(P).max()
    assert np.abs(P - bddc.parallel_sum(B, A, 1e-12)).max() <= 1e-12 * np.abs(P).max()
    assert np.linalg.eigvalsh(A - P).min() >= -1e-12 and np.linalg.eigvalsh(B - P).min() >= -1e-12
    o = small_loose
    for k in o.topo.faces[:4]:
        i, j = o.topo.objects[k]["subs"]
        loc = o.topo.sub[i]["obj_local"][k]
        for _ in range(5):
            w = rng.standard_normal(o.topo.sub[i]["nB"])
            assert w @ o.B[i] @ w >= w[loc] @ o.face_aux[k]["Bti"] @ w[loc] * (1 - 1e-12)
        Bt = o.face_aux[k]["Bt"]
        assert np.linalg.eigvalsh(o.face_aux[k]["Bti"] - Bt).min() >= -1e-10 * np.abs(Bt).max()


def test_gep_residual_and_normalisation(small_loose):
    """B_F v = lambda Btilde_F v in reciprocal form, v^T B_F v = I and
    Btilde_F-orthogonality across the selected / rejected split."""
    o = small_loose
    for k in o.topo.faces:
        aux = o.face_aux[k]
        BF, Bt, X, mu = aux["BF"], aux["Bt"], aux["X"], o.face_mu[k]
        V = np.linalg.solve(BF, X)            # v_l = B_F^{-1} (B_F v_l)
        assert np.abs(V.T @ BF @ V - np.eye(V.shape[1])).max() <= 1e-9
        res = Bt @ V - BF @ V * mu
        assert np.abs(res).max() <= 1e-9 * np.abs(BF).max()
        sel = aux["sel"]
        cross = (Bt @ V[:, sel]).T @ V[:, ~sel]
        if cross.size:
            assert np.abs(cross).max() <= 1e-9 * np.abs(Bt).max()
    for k in o.topo.edges:
        aux = o.edge_aux[k]
        ME, Btt, X, mu = aux["ME"], aux["BttE"], aux["X"], o.edge_mu[k]
        V = np.linalg.solve(ME, X)
        assert np.abs(V.T @ ME @ V - np.eye(V.shape[1])).max() <= 1e-9
        assert np.abs(Btt @ V - ME @ V * mu).max() <= 1e-9 * np.abs(ME).max()


def _max_quotient(A, B, Q):
    """max over span(Q) of x^T A x / x^T B x (B SPD on span(Q))."""
    if Q.shape[1] == 0:
        return 0.0
    return float(eigh(Q.T @ A @ Q, Q.T @ B @ Q, eigvals_only=True).max())


def test_face_constrained_rayleigh_and_lemma_F(small_loose):
    """On jumps satisfying the face constraints the generalized Rayleigh
    quotient (w_i - w_j)^T B_F (.) / (.)^T Btilde_F (.) is <= Theta_F (its
    maximum over the whole constrained subspace), and Lemma F's 2 Theta_F
    bound holds for random constrained w."""
    o = small_loose
    th = o.opt["theta_face"]
    rng = np.random.default_rng(6)
    for k in o.topo.faces:
        aux = o.face_aux[k]
        T, p = o.face_T[k], o.face_p[k]
        # reciprocal form: min of Btilde_F / B_F on the constrained space >= 1/Theta
        if p < T.shape[0]:
            Qp = T[:, p:]
            mu = eigh(Qp.T @ aux["Bt"] @ Qp, Qp.T @ aux["BF"] @ Qp, eigvals_only=True)
            assert mu.min() >= (1.0 / th) * (1 - 1e-9)
        # the rejected eigenvectors' constraint vectors lie in range(Q_F^perp) ... and the
        # selected ones in range(Q_F)
        Xs = aux["X"][:, aux["sel"]]
        if p:
            assert np.abs(T[:, p:].T @ Xs).max() <= 1e-10 * np.abs(Xs).max()
        i, j = o.topo.objects[k]["subs"]
        for _ in range(4):
            d = T[:, p:] @ rng.standard_normal(T.shape[0] - p)
            wi = rng.standard_normal(o.topo.sub[i]["nB"])
            wj = rng.standard_normal(o.topo.sub[j]["nB"])
            li, lj = o.topo.sub[i]["obj_local"][k], o.topo.sub[j]["obj_local"][k]
            wi[li] = wj[lj] + d
            Di, Dj = o.D[(k, i)], o.D[(k, j)]
            avg = Di @ wi[li] + Dj @ wj[lj]
            lhs = sum((w[l] - avg) @ o._block(o.B[s], s, k) @ (w[l] - avg)
                      for w, l, s in ((wi, li, i), (wj, lj, j)))
            rhs = 2 * th * (wi @ o.B[i] @ wi + wj @ o.B[j] @ wj)
            assert lhs <= rhs * (1 + 1e-10)


def test_edge_constrained_rayleigh(small_loose):
    """Jumps orthogonal to the constraint vectors M_E v_l satisfy
    wcheck^T M_E wcheck <= Theta_E wcheck^T Btilde~_E wcheck (maximum over
    the constrained subspace); the SVD+QR basis realises the constraints:
    Q_E^T wcheck_k = 0 for every block implies (M_E v_l)^T wcheck = 0, and
    the bound holds on that smaller subspace too."""
    o = small_loose
    th = o.opt["theta_edge"]
    nsel_total = 0
    for k in o.topo.edges:
        aux = o.edge_aux[k]
        sel, X = aux["sel"], aux["X"]
        nsel_total += int(sel.sum())
        C = X[:, sel]
        n = X.shape[0]
        U, sv, _ = np.linalg.svd(C) if C.shape[1] else (np.eye(n), np.zeros(0), None)
        Nc = U[:, C.shape[1]:]                       # orthogonal complement of range(C)
        mu = eigh(Nc.T @ aux["BttE"] @ Nc, Nc.T @ aux["ME"] @ Nc, eigvals_only=True)
        assert mu.min() >= (1.0 / th) * (1 - 1e-9)
        T, r, nE, m = o.edge_T[k], o.edge_r[k], aux["nE"], aux["m"]
        Qp = np.kron(np.eye(m - 1), T[:, r:])        # blocks in range(Q_E^perp)
        if C.shape[1] and Qp.shape[1]:
            assert np.abs(C.T @ Qp).max() <= 1e-10 * np.abs(C).max()
        if Qp.shape[1]:
            mu2 = eigh(Qp.T @ aux["BttE"] @ Qp, Qp.T @ aux["ME"] @ Qp, eigvals_only=True)
            assert mu2.min() >= (1.0 / th) * (1 - 1e-9)
    assert nsel_total > 0


def test_edge_schur_is_constrained_minimum_energy(small_loose):
    """wcheck^T Btilde~_E wcheck equals the minimum of sum_k w_k^T B^(k) w_k
    over whole local interface vectors w_k whose edge values have the jumps
    wcheck and whose prior-selected primal unknowns (vertex values and face
    primal coordinates Q_F^T w_F) agree between the subdomains sharing them
    (the quantity bounded below eq. estimate-key-E-3, solved as a KKT system)."""
    o = small_loose
    topo = o.topo
    rng = np.random.default_rng(11)
    for k in topo.edges:
        aux = o.edge_aux[k]
        subs, nE, m = aux["subs"], aux["nE"], aux["m"]
        nB = [topo.sub[s]["nB"] for s in subs]
        offs = np.concatenate([[0], np.cumsum(nB)])
        ntot = offs[-1]
        Bbig = np.zeros((ntot, ntot))
        for a, s in enumerate(subs):
            Bbig[offs[a]:offs[a + 1], offs[a]:offs[a + 1]] = o.B[s]
        wch = rng.standard_normal((m - 1) * nE)
        rows, rhs = [], []
        E0 = offs[0] + topo.sub[subs[0]]["obj_local"][k]
        for a in range(1, m):
            Ea = offs[a] + topo.sub[subs[a]]["obj_local"][k]
            for q in range(nE):
                c = np.zeros(ntot)
                c[Ea[q]] += 1.0
                c[E0[q]] -= 1.0
                rows.append(c)
                rhs.append(wch[(a - 1) * nE + q])
        for kk, obj in enumerate(topo.objects):
            share = [a for a, s in enumerate(subs) if s in obj["subs"]]
            if len(share) < 2 or obj["kind"] == "edge":
                continue
            for a, b in zip(share[:-1], share[1:]):
                la = offs[a] + topo.sub[subs[a]]["obj_local"][kk]
                lb = offs[b] + topo.sub[subs[b]]["obj_local"][kk]
                if obj["kind"] == "vertex":
                    funcs = np.eye(1)
                else:
                    funcs = o.face_T[kk][:, :o.face_p[kk]].T
                for f in funcs:
                    c = np.zeros(ntot)
                    c[la] += f
                    c[lb] -= f
                    rows.append(c)
                    rhs.append(0.0)
        Cm = np.array(rows)
        K = np.block([[2 * Bbig, Cm.T], [Cm, np.zeros((len(rows), len(rows)))]])
        sol = np.linalg.lstsq(K, np.concatenate([np.zeros(ntot), rhs]), rcond=None)[0]
        x = sol[:ntot]
        assert np.abs(Cm @ x - rhs).max() <= 1e-9
        emin = x @ Bbig @ x
        assert abs(emin - wch @ aux["BttE"] @ wch) <= 1e-8 * emin


def test_edge_count_structure(small_loose):
    """Generic rank of the edge constraint blocks: r_E = min(n_E, (|n(E)|-1) |N_E|)."""
    o = small_loose
    seen = set()
    for k in o.topo.edges:
        a = o.edge_aux[k]
        r = o.edge_r[k]
        assert r == min(a["nE"], (a["m"] - 1) * o.edge_nsel[k])
        seen.add(o.edge_nsel[k])
    assert len(seen) >= 2


# ----------------------------------------------------------------- invariances
def test_edge_reference_invariance():
    p = W.uniform(2, 5, beta=(0.7, -0.4, 1.1))
    sx, _, sz = W.element_subdomain(p["widths"])
    p["nu"] = np.where(sx == 0, 1.0, 1e-3) * np.where(sz == 0, 1.0, 0.1)
    o0 = _setup(p, LOOSE)
    o2 = _setup(p, dict(LOOSE, edge_ref=2))
    for k in o0.topo.edges:
        assert np.allclose(np.sort(o0.edge_mu[k]), np.sort(o2.edge_mu[k]), rtol=1e-9, atol=1e-12)
        r = o0.edge_r[k]
        assert r == o2.edge_r[k]
        P0 = o0.edge_T[k][:, :r] @ o0.edge_T[k][:, :r].T
        P2 = o2.edge_T[k][:, :r] @ o2.edge_T[k][:, :r].T
        assert np.abs(P0 - P2).max() <= 1e-9


def test_basis_choice_invariance(small_loose):
    """M^{-1} r depends on span(Q_X) only, not on the orthonormal bases
    chosen inside span(Q_X) and its complement."""
    o = small_loose
    r = np.random.default_rng(8).standard_normal(o.topo.n_gamma)
    z0 = o.apply_bddc(r)
    rng = np.random.default_rng(9)
    saved = dict(o.face_T)
    for k in o.topo.faces:
        T, p = o.face_T[k], o.face_p[k]
        G1, _ = np.linalg.qr(rng.standard_normal((p, p))) if p else (np.zeros((0, 0)), None)
        G2, _ = np.linalg.qr(rng.standard_normal((T.shape[0] - p,) * 2))
        o.face_T[k] = np.concatenate([T[:, :p] @ G1, T[:, p:] @ G2], axis=1)
    o._change_of_basis()
    o._coarse()
    z1 = o.apply_bddc(r)
    o.face_T.update(saved)
    o._change_of_basis()
    o._coarse()
    assert np.linalg.norm(z1 - z0) <= 1e-10 * np.linalg.norm(z0)


# ---------------------------------------------------------------------- GMRES
def test_gmres_full_space_and_monotone():
    rng = np.random.default_rng(10)
    n = 25
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    b = rng.standard_normal(n)
    Mi = np.linalg.inv(A + 0.3 * rng.standard_normal((n, n)))
    x, info = bddc.gmres(lambda v: A @ v, lambda v: Mi @ v, b, restart=n, rtol=1e-13, maxit=n)
    assert info["iters"] <= n
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)
    h = np.array(info["history"])
    assert np.all(np.diff(h) <= 1e-14)
    # the Arnoldi basis stays orthonormal to working precision (Gram-Schmidt
    # applied twice) even for an ill-conditioned operator
    B = np.diag(np.logspace(0, 12, n)) + np.triu(rng.standard_normal((n, n)), 1)
    _, info3 = bddc.gmres(lambda v: B @ v, lambda v: v, b, restart=n, rtol=1e-15, maxit=n,
                          keep_basis=True)
    V = info3["basis"]
    assert np.abs(V @ V.T - np.eye(V.shape[0])).max() <= 1e-13
    # restarted run still converges and reports true residual
    x2, info2 = bddc.gmres(lambda v: A @ v, lambda v: v, b, restart=5, rtol=1e-10, maxit=400)
    assert info2["relres_true"] <= 1e-10 and info2["restarts"] >= 1


def test_options_variants_run():
    p = W.config1a()
    for opts in ({"edge_h_mode": "separate"}, {"deluxe_source": "B"}):
        o, info = bddc.solve(p, dict(LOOSE, **opts), rtol=1e-10)
        assert info["relres_true"] <= 1e-10


# ------------------------------------------------------------- deluxe weights
def _schur_by_inverse(p, o):
    """S^(k) formed apart from the oracle's elimination, from the local
    matrices of the finite-element assembly: by the block-inverse formula
    the boundary block of (A^(k))^{-1} is (S^(k))^{-1}; a floating subdomain
    (A^(k) singular) takes A_BB - A_BI A_II^{-1} A_IB with an LU of A_II."""
    from scipy.linalg import lu_factor, lu_solve
    local = fem.assemble_subdomains(p, o.topo, 3)
    out = []
    for s, (Al, _) in enumerate(local):
        nI = o.topo.sub[s]["nI"]
        if np.linalg.cond(Al) < 1e12:
            out.append(np.linalg.inv(np.linalg.inv(Al)[nI:, nI:]))
        else:
            X = lu_solve(lu_factor(Al[:nI, :nI]), Al[:nI, nI:])
            out.append(Al[nI:, nI:] - Al[nI:, :nI] @ X)
    return out


def _obj_block(M, o, s, k):
    loc = o.topo.sub[s]["obj_local"][k]
    return M[np.ix_(loc, loc)]


@pytest.mark.parametrize("nsub,hh", [(2, 4), (3, 3)])
def test_deluxe_average_minimises_weighted_jump(nsub, hh):
    """Deluxe scaling (Section 3) with a = 0: every S^(k) is symmetric and
    S_XX^(k) positive definite, and the deluxe average
    what = sum_k D_X^(k) w_k is the unique minimiser of
    sum_k (w_k - what)^T S_XX^(k) (w_k - what).  The minimiser is found here
    as a least-squares problem with the Cholesky factors of the blocks, on
    random w_k, for every face and edge (two and four subdomains)."""
    p = W.random_field(nsub, hh, 11, lo=-2, hi=1, beta=(0.0, 0.0, 0.0))
    o = _setup(p, {"theta_face": 10.0, "theta_edge": 10.0})
    S = _schur_by_inverse(p, o)
    rng = np.random.default_rng(5)
    checked = 0
    for k, obj in enumerate(o.topo.objects):
        if obj["kind"] == "vertex":
            continue
        subs = list(obj["subs"])
        n = obj["nodes"].size
        blocks = [_obj_block(S[s], o, s, k) for s in subs]
        w = [rng.standard_normal(n) for _ in subs]
        C = [np.linalg.cholesky(0.5 * (b + b.T)).T for b in blocks]      # S_XX^(k) = C^T C
        lhs = np.concatenate(C, axis=0)
        rhs = np.concatenate([c @ wk for c, wk in zip(C, w)])
        wmin = np.linalg.lstsq(lhs, rhs, rcond=None)[0]
        what = sum(o.D[(k, s)] @ wk for s, wk in zip(subs, w))
        assert np.linalg.norm(what - wmin) <= 1e-10 * np.linalg.norm(wmin), (obj["kind"], k)
        checked += 1
    assert checked == len(o.topo.faces) + len(o.topo.edges)


@pytest.mark.parametrize("source", ["S", "B"])
def test_deluxe_weight_equation_nonsymmetric(source):
    """Deluxe scaling (Section 3) with a != 0: D_X^(k) solves
    (sum_j M_XX^(j)) D_X^(k) = M_XX^(k) with M = S^(j) (nonsymmetric) or
    M = B^(j) = sym S^(j), the blocks taken from Schur complements formed
    apart from the oracle (block-inverse formula); faces and edges."""
    p = W.random_field(2, 4, 13, lo=-2, hi=0, beta=(3.0, -2.0, 1.5))
    o = _setup(p, {"theta_face": 10.0, "theta_edge": 10.0, "deluxe_source": source})
    S = _schur_by_inverse(p, o)
    M = S if source == "S" else [0.5 * (s + s.T) for s in S]
    for k, obj in enumerate(o.topo.objects):
        if obj["kind"] == "vertex":
            continue
        subs = list(obj["subs"])
        blocks = [_obj_block(M[s], o, s, k) for s in subs]
        tot = sum(blocks)
        asym = max(np.abs(b - b.T).max() / np.abs(b).max() for b in blocks)
        if source == "S":
            assert asym > 1e-6     # the blocks are genuinely nonsymmetric here
        for s, blk in zip(subs, blocks):
            assert np.abs(tot @ o.D[(k, s)] - blk).max() <= 1e-11 * np.abs(blk).max(), (obj["kind"], k, s)
