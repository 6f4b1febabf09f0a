"""GPU tests of the batched dense primitives the setup is built from, against
plain numpy on the same inputs (FP64: 1e-12 relative; FP32: 1e-4)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_01676_amd import api
    return api


def _posreal(n, rng, skew=3.0):
    X = rng.standard_normal((n, n))
    Z = rng.standard_normal((n, n))
    return X @ X.T / n + np.eye(n) + skew * (Z - Z.T) / np.sqrt(n)


@pytest.mark.parametrize("transA,transB", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_matches_numpy(transA, transB):
    api = _api()
    rng = np.random.default_rng(0)
    # tiled shapes, and thin ones (k <= 32 with n <= 32 or m <= 32) that take
    # the streaming kernel: tall, wide, both sides at the limit, single rows
    shapes = [(1, 1, 1), (16, 16, 4), (63, 65, 33), (130, 70, 97), (5, 200, 64),
              (300, 7, 7), (7, 300, 7), (257, 32, 32), (32, 513, 31), (1, 100, 1), (700, 3, 20), (40, 33, 32)]
    for alpha, beta in ((-0.5, 2.0), (1.5, 0.0)):
        As, Bs, Cs, ref = [], [], [], []
        for m, n, k in shapes:
            A = rng.standard_normal((k, m) if transA else (m, k))
            B = rng.standard_normal((n, k) if transB else (k, n))
            Cm = rng.standard_normal((m, n))
            As.append(A); Bs.append(B); Cs.append(Cm)
            ref.append(alpha * (A.T if transA else A) @ (B.T if transB else B) + beta * Cm)
        out = api.gemm(As, Bs, Cs, transA, transB, alpha=alpha, beta=beta)
        for (m, n, k), o, r in zip(shapes, out, ref):
            assert np.abs(o - r).max() <= 1e-12 * max(1.0, np.abs(r).max()), (m, n, k, alpha, beta)


@pytest.mark.parametrize("precision", [0, 1])
def test_partial_lu_schur_complement(precision):
    api = _api()
    rng = np.random.default_rng(1)
    # (nrow, ncol, k): ragged batch; k around the 64-column panels and their
    # pairs (64, 65, 128, 129, 192, 256), wide and tall matrices
    cases = [(5, 7, 3), (64, 65, 64), (100, 101, 37), (200, 203, 131), (300, 300, 300), (260, 140, 128),
             (129, 300, 129), (321, 257, 192), (190, 190, 65), (257, 257, 256)]
    mats, ks, refs = [], [], []
    for nr, nc, k in cases:
        M = rng.standard_normal((nr, nc))
        M[:k, :k] = _posreal(k, rng)
        mats.append(M); ks.append(k)
        A11, A12, A21, A22 = M[:k, :k], M[:k, k:], M[k:, :k], M[k:, k:]
        refs.append(A22 - A21 @ np.linalg.solve(A11, A12))
    out = api.partial_lu(mats, ks, precision)
    tol = 1e-11 if precision == 0 else 2e-4
    for o, k, r in zip(out, ks, refs):
        S = o[k:, k:]
        if r.size:
            assert np.abs(S - r).max() <= tol * max(1.0, np.abs(r).max())
    # the factors reproduce A11 = L U, A21 = L21 U, A12 = L U12
    ftol = 1e-11 if precision == 0 else 1e-4
    for o, k, M in zip(out, ks, mats):
        L = np.tril(o[:k, :k], -1) + np.eye(k)
        U = np.triu(o[:k, :k])
        scale = np.abs(M).max()
        assert np.abs(L @ U - M[:k, :k]).max() <= ftol * scale
        if M.shape[0] > k:
            assert np.abs(o[k:, :k] @ U - M[k:, :k]).max() <= ftol * scale
        if M.shape[1] > k:
            assert np.abs(L @ o[:k, k:] - M[:k, k:]).max() <= ftol * scale


def test_partial_lu_large_batch():
    """A ragged batch of 140 matrices (more diagonal-block workgroups than
    half the CUs, running beside the band / lead tiles) against numpy."""
    api = _api()
    rng = np.random.default_rng(5)
    mats, ks, refs = [], [], []
    for b in range(140):
        n = int(rng.integers(70, 210))
        k = int(rng.integers(1, n - 5))
        M = rng.standard_normal((n, n + 3))
        M[:k, :k] = _posreal(k, rng)
        mats.append(M); ks.append(k)
        refs.append(M[k:, k:] - M[k:, :k] @ np.linalg.solve(M[:k, :k], M[:k, k:]))
    out = api.partial_lu(mats, ks, 0)
    for o, k, r in zip(out, ks, refs):
        assert np.abs(o[k:, k:] - r).max() <= 1e-11 * max(1.0, np.abs(r).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_partial_lu_long_eliminations(precision):
    """Batches whose longest elimination exceeds 512 pivots take the panels in
    groups of four (band updates at depth 64, 128, 192, lead at 256): a ragged
    batch with k on both sides of group and panel boundaries, against numpy."""
    api = _api()
    rng = np.random.default_rng(9)
    shapes = [(700, 705, 600), (650, 650, 513), (600, 610, 257), (300, 300, 256), (200, 205, 65), (90, 90, 1)]
    mats, ks, refs = [], [], []
    for n, m, k in shapes:
        M = rng.standard_normal((n, m))
        M[:k, :k] = _posreal(k, rng)
        mats.append(M); ks.append(k)
        refs.append(M[k:, k:] - M[k:, :k] @ np.linalg.solve(M[:k, :k], M[:k, k:]))
    out = api.partial_lu(mats, ks, precision)
    tol = 1e-11 if precision == 0 else 2e-3
    for o, k, r in zip(out, ks, refs):
        assert np.abs(o[k:, k:] - r).max() <= tol * max(1.0, np.abs(r).max())


def test_partial_lu_inverse_trick():
    """Schur complement of [[A, I], [-I, 0]] onto the trailing block is A^{-1}."""
    api = _api()
    rng = np.random.default_rng(2)
    n = 150
    A = _posreal(n, rng)
    M = np.block([[A, np.eye(n)], [-np.eye(n), np.zeros((n, n))]])
    out = api.partial_lu([M], [n])[0]
    assert np.abs(out[n:, n:] - np.linalg.inv(A)).max() <= 1e-10 * np.abs(np.linalg.inv(A)).max()


def _pinv_ref(S, rtol):
    lam, V = np.linalg.eigh(0.5 * (S + S.T))
    keep = lam > rtol * lam.max()
    return (V[:, keep] / lam[keep]) @ V[:, keep].T


def test_parallel_sum_lu_and_eigen_paths():
    """sym(A (A + B)^+ B) for a ragged batch mixing the three kinds of face:
    A + B well conditioned (LU path), singular (a shared null vector) and
    nonsingular with an eigenvalue below the cut (both eigenvalue path);
    orders on both sides of 64."""
    api = _api()
    rng = np.random.default_rng(5)
    rtol = 1e-10
    As, Bs, refs, kinds = [], [], [], []
    for i, n in enumerate((1, 7, 49, 64, 65, 100, 121, 128, 49, 121, 7, 96)):
        kind = i % 3 if n > 2 else 0
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        if kind == 0:
            s = rng.uniform(0.1, 1.0, n)
        elif kind == 1:
            s = np.concatenate([[0.0], rng.uniform(0.1, 1.0, n - 1)])
        else:
            s = np.concatenate([[1e-12], rng.uniform(0.1, 1.0, n - 1)])
        S = (Q * s) @ Q.T
        t = rng.uniform(0.3, 0.7)
        # a symmetric split of S that keeps its small eigenspace: E lives on
        # the span of the eigenvectors with s > 1e-3
        F = rng.standard_normal((n, n)) * 0.01
        P = Q[:, s > 1e-3] @ Q[:, s > 1e-3].T
        E = P @ (F + F.T) @ P
        A = t * S + E
        B = (1 - t) * S - E
        As.append(A); Bs.append(B); kinds.append(kind)
        refs.append(0.5 * ((A @ _pinv_ref(A + B, rtol) @ B) + (A @ _pinv_ref(A + B, rtol) @ B).T))
    out = api.parallel_sum(As, Bs, rtol)
    for o, r, kind in zip(out, refs, kinds):
        assert np.abs(o - r).max() <= 1e-11 * max(1.0, np.abs(r).max()), (kind, np.abs(o - r).max())


def test_schur_pinv_singular_and_regular_blocks():
    """M22 - M21 (sym M11)^+ M12 for a ragged batch: M11 positive definite
    (LU path), singular with a null space of dimension 1 or 3, indefinite
    (negative eigenvalues dropped), and k = 0 or k = nv."""
    api = _api()
    rng = np.random.default_rng(6)
    rtol = 1e-10
    mats, ks, refs = [], [], []
    cases = [(10, 4, "spd"), (74, 47, "null1"), (60, 33, "null3"), (90, 64, "indef"), (150, 100, "spd"),
             (150, 100, "null1"), (8, 0, "spd"), (12, 12, "spd"), (200, 128, "null1")]
    for nv, k, kind in cases:
        M = rng.standard_normal((nv, nv))
        if k:
            Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
            lam = rng.uniform(0.1, 1.0, k)
            if kind == "null1":
                lam[0] = 0.0
            elif kind == "null3":
                lam[:3] = 0.0
            elif kind == "indef":
                lam[:2] = -0.5
            M[:k, :k] = (Q * lam) @ Q.T
        mats.append(M); ks.append(k)
        if k:
            refs.append(M[k:, k:] - M[k:, :k] @ _pinv_ref(M[:k, :k], rtol) @ M[:k, k:])
        else:
            refs.append(M.copy())
    out = api.schur_pinv(mats, ks, rtol)
    for o, r, (nv, k, kind) in zip(out, refs, cases):
        if r.size:
            assert np.abs(o - r).max() <= 1e-10 * max(1.0, np.abs(r).max()), (nv, k, kind, np.abs(o - r).max())


def test_sygv_matches_eigen_equation():
    api = _api()
    rng = np.random.default_rng(3)
    As, Bs = [], []
    for n in (1, 2, 7, 21, 49, 64, 65, 100, 121, 128):
        X = rng.standard_normal((n, n))
        Y = rng.standard_normal((n, n))
        As.append(X @ X.T)
        Bs.append(Y @ Y.T + n * np.eye(n))
    ws, Xs = api.sygv(As, Bs)
    for A, B, w, X in zip(As, Bs, ws, Xs):
        ref = np.sort(np.linalg.eigvals(np.linalg.solve(B, A)).real)
        assert np.abs(w - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
        assert np.all(np.diff(w) >= 0)
        V = np.linalg.solve(B, X)     # X = B v
        assert np.abs(V.T @ B @ V - np.eye(len(w))).max() <= 1e-10
        assert np.abs(A @ V - B @ V * w).max() <= 1e-9 * np.abs(A).max()


def test_parallel_sum_large_orders():
    """Orders above 128 (the global-memory variants): sym(A (A + B)^+ B) with
    A + B well conditioned, against the eigenvalue pseudo-inverse."""
    api = _api()
    rng = np.random.default_rng(8)
    rtol = 1e-10
    As, Bs, refs = [], [], []
    for n in (129, 200, 384):
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        S = (Q * rng.uniform(0.1, 1.0, n)) @ Q.T
        F = rng.standard_normal((n, n)) * 0.01
        t = rng.uniform(0.3, 0.7)
        A = t * S + (F + F.T)
        B = (1 - t) * S - (F + F.T)
        As.append(A); Bs.append(B)
        R = A @ _pinv_ref(A + B, rtol) @ B
        refs.append(0.5 * (R + R.T))
    out = api.parallel_sum(As, Bs, rtol)
    for o, r in zip(out, refs):
        assert np.abs(o - r).max() <= 1e-11 * max(1.0, np.abs(r).max()), np.abs(o - r).max()


def test_sygv_select_eigenvalues_and_selected_vectors():
    """Tridiagonalisation + bisection + inverse iteration: every eigenvalue,
    and B-orthonormal eigenvectors (X = B V) for mu <= sel, including
    multiple eigenvalues across the selection (clusters) and singular A."""
    api = _api()
    rng = np.random.default_rng(4)
    sel = 0.1
    As, Bs, mus = [], [], []
    for n in (1, 2, 3, 7, 21, 49, 64, 65, 100, 121, 128, 129, 225, 512):
        mu = rng.uniform(0.0, 1.0, n)
        if n >= 7:
            mu[:3] = 0.0                       # null space of A
            mu[3:6] = 0.05                     # a triple eigenvalue below sel
            mu[6] = 0.05 + 1e-9                # and one just beside it
        if n >= 21:
            mu[7:9] = 0.5                      # double eigenvalue above sel
            mu[9] = 0.099                      # near the cut, below
            mu[10] = 0.101                     # near the cut, above
        Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
        V = Q * rng.uniform(0.5, 2.0, n)        # cond(B) <= 16
        Vi = np.linalg.inv(V)
        B = Vi.T @ Vi
        A = Vi.T @ np.diag(mu) @ Vi
        As.append(0.5 * (A + A.T)); Bs.append(0.5 * (B + B.T)); mus.append(np.sort(mu))
    ws, Xs = api.sygv_select(As, Bs, sel)
    for A, B, mu, w, X in zip(As, Bs, mus, ws, Xs):
        n = len(w)
        Lc = np.linalg.cholesky(B)
        Li = np.linalg.inv(Lc)
        ref = np.linalg.eigvalsh(Li @ A @ Li.T)
        scale = max(1.0, np.abs(ref).max())
        assert np.all(np.diff(w) >= 0)
        assert np.abs(w - ref).max() <= 1e-12 * scale, (n, np.abs(w - ref).max())
        p = int(np.sum(w <= sel))
        assert p == int(np.sum(ref <= sel))
        if p == 0:
            continue
        Vs = np.linalg.solve(B, X[:, :p])      # X = B v
        assert np.abs(Vs.T @ B @ Vs - np.eye(p)).max() <= 1e-10, n
        res = A @ Vs - B @ Vs * w[:p]
        assert np.abs(res).max() <= 1e-10 * max(np.abs(A).max(), np.abs(B).max()), (n, np.abs(res).max())

