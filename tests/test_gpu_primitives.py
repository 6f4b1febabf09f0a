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
    shapes = [(1, 1, 1), (16, 16, 4), (63, 65, 33), (130, 70, 97), (5, 200, 64)]
    As, Bs, Cs, ref = [], [], [], []
    for m, n, k in shapes:
        A = rng.standard_normal((k, m) if transA else (m, k))
        B = rng.standard_normal((n, k) if transB else (k, n))
        Cm = rng.standard_normal((m, n))
        As.append(A); Bs.append(B); Cs.append(Cm)
        ref.append(-0.5 * (A.T if transA else A) @ (B.T if transB else B) + 2.0 * Cm)
    out = api.gemm(As, Bs, Cs, transA, transB, alpha=-0.5, beta=2.0)
    for o, r in zip(out, ref):
        assert np.abs(o - r).max() <= 1e-12 * max(1.0, np.abs(r).max())


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


def test_partial_lu_inverse_trick():
    """Schur complement of [[A, I], [-I, 0]] onto the trailing block is A^{-1}."""
    api = _api()
    rng = np.random.default_rng(2)
    n = 150
    A = _posreal(n, rng)
    M = np.block([[A, np.eye(n)], [-np.eye(n), np.zeros((n, n))]])
    out = api.partial_lu([M], [n])[0]
    assert np.abs(out[n:, n:] - np.linalg.inv(A)).max() <= 1e-10 * np.abs(np.linalg.inv(A)).max()


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
