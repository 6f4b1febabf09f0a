"""Error paths of the C ABI on the GPU.  Every condition is either rejected
on the host before any kernel runs, or raised from a flag that a kernel sets
while it finishes normally (no test makes a kernel fault, trap or hang)."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2501_01676_amd import workloads as W  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _code(fn, *a, **kw):
    from paper_2501_01676_amd import _lib as L
    with pytest.raises(L.AbddcError) as e:
        fn(*a, **kw)
    return e.value.code


def test_calls_out_of_order_return_estate():
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    g = api.Solver(W.config1a())
    r = torch.zeros(g.n_gamma, dtype=torch.float64, device="cuda")
    assert _code(g.apply_bddc, r) == L.ESTATE
    assert _code(g.gmres_solve) == L.ESTATE
    assert _code(g.stage, 2, 0) == L.ESTATE       # face spectrum before setup
    assert _code(g.stage, 6) == L.ESTATE          # counts before setup
    # assembled state allows the Schur operator and the local stages
    g.apply_schur(r)
    assert g.stage(0, 0).size > 0
    g.close()


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
@pytest.mark.parametrize("on_device", [False, True])
def test_nonpositive_or_nonfinite_nu_is_einval(bad, on_device):
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    p = W.config1a()
    p["nu"] = p["nu"].copy()
    p["nu"][37] = bad
    if on_device:
        p["nu"] = torch.from_numpy(p["nu"]).cuda()
    assert _code(api.Solver, p) == L.EINVAL
    assert b"nu" in L.load().abddc_last_error()


def test_invalid_solver_arguments_are_einval():
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    g = api.Solver(W.config1a())
    assert _code(g.setup_coarse_space, theta_face=-1.0) == L.EINVAL
    assert _code(g.setup_coarse_space, edge_h_mode=7) == L.EINVAL
    assert _code(g.setup_coarse_space, precision=3) == L.EINVAL
    g.setup_coarse_space()
    for kw in (dict(restart=0), dict(restart=64), dict(rtol=0.0), dict(rtol=1.0), dict(maxit=0)):
        assert _code(g.gmres_solve, **kw) == L.EINVAL, kw
    p = W.config1a()
    p["tau"] = 0.0
    assert _code(api.Solver, p) == L.EINVAL
    g.close()


def test_not_converged_returns_last_iterate():
    """maxit reached first: ABDDC_NOT_CONVERGED (a warning, not an error),
    info filled, and the returned u is the iterate after maxit Arnoldi steps
    (with the interiors recovered from it), equal to the oracle's."""
    _need_gpu()
    from oracle import bddc
    from paper_2501_01676_amd import api
    p = W.config1b()
    g = api.Solver(p)
    g.setup_coarse_space()
    u, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=3)
    assert not info["converged"] and info["iters"] == 3 and info["relres_true"] > 1e-8
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({})
    u_ref, info_ref = o.gmres_solve(30, 1e-8, 3)
    assert info_ref["iters"] == 3
    assert abs(info["relres_true"] - info_ref["relres_true"]) <= 1e-9 * info_ref["relres_true"]
    assert np.linalg.norm(u.cpu().numpy() - u_ref) <= 1e-10 * np.linalg.norm(u_ref)
    g.close()


def test_zero_load_gives_zero_solution():
    """ghat = 0: converged at once with no Arnoldi step, u = 0."""
    _need_gpu()
    from paper_2501_01676_amd import api
    g = api.Solver(W.uniform(2, 4, f=0.0))
    g.setup_coarse_space()
    u, info = g.gmres_solve()
    assert info["converged"] and info["iters"] == 0
    assert torch.count_nonzero(u).item() == 0
    g.close()


def test_zero_leading_pivot_is_esingular():
    """The partial LU flags a zero pivot (the kernels run to the end on the
    resulting non-finite values) and the hook returns ESINGULAR."""
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    rng = np.random.default_rng(0)
    A = rng.standard_normal((20, 20)) + 20 * np.eye(20)
    A[0, 0] = 0.0
    B = rng.standard_normal((30, 30)) + 30 * np.eye(30)
    assert _code(api.partial_lu, [A, B], [10, 10]) == L.ESINGULAR
    # the same batch with a nonzero pivot passes
    A[0, 0] = 5.0
    api.partial_lu([A, B], [10, 10])


def test_null_arguments_are_einval():
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    lib = L.load()
    g = api.Solver(W.config1a())
    g.setup_coarse_space()
    assert lib.abddc_apply_bddc(g.ctx, None, None) == L.EINVAL
    assert lib.abddc_gmres_solve(g.ctx, 30, 1e-8, 10, None, None) == L.EINVAL
    assert lib.abddc_setup_coarse_space(None, None, None) == L.EINVAL
    assert lib.abddc_get_stage(g.ctx, 99, 0, None, 0) == L.EINVAL
    assert lib.abddc_get_stage(g.ctx, 0, 10 ** 6, None, 0) == L.EINVAL
    assert lib.abddc_kernel_stats(g.ctx, 99, None, None, None) == L.EINVAL
    g.close()


def test_learned_constraints_refuse_tetrahedra():
    """Edge features read one viscosity per box, so the learned path is
    refused (EINVAL, before any feature kernel) on linear-tetrahedron
    problems; the exact path on the same context still works."""
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    g = api.Solver(W.example_helicoid(1, 1.0, 1e-7, 2))
    assert _code(g.edge_features) == L.EINVAL
    assert b"trilinear boxes" in L.load().abddc_last_error()
    net = api.MLP(W.mlp_init_params(0))
    assert _code(g.setup_coarse_space, constraint_source=1, mlp=net) == L.EINVAL
    assert b"trilinear boxes" in L.load().abddc_last_error()
    counts = g.setup_coarse_space(theta_face=1.0 + np.log(2.0))
    assert counts["n_vertex"] == 1
    g.close()
