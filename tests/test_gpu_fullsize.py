"""GPU parity at the benchmark's full sizes (seed 0, Theta_F = Theta_E = 10,
GMRES(30), rtol 1e-8), in the launch configuration bench.py times, against
the oracle's results stored by tests/golden/make_fullsize.py (which calls
only oracle/).

FP64: identical primal counts per face and per edge (unless the oracle
reports a near tie), every face and edge spectrum mu = 1/lambda within
1e-9 of the largest |mu| (at least 1), the solution within 1e-10 of the
oracle's relative to its norm, the same iteration count (+-1 at a threshold
crossing).  Mixed precision: the same counts, and the true residual of the
oracle's assembled global system, restricted to the interface rows, at most
rtol ||ghat|| (with the interior rows satisfied to rounding).  The literal
stacked prior-primal reading of the coupled edge matrix: the same counts per
edge and iterations as the oracle in that reading."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2501_01676_amd import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
KEYS = ("n_vertex", "pnum_face", "pnum_edge", "n_primal", "n_near_ties")
FULL = ["config3", "config4", "config5"]


def _golden(name):
    with np.load(os.path.join(GOLDEN, f"oracle_{name}_seed0.npz")) as z:
        return {k: z[k] for k in z.files}


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _counts(ref, key="counts"):
    return dict(zip(KEYS, (int(v) for v in ref[key])))


def _check_setup(g, ref):
    nf = g.n_face
    cnt = g.stage(6)
    assert list(cnt[:nf].astype(int)) == list(ref["face_p"])
    assert list(cnt[nf:].astype(int)) == list(ref["edge_r"])
    fp, fmu = ref["face_mu_ptr"], ref["face_mu"]
    for f in range(nf):
        mu, r = g.stage(2, f), fmu[fp[f]:fp[f + 1]]
        assert mu.size == r.size and np.abs(mu - r).max() <= 1e-9 * max(1.0, np.abs(r).max()), f
    ep, emu = ref["edge_mu_ptr"], ref["edge_mu"]
    for e in range(g.n_edge):
        mu, r = g.stage(3, e), emu[ep[e]:ep[e + 1]]
        assert mu.size == r.size and np.abs(mu - r).max() <= 1e-9 * max(1.0, np.abs(r).max()), e


@pytest.mark.parametrize("name", FULL)
def test_full_size_fp64(name):
    _need_gpu()
    from paper_2501_01676_amd import api
    ref = _golden(name)
    p = W.get(name, 0)
    print(f"[fullsize] {name} FP64: gpu solve", flush=True)
    g = api.Solver(p)
    counts = g.setup_coarse_space()
    rc = _counts(ref)
    if rc["n_near_ties"] == 0:
        assert counts == rc
        _check_setup(g, ref)
    u, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=300)
    u = u.cpu().numpy()
    assert info["converged"] and info["relres_true"] <= 1e-8
    assert abs(info["iters"] - int(ref["iters"])) <= 1
    err = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    print(f"[fullsize] {name}: iters {info['iters']}/{int(ref['iters'])} rel.err {err:.2e}", flush=True)
    assert err <= 1e-10, err
    m = min(len(info["history"]), len(ref["history"]))
    assert np.allclose(info["history"][:m], ref["history"][:m], rtol=1e-6, atol=1e-14)
    g.close()


def test_full_size_mixed_config3():
    _need_gpu()
    from oracle import Topology, fem
    from paper_2501_01676_amd import api
    ref = _golden("config3")
    p = W.config3(0)
    print("[fullsize] config3 mixed: gpu solve", flush=True)
    g = api.Solver(p)
    counts = g.setup_coarse_space(precision=1)
    rc = _counts(ref)
    if rc["n_near_ties"] == 0:
        assert counts == rc
    u, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=300)
    u = u.cpu().numpy()
    g.close()
    assert info["converged"] and info["relres_true"] <= 1e-8
    assert info["iters"] <= int(ref["iters"]) + 3
    topo = Topology(p["nsub"], p["widths"])
    A, b = fem.assemble_global(p, topo)
    r = b - A @ u
    iface = np.zeros(topo.n_dof, dtype=bool)
    iface[topo.dof_of_node[topo.iface_nodes]] = True
    res_gamma = np.linalg.norm(r[iface]) / float(ref["ghat_norm"])
    res_int = np.linalg.norm(r[~iface]) / np.linalg.norm(b)
    print(f"[fullsize] config3 mixed: iters {info['iters']} interface residual {res_gamma:.2e} "
          f"interior residual {res_int:.2e}", flush=True)
    assert res_gamma <= 1.05e-8, res_gamma
    assert res_int <= 1e-12, res_int


@pytest.mark.parametrize("name", FULL)
def test_full_size_separate_prior_primals(name):
    _need_gpu()
    from paper_2501_01676_amd import api
    ref = _golden(name)
    g = api.Solver(W.get(name, 0))
    counts = g.setup_coarse_space(edge_h_mode=1)
    rc = _counts(ref, "sep_counts")
    print(f"[fullsize] {name} separate: counts {counts} oracle {rc}", flush=True)
    if rc["n_near_ties"] == 0:
        assert counts == rc
        cnt = g.stage(6)
        assert list(cnt[g.n_face:].astype(int)) == list(ref["sep_edge_r"])
    _, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=300, history=False)
    g.close()
    assert info["converged"] and abs(info["iters"] - int(ref["sep_iters"])) <= 1


def test_full_size_earlier_edge_eigenproblem_config3():
    """The earlier edge eigenproblem (eq. equ-4-8-E) on config3 at full
    size: identical counts per face and per edge, every edge spectrum within
    1e-9, the solution within 1e-10, iterations +-1."""
    _need_gpu()
    from paper_2501_01676_amd import api
    with np.load(os.path.join(GOLDEN, "oracle_config3_seed0_old.npz")) as z:
        ref = {k: z[k] for k in z.files}
    g = api.Solver(W.config3(0))
    counts = g.setup_coarse_space(edge_variant=1)
    rc = _counts(ref)
    print(f"[fullsize] config3 earlier edges: counts {counts} oracle {rc}", flush=True)
    if rc["n_near_ties"] == 0:
        assert counts == rc
        cnt = g.stage(6)
        assert list(cnt[:g.n_face].astype(int)) == list(ref["face_p"])
        assert list(cnt[g.n_face:].astype(int)) == list(ref["edge_r"])
        ep, emu = ref["edge_mu_ptr"], ref["edge_mu"]
        for e in range(g.n_edge):
            mu, r = g.stage(3, e), emu[ep[e]:ep[e + 1]]
            assert mu.size == r.size and np.abs(mu - r).max() <= 1e-9 * max(1.0, np.abs(r).max()), e
    u, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=300)
    u = u.cpu().numpy()
    g.close()
    assert info["converged"] and abs(info["iters"] - int(ref["iters"])) <= 1
    err = np.linalg.norm(u - ref["u"]) / np.linalg.norm(ref["u"])
    assert err <= 1e-10, err
