"""GPU parity of the learned edge constraints: the network's forward and
backward kernels, the Adam step, edge features and training targets against
the CPU oracle (oracle/learned.py), and the learned setup end to end.

Tolerances: the network rounds weights and layer inputs to bfloat16 on both
sides; the GPU accumulates in FP32, so a rounded value can differ by one
bfloat16 unit (2^-8 relative) where the FP32 pre-activation sits on a
rounding boundary.  Outputs and gradients are compared at 2 % of their
largest magnitude elementwise and 0.5 % in relative Frobenius norm.
Features are FP32 copies of FP64 values: 1e-5 absolute."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle import Topology, bddc  # noqa: E402
from oracle import learned as Lr  # noqa: E402
from paper_2501_01676_amd import workloads as W  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _close(a, b, elem=2e-2, fro=5e-3):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    scale = max(np.abs(b).max(), 1e-30)
    assert np.abs(a - b).max() <= elem * scale, np.abs(a - b).max() / scale
    assert np.linalg.norm(a - b) <= fro * max(np.linalg.norm(b), 1e-30), np.linalg.norm(a - b) / np.linalg.norm(b)


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, Lr.N_FEAT)).astype(np.float32)
    T = rng.uniform(-0.2, 1.0, (n, Lr.N_OUT)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("n", [1, 37, 300])
def test_forward_matches_oracle(n):
    _need_gpu()
    from paper_2501_01676_amd import api
    p = W.mlp_init_params(7) * 2.0
    X, _ = _batch(n, n)
    net = api.MLP(p)
    Y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    Yr, _ = Lr.forward(p, X)
    _close(Y, Yr)
    net.close()


def test_loss_grad_matches_oracle():
    _need_gpu()
    from paper_2501_01676_amd import api
    p = W.mlp_init_params(11) * 2.0
    X, T = _batch(257, 5)
    net = api.MLP(p)
    loss, g = net.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    g = g.cpu().numpy()
    Yr, cache = Lr.forward(p, X)
    Lref, dY = Lr.loss_grad_output(Yr, T)
    gref = Lr.backward(cache, dY)
    assert abs(loss - Lref) <= 1e-3 * Lref
    o = 0
    for shape in Lr.param_shapes():
        k = int(np.prod(shape))
        _close(g[o:o + k], gref[o:o + k], elem=3e-2, fro=1e-2)
        o += k
    net.close()


def test_adam_step_matches_oracle():
    _need_gpu()
    from paper_2501_01676_amd import api
    p = W.mlp_init_params(13)
    X, T = _batch(128, 6)
    net = api.MLP(p)
    lr = 1e-3
    net.train_step(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), lr)
    q = net.params()
    Yr, cache = Lr.forward(p, X)
    _, dY = Lr.loss_grad_output(Yr, T)
    g = Lr.backward(cache, dY)
    qr, _, _ = Lr.adam_step(p.astype(np.float64), g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    # first step moves every weight by about lr in the direction of -sign(g)
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert np.allclose(q[big], qr[big], atol=1e-2 * lr, rtol=0)
    assert np.all(np.abs(q - p) <= lr * (1 + 1e-3))
    net.close()


def _channel_problem(seed, nsub=(3, 3, 3)):
    widths = [[8] * nsub[a] for a in range(3)]
    nu = W.channel_field(widths, 6, seed)
    p = W._problem(nsub, widths, nu, (50.0, 20.0, 10.0), name=f"channels_{seed}")
    p["beta1"] = np.array([[0.0, -5.0, 0.0], [5.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    return p


def test_edge_features_match_oracle():
    _need_gpu()
    from paper_2501_01676_amd import api
    p = _channel_problem(2)
    g = api.Solver(p)
    X, el = g.edge_features()
    X, el = X.cpu().numpy(), el.cpu().numpy()
    t = Topology(p["nsub"], p["widths"])
    assert X.shape == (len(t.edges), Lr.N_FEAT)
    for e, k in enumerate(t.edges):
        ref = Lr.edge_features(p, t, k)
        assert np.abs(X[e] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), e
        assert el[e] == int(Lr.eligible(t, k))
    g.close()


def _layered8():
    p = W.uniform(2, 8, beta=(0.7, -0.4, 1.1))
    sx, _, sz = W.element_subdomain(p["widths"])
    p["nu"] = np.where(sx == 0, 1.0, 1e-3) * np.where(sz == 0, 1.0, 0.1)
    return p


def test_edge_projectors_match_oracle():
    _need_gpu()
    from paper_2501_01676_amd import api
    p = _layered8()
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 2.0, "theta_edge": 2.0})
    g = api.Solver(p)
    g.setup_coarse_space(theta_face=2.0, theta_edge=2.0)
    Y = g.edge_projectors().cpu().numpy()
    assert any(o.edge_r[k] > 0 for k in o.topo.edges)
    for e, k in enumerate(o.topo.edges):
        ref = Lr.projector_upper(o.edge_T[k][:, :o.edge_r[k]])
        assert np.abs(Y[e] - ref).max() <= 1e-6, e
    g.close()


# thresholds at which part of the channel problem's edges select constraints
# (about 7 % at Theta_E = 2; at 1.5 about 75 % do, but those projectors
# depend on the coefficients of the whole neighbouring subdomains, which the
# features do not see, and the gate returns nearly every edge to the exact
# eigenproblem)
THETA_F_L, THETA_E_L = 10.0, 2.0


def _channels4(seed):
    """4x4x4 subdomains, H/h = 8, nu = 1e-4 in 8 seeded straight channels of
    2x2 elements, 1 elsewhere, a = (50, 20, 10): the channel workload at the
    size of one eighth of its 8x8x8 form."""
    widths = [[8] * 4] * 3
    nu = W.channel_field(widths, 8, seed)
    return W._problem((4, 4, 4), widths, nu, (50.0, 20.0, 10.0), name=f"channels4_{seed}")


def _exact(p, **kw):
    from paper_2501_01676_amd import api
    g = api.Solver(p)
    c = g.setup_coarse_space(theta_face=THETA_F_L, theta_edge=kw.pop("theta_edge", THETA_E_L), **kw)
    return g, c


def test_learned_setup_end_to_end():
    """Train on exact setups of six seeded channel problems whose exact edge
    eigenproblems select constraints on many edges, then solve held-out
    seeds with learned edge constraints and compare with the exact method
    and with no edge constraints at all.  Checks: non-trivial labels; the
    loss falls; every edge is predicted or sent back by the gate; faces are
    untouched; the solve converges; the eigenvalue bound of the exact method
    (min constrained quotient of (Btilde~_E, M_E) >= 1 / Theta_E, from the
    oracle's edge operators) holds on at least 90 % of the edges; the
    iteration count is within the judge's 1.2 of the exact one, or the
    library's judge redid the setup exactly; at least 80 % of the edges are
    predicted.  (The edge-phase times are printed: at this size the exact
    edge pipeline is bound by launch latency, so a smaller edge batch does
    not make it faster; the gain is measured at full size by bench.py.)"""
    _need_gpu()
    from paper_2501_01676_amd import api
    Xs, Ts, ref_iters, nonzero, total = [], [], [], 0, 0
    for seed in range(20, 26):
        g, c = _exact(_channels4(seed))
        X, el = g.edge_features()
        T = g.edge_projectors()
        keep = el.bool()
        Xs.append(X[keep])
        Ts.append(T[keep])
        nonzero += int((T[keep].abs().sum(dim=1) > 0).sum().item())
        total += int(keep.sum().item())
        _, info = g.gmres_solve(30, 1e-8, 300, history=False)
        ref_iters.append(info["iters"])
        g.close()
    print(f"[learned] training edges {total}, with constraints {nonzero}; exact iterations {ref_iters}", flush=True)
    assert nonzero >= 0.05 * total and nonzero <= 0.9 * total
    X = torch.cat(Xs).contiguous()
    T = torch.cat(Ts).contiguous()
    net = api.MLP(W.mlp_init_params(0))
    net.set_ranges(X)
    first = net.train_step(X, T, 1e-3, want_loss=True)
    for _ in range(600):
        net.train_step(X, T, 1e-3)
    last = net.train_step(X, T, 1e-3, want_loss=True)
    print(f"[learned] training loss {first:.4g} -> {last:.4g}", flush=True)
    assert last < 0.5 * first
    judge = max(ref_iters)
    for seed in (90, 91):
        p = _channels4(seed)
        ge, ce = _exact(p)
        _, ie = ge.gmres_solve(30, 1e-8, 300, history=False)
        te = ge.phase_times()[4]
        gn, cn = _exact(p, theta_edge=1e300)
        _, i_none = gn.gmres_solve(30, 1e-8, 300, history=False)
        gl, cl = _exact(p, constraint_source=1, mlp=net, judge_iters=judge)
        st = gl.learned_stats()
        tl = gl.phase_times()[4]
        assert st["predicted"] + st["exact"] == gl.n_edge
        assert cl["pnum_face"] == ce["pnum_face"]
        cnt = gl.stage(6)
        nf = gl.n_face
        o = bddc.OracleBDDC(p)
        o.assemble()
        o.setup_coarse_space({"theta_face": THETA_F_L, "theta_edge": THETA_E_L})
        ok = 0
        for e, k in enumerate(o.topo.edges):
            r = int(cnt[nf + e])
            n = o.topo.objects[k]["nodes"].size
            Tb = gl.stage(5, e).reshape(n, n)
            aux = o.edge_aux[k]
            q = Lr.constrained_min_quotient(aux["ME"], aux["BttE"], Tb[:, :r], aux["nE"], aux["m"])
            ok += q >= (1.0 / THETA_E_L) * (1 - 1e-6)
        u, il = gl.gmres_solve(30, 1e-8, 300, history=False)
        print(f"[learned] seed {seed}: predicted {st['predicted']} exact {st['exact']}; pnumE learned "
              f"{cl['pnum_edge']} exact {ce['pnum_edge']}; bound holds on {ok}/{gl.n_edge} edges; iterations "
              f"learned {il['first_iters']} (redone {il['redone']}) exact {ie['iters']} none {i_none['iters']}; "
              f"edge phase learned {tl * 1e3:.2f} ms exact {te * 1e3:.2f} ms", flush=True)
        assert il["converged"] and il["relres_true"] <= 1e-8
        assert gl.n_edge - ok <= 0.1 * gl.n_edge
        assert il["redone"] or il["iters"] <= 1.2 * judge
        assert st["predicted"] >= 0.8 * gl.n_edge
        for g in (ge, gn, gl):
            g.close()
    net.close()


def test_judge_redoes_with_exact_constraints():
    """The library's judge: a network that predicts no constraint on any
    edge (zero weights, every edge inside the training range) with a tight
    reference iteration count makes gmres_solve redo the setup with the exact
    edge eigenproblems and solve again -- bit for bit the exact solve; without
    a reference, or with a loose one, nothing is redone."""
    _need_gpu()
    from paper_2501_01676_amd import api
    p = _channels4(30)
    ge, ce = _exact(p)
    ue, ie = ge.gmres_solve(30, 1e-8, 300)
    X, _ = ge.edge_features()
    from paper_2501_01676_amd import _lib as L
    net = api.MLP(np.zeros(L.MLP_PARAMS, dtype=np.float32))
    net.set_ranges(X)
    for judge, expect in ((1, True), (0, False), (1000, False)):
        gl, cl = _exact(p, constraint_source=1, mlp=net, judge_iters=judge)
        st = gl.learned_stats()
        assert st["predicted"] > 0 and cl["pnum_edge"] < ce["pnum_edge"]
        ul, il = gl.gmres_solve(30, 1e-8, 300)
        assert il["redone"] == expect
        if expect:
            assert il["first_iters"] > 1.2 * judge
            assert il["iters"] == ie["iters"] and torch.equal(ul, ue)
            assert gl.learned_stats() == {"predicted": 0, "exact": gl.n_edge}
        else:
            assert il["first_iters"] == il["iters"]
        gl.close()
    ge.close()
    net.close()


def test_gate_out_of_range_falls_back_to_exact():
    """Features outside the training range send every edge to the exact
    eigenproblem: the learned setup then equals the exact one bit for bit."""
    _need_gpu()
    from paper_2501_01676_amd import api
    p = _layered8()
    net = api.MLP(W.mlp_init_params(1))
    # a training range of one far-away feature vector: every real edge is outside it
    net.set_ranges(torch.full((1, Lr.N_FEAT), 100.0, dtype=torch.float32, device="cuda"))
    ge = api.Solver(p)
    ce = ge.setup_coarse_space(theta_face=2.0, theta_edge=2.0)
    ue, ie = ge.gmres_solve(30, 1e-8, 300)
    gl = api.Solver(p)
    cl = gl.setup_coarse_space(theta_face=2.0, theta_edge=2.0, constraint_source=1, mlp=net)
    st = gl.learned_stats()
    assert st == {"predicted": 0, "exact": gl.n_edge}
    ul, il = gl.gmres_solve(30, 1e-8, 300)
    assert cl == ce and il["iters"] == ie["iters"]
    assert torch.equal(ul, ue)
    ge.close()
    gl.close()
    net.close()


def test_learned_options_rejected_without_network():
    _need_gpu()
    from paper_2501_01676_amd import api
    from paper_2501_01676_amd import _lib as L
    g = api.Solver(W.config1a())
    with pytest.raises(L.AbddcError) as e:
        g.setup_coarse_space(constraint_source=1, mlp=None)
    assert e.value.code == L.EINVAL
    g.close()
