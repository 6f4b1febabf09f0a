"""Pins of the learned-constraint oracle (oracle/learned.py) against facts
that do not come from the oracle itself: finite differences, closed forms,
the IEEE bfloat16 pattern (torch's own conversion), a rotation of the whole
problem, projector identities, and the edge spectrum of the exact method."""
import numpy as np
import pytest

from oracle import Topology, bddc
from oracle import learned as Lr
from paper_2501_01676_amd import workloads as W


def test_bf16_rounding_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(2000).astype(np.float32) * 10 ** rng.uniform(-8, 8, 2000).astype(np.float32),
                        np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, -0.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(Lr.bf16(x), ref)
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to the even one (1)
    assert Lr.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert Lr.bf16(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)


def test_param_layout():
    assert Lr.n_params() == 37276
    p = W.mlp_init_params(0)
    parts = Lr.unpack(p)
    assert [x.shape for x in parts] == [(128, 133), (128,), (128, 128), (128,), (28, 128), (28,)]
    assert np.allclose(Lr.pack(parts), p)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = W.mlp_init_params(3).astype(np.float64) * 3.0
    X = rng.standard_normal((6, Lr.N_FEAT))
    T = rng.standard_normal((6, Lr.N_OUT))

    def loss(q):
        Y, _ = Lr.forward(q, X, round_bf16=False)
        return Lr.loss_grad_output(Y, T)[0]

    Y, cache = Lr.forward(p, X, round_bf16=False)
    _, dY = Lr.loss_grad_output(Y, T)
    g = Lr.backward(cache, dY)
    idx = rng.choice(p.size, 60, replace=False)
    # include every bias block and the last layer
    idx = np.concatenate([idx, [128 * 133, 128 * 133 + 127, Lr.n_params() - 1, Lr.n_params() - 29]])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (loss(p + e) - loss(p - e)) / 2e-6
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_loss_closed_form():
    T = np.random.default_rng(2).standard_normal((3, Lr.N_OUT))
    assert Lr.loss_grad_output(T, T)[0] == 0.0
    w = Lr.entry_weights()
    for j in (0, 1, 7):            # diagonal (0, 0), off-diagonal (0, 1), diagonal (1, 1)
        Y = T.copy()
        Y[1, j] += 0.5
        L, dY = Lr.loss_grad_output(Y, T)
        assert np.isclose(L, w[j] * 0.25 / 3)
        assert np.isclose(dY[1, j], 2 * w[j] * 0.5 / 3)
    # the weighted sum equals the Frobenius norm of the full symmetric difference
    Y = T + np.random.default_rng(3).standard_normal(T.shape)
    full = sum(np.sum((Lr.upper_to_sym(Y[b]) - Lr.upper_to_sym(T[b])) ** 2) for b in range(3)) / 3
    assert np.isclose(Lr.loss_grad_output(Y, T)[0], full)


def test_first_adam_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.zeros(4)
    q, m, v = Lr.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected first step: m-hat = g, v-hat = g^2
    assert np.allclose(q, -0.01 * g / (np.abs(g) + 1e-8))


def _rotate(problem):
    """The problem with axes relabelled a -> a + 1 (mod 3)."""
    ne = [int(np.sum(w)) for w in problem["widths"]]
    nu = problem["nu"].reshape(ne[2], ne[1], ne[0])      # [z, y, x]
    # new axis (a + 1) = old axis a: new x = old z, new y = old x, new z = old y
    nu_new = np.transpose(nu, (1, 2, 0))                   # [y, x, z] = [new z, new y, new x]
    P = np.zeros((3, 3))
    for a in range(3):
        P[(a + 1) % 3, a] = 1.0
    out = dict(problem)
    out["nsub"] = tuple(problem["nsub"][(a + 2) % 3] for a in range(3))
    out["widths"] = [problem["widths"][(a + 2) % 3] for a in range(3)]
    out["length"] = [problem["length"][(a + 2) % 3] for a in range(3)]
    out["nu"] = np.ascontiguousarray(nu_new).ravel()
    out["beta0"] = P @ problem["beta0"]
    out["beta1"] = P @ problem["beta1"] @ P.T
    return out, P


def test_features_invariant_under_rotation_of_the_problem():
    p = W.ragged((2, 3, 2), [8], 5, beta0=(3.0, -1.0, 0.5))
    p["beta1"] = np.array([[0.1, 0.2, 0.0], [0.0, -0.3, 0.4], [0.5, 0.0, 0.2]])
    q, P = _rotate(p)
    t1 = Topology(p["nsub"], p["widths"])
    t2 = Topology(q["nsub"], q["widths"])
    assert len(t1.edges) == len(t2.edges) > 0
    # map node coordinates: new coordinate (a + 1) = old coordinate a
    key2 = {}
    for k in t2.edges:
        c = t2.node_coords(int(t2.objects[k]["nodes"][0]))
        key2[tuple(int(v) for v in c)] = k
    for k in t1.edges:
        c = t1.node_coords(int(t1.objects[k]["nodes"][0]))
        cn = [0, 0, 0]
        for a in range(3):
            cn[(a + 1) % 3] = int(c[a])
        k2 = key2[tuple(cn)]
        f1 = Lr.edge_features(p, t1, k)
        f2 = Lr.edge_features(q, t2, k2)
        assert np.allclose(f1, f2, rtol=1e-12, atol=1e-12), k


def test_features_of_a_constant_field():
    p = W.uniform(2, 8, beta=(2.0, 0.0, 0.0))
    p["nu"] = np.full_like(p["nu"], 0.01)
    t = Topology(p["nsub"], p["widths"])
    for k in t.edges:
        f = Lr.edge_features(p, t, k)
        assert np.all(f[:128] == -2.0)
        a = Lr.edge_axis(t, k)
        # velocity (2, 0, 0) in the edge frame (b, c, a)
        v = np.zeros(3)
        v[[(a + 1) % 3, (a + 2) % 3, a].index(0)] = 2.0
        assert np.allclose(f[128:131], np.arcsinh(v))
        h = 1.0 / 16
        assert np.isclose(f[131], np.log10(h * 2.0 / 0.01)) and np.isclose(f[132], f[131])


@pytest.fixture(scope="module")
def loose_edges():
    p = W.uniform(2, 8, beta=(0.7, -0.4, 1.1))
    sx, _, sz = W.element_subdomain(p["widths"])
    p["nu"] = np.where(sx == 0, 1.0, 1e-3) * np.where(sz == 0, 1.0, 0.1)
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 2.0, "theta_edge": 2.0})
    return o


def test_exact_projector_and_rayleigh_judge(loose_edges):
    o = loose_edges
    th = 2.0
    some_constrained = False
    for k in o.topo.edges:
        r, T = o.edge_r[k], o.edge_T[k]
        y = Lr.projector_upper(T[:, :r])
        P = Lr.upper_to_sym(y)
        assert np.allclose(P @ P, P, atol=1e-12) and np.isclose(np.trace(P), r)
        aux = o.edge_aux[k]
        # no constraint: the quotient minimum is the edge spectrum minimum
        q0 = Lr.constrained_min_quotient(aux["ME"], aux["BttE"], np.zeros((aux["nE"], 0)), aux["nE"], aux["m"])
        assert np.isclose(q0, np.min(o.edge_mu[k]), rtol=1e-8, atol=1e-12)
        # the exact constraints bound every quotient by Theta_E
        qx = Lr.constrained_min_quotient(aux["ME"], aux["BttE"], T[:, :r], aux["nE"], aux["m"])
        assert qx >= (1.0 / th) * (1 - 1e-8)
        if r > 0:
            some_constrained = True
            assert q0 < 1.0 / th
    assert some_constrained


def test_gate_rules():
    fmin, fmax = np.zeros(Lr.N_FEAT), np.ones(Lr.N_FEAT)
    x = np.full(Lr.N_FEAT, 0.5)
    Q = np.linalg.qr(np.random.default_rng(4).standard_normal((7, 2)))[0]
    use, B = Lr.gate(Lr.projector_upper(Q), x, fmin, fmax)
    assert use and B.shape == (7, 2) and np.allclose(B @ B.T, Q @ Q.T)
    use, _ = Lr.gate(0.5 * Lr.projector_upper(Q), x, fmin, fmax)        # eigenvalue 0.5: uncertain
    assert not use
    x2 = x.copy()
    x2[3] = 1.2                                                          # outside [-0.1, 1.1]
    assert not Lr.gate(Lr.projector_upper(Q), x2, fmin, fmax)[0]
    x2[3] = 1.05
    assert Lr.gate(Lr.projector_upper(Q), x2, fmin, fmax)[0]
