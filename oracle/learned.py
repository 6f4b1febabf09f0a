"""Learned edge constraints: features, the MLP, its training step and the
gate/judge around it (a library extension built on the edge eigenproblem of
Section 3, eq. equ-5-21 and equ-5-22).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network predicts, for an edge E of n_E = 7 dofs (H/h = 8 along the
edge), the orthogonal projector P = Q_E Q_E^T onto the span of the edge's
primal constraint vectors chosen by the exact method (Q_E = first r_E
columns of the SVD + QR edge basis).  The projector is invariant under
rotations inside span(Q_E), so it is a well-defined regression target.

  features (133)  log10 nu on the 4 x 4 x 8 element tube around the edge in
                  the edge frame (edge axis last; the two transverse axes in
                  cyclic order after it), asinh of the velocity at the edge
                  midpoint in that frame (3), log10 of the mean and maximum
                  element Peclet number h |a| / nu over the tube (2)
  network         133 -> 128 (ReLU) -> 128 (ReLU) -> 28, weights and the
                  inputs of every product rounded to bfloat16, products
                  accumulated exactly here (FP32 on the GPU), biases FP32
  output          upper triangle (row-major, diagonal included) of P-hat
  loss            mean over the batch of ||P-hat - P||_F^2
  optimiser       Adam (Kingma and Ba 2015) on FP32 master weights
  gate            an edge goes to the exact eigenproblem when an eigenvalue
                  of P-hat lies in [0.3, 0.7] or a feature lies outside the
                  training range widened by 10 %; otherwise its predicted
                  basis is the eigenvectors of P-hat with eigenvalue > 1/2
  judge           max generalized Rayleigh quotient of (M_E, Btilde~_E) on
                  the subspace the predicted constraints leave free, to be
                  compared with Theta_E; and the GMRES iteration count

Pins (tests/test_oracle_learned.py): finite-difference gradients of the
exact-arithmetic network, closed forms of the loss and of the first Adam
step, bf16 rounding against the IEEE bit pattern, feature invariance under a
rotation of the whole problem, the projector of the exact basis, and the
Rayleigh bound of the exact constraints against the edge spectrum.
"""
from __future__ import annotations

import numpy as np

N_FEAT = 133
N_HID = 128
N_E = 7
N_OUT = N_E * (N_E + 1) // 2
TUBE_LEN = 8
LAYERS = ((N_HID, N_FEAT), (N_HID, N_HID), (N_OUT, N_HID))
GATE_LO, GATE_HI = 0.3, 0.7
RANGE_SLACK = 0.1


# ------------------------------------------------------------- bfloat16
def bf16(x):
    """Round float32 values to bfloat16 (round to nearest, ties to even),
    returned as float32 (the upper 16 bits of the IEEE single pattern)."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).reshape(a.shape)
    out[nan] = np.nan
    return out


# -------------------------------------------------------------- features
def edge_axis(topo, k):
    """The axis along the edge: the one whose node coordinate is not a
    subdomain cut (an edge node lies on cut planes of the two others)."""
    x = topo.node_coords(int(topo.objects[k]["nodes"][0]))
    return [a for a in range(3) if int(x[a]) not in set(int(v) for v in topo.cuts[a])][0]


def eligible(topo, k):
    return topo.objects[k]["kind"] == "edge" and topo.objects[k]["nodes"].size == N_E


def edge_features(problem, topo, k):
    """Feature vector of edge object k (133 values, float64)."""
    nodes = topo.objects[k]["nodes"]
    a = edge_axis(topo, k)
    b, c = (a + 1) % 3, (a + 2) % 3
    coords = np.array([topo.node_coords(int(n)) for n in nodes])
    i_lo, i_hi = int(coords[:, a].min()) - 1, int(coords[:, a].max()) + 1   # element range [i_lo, i_hi)
    tb, tc = int(coords[0, b]), int(coords[0, c])
    ne = topo.ne_axis
    L = problem["length"]
    h = np.array([L[d] / ne[d] for d in range(3)])
    nu = problem["nu"]
    feats = np.zeros(N_FEAT)
    pe = []
    for t in range(TUBE_LEN):
        ea = i_lo + int(np.floor((t + 0.5) * (i_hi - i_lo) / TUBE_LEN))
        for u in range(4):
            eb = min(max(tb - 2 + u, 0), ne[b] - 1)
            for v in range(4):
                ec = min(max(tc - 2 + v, 0), ne[c] - 1)
                e3 = [0, 0, 0]
                e3[a], e3[b], e3[c] = ea, eb, ec
                eid = topo.elem_id(*e3)
                feats[t * 16 + u * 4 + v] = np.log10(nu[eid])
                centre = (np.array(e3) + 0.5) * h
                vel = problem["beta0"] + problem["beta1"] @ centre
                pe.append(h.max() * np.linalg.norm(vel) / nu[eid])
    mid = np.zeros(3)
    mid[a] = 0.5 * (i_lo + i_hi) * h[a]
    mid[b] = tb * h[b]
    mid[c] = tc * h[c]
    vel = problem["beta0"] + problem["beta1"] @ mid
    feats[128:131] = np.arcsinh([vel[b], vel[c], vel[a]])
    pe = np.array(pe)
    feats[131] = np.log10(pe.mean() + 1e-30)
    feats[132] = np.log10(pe.max() + 1e-30)
    return feats


# ---------------------------------------------------------------- labels
def projector_upper(Q):
    """Upper triangle (row-major, diagonal included) of Q Q^T."""
    P = Q @ Q.T
    iu = np.triu_indices(P.shape[0])
    return P[iu]


def upper_to_sym(y, n=N_E):
    P = np.zeros((n, n))
    iu = np.triu_indices(n)
    P[iu] = y
    P = P + P.T - np.diag(np.diag(P))
    return P


def entry_weights(n=N_E):
    """Frobenius weights of the upper-triangle entries: 1 on the diagonal,
    2 off it (each off-diagonal entry appears twice in P)."""
    iu = np.triu_indices(n)
    return np.where(iu[0] == iu[1], 1.0, 2.0)


# ------------------------------------------------------------------- MLP
def param_shapes():
    out = []
    for (nout, nin) in LAYERS:
        out += [(nout, nin), (nout,)]
    return out


def n_params():
    return int(sum(np.prod(s) for s in param_shapes()))


def unpack(flat):
    out, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(arrs):
    return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in arrs])


def forward(flat, X, round_bf16=True):
    """Y = MLP(X); returns Y and the cache for backward.  With round_bf16
    the weights and the input of every product are rounded to bfloat16 and
    the pre-activations are float32 values (the GPU's arithmetic)."""
    W1, b1, W2, b2, W3, b3 = unpack(flat)
    rd = (lambda v: bf16(v).astype(np.float64)) if round_bf16 else (lambda v: np.asarray(v, np.float64))
    f32 = (lambda v: np.asarray(v, np.float32).astype(np.float64)) if round_bf16 else (lambda v: v)
    X0 = rd(X)
    Z1 = f32(X0 @ rd(W1).T + b1)
    H1 = rd(np.maximum(Z1, 0.0))
    Z2 = f32(H1 @ rd(W2).T + b2)
    H2 = rd(np.maximum(Z2, 0.0))
    Y = f32(H2 @ rd(W3).T + b3)
    return Y, {"X0": X0, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2, "W": (W1, W2, W3), "rd": rd}


def loss_grad_output(Y, T):
    """L = mean_b ||P-hat_b - P_b||_F^2 and dL/dY."""
    w = entry_weights()
    B = Y.shape[0]
    D = Y - T
    L = float(np.sum(w * D * D) / max(B, 1))
    return L, 2.0 * w * D / max(B, 1)


def backward(cache, dY):
    """Gradients (same layout as the parameters) of sum(dY * Y)."""
    rd = cache["rd"]
    W1, W2, W3 = cache["W"]
    g3 = rd(dY)
    dW3 = g3.T @ cache["H2"]
    db3 = dY.sum(axis=0)
    dZ2 = (g3 @ rd(W3)) * (cache["Z2"] > 0)
    g2 = rd(dZ2)
    dW2 = g2.T @ cache["H1"]
    db2 = dZ2.sum(axis=0)
    dZ1 = (g2 @ rd(W2)) * (cache["Z1"] > 0)
    g1 = rd(dZ1)
    dW1 = g1.T @ cache["X0"]
    db1 = dZ1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(flat, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments), t = 1, 2, ..."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------ gate, judge
def gate(y, x, fmin, fmax):
    """(use_prediction, basis) for one edge: the eigenvectors of P-hat with
    eigenvalue > 1/2, unless an eigenvalue lies in [0.3, 0.7] or a feature
    is outside the widened training range."""
    lam, V = np.linalg.eigh(upper_to_sym(y))
    span = fmax - fmin
    lo, hi = fmin - RANGE_SLACK * span, fmax + RANGE_SLACK * span
    if np.any((lam >= GATE_LO) & (lam <= GATE_HI)) or np.any(x < lo) or np.any(x > hi):
        return False, None
    return True, V[:, lam > 0.5]


def constrained_min_quotient(ME, BttE, Q, nE, m):
    """min over the jumps wcheck left free by the constraints Q^T wcheck_b = 0
    (every block b) of (wcheck^T Btilde~_E wcheck) / (wcheck^T M_E wcheck);
    the constraints bound the edge's Rayleigh quotients of (M_E, Btilde~_E)
    by Theta_E exactly when this is >= 1 / Theta_E."""
    r = Q.shape[1]
    if r == 0:
        N = np.eye((m - 1) * nE)
    else:
        C = np.kron(np.eye(m - 1), Q.T)              # ((m-1) r, (m-1) nE)
        _, s, Vt = np.linalg.svd(C)
        N = Vt[(m - 1) * r:].T
    if N.shape[1] == 0:
        return np.inf
    A = N.T @ BttE @ N
    Bm = N.T @ ME @ N
    Lc = np.linalg.cholesky(0.5 * (Bm + Bm.T))
    Li = np.linalg.inv(Lc)
    return float(np.linalg.eigvalsh(Li @ (0.5 * (A + A.T)) @ Li.T).min())
