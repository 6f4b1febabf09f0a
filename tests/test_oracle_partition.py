"""Pins of the oracle on general partitions (Section 4's irregular
subdomains): the classification against the box partition it generalises,
structural invariants of the interface classes, subassembly, the direct
solve, all-primal exactness and the SPD lower bound."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2501_01676_amd import workloads as W
from oracle import PartitionTopology, Topology, bddc, fem


def _box_part(T):
    ne = T.ne_axis
    e = np.arange(T.n_elem)
    ex, ey, ez = e % ne[0], (e // ne[0]) % ne[1], e // (ne[0] * ne[1])
    s = [np.searchsorted(T.cuts[a], c, side="right") - 1 for a, c in enumerate((ex, ey, ez))]
    return s[0] + T.nsub[0] * (s[1] + T.nsub[1] * s[2])


@pytest.mark.parametrize("nsub,widths", [((2, 2, 2), [[3, 4], [4, 3], [3, 3]]),
                                         ((3, 2, 2), [[3, 4, 3], [3, 3], [4, 3]])])
def test_box_partition_reproduced(nsub, widths):
    """On a tensor-product partition (every edge of two or more nodes) the
    general rule gives the box classification, orderings and local lists."""
    T = Topology(nsub, widths)
    P = PartitionTopology([[sum(w)] for w in widths], _box_part(T), int(np.prod(nsub)))
    assert [o["kind"] for o in P.objects] == [o["kind"] for o in T.objects]
    for a, b in zip(P.objects, T.objects):
        assert np.array_equal(a["nodes"], b["nodes"]) and list(a["subs"]) == list(b["subs"])
    for s in range(T.n_sub):
        assert np.array_equal(P.sub[s]["interior"], T.sub[s]["interior"])
        assert np.array_equal(P.sub[s]["gamma"], T.sub[s]["gamma"])


@pytest.mark.parametrize("N,n,seed", [(8, 8, 0), (27, 12, 1), (12, 10, 5)])
def test_irregular_classes_invariants(N, n, seed):
    """Every free node is interior to one subdomain or in exactly one
    object; an object's subdomains are exactly those holding a box at each of
    its nodes; faces have two, edges and vertices three or more; pieces are
    connected through common boxes and maximal; every subdomain's local nodes
    are the free nodes of its boxes."""
    part = W.aggregate_partition((n, n, n), N, seed)
    P = PartitionTopology([[n], [n], [n]], part, N)
    nx = n + 1
    owner = -np.ones(P.n_nodes, dtype=np.int64)
    for k, o in enumerate(P.objects):
        assert np.all(owner[o["nodes"]] < 0)
        owner[o["nodes"]] = k
    inside = np.zeros(P.n_nodes, dtype=np.int64)
    for s in range(N):
        inside[P.sub[s]["interior"]] += 1
    free = P.dof_of_node >= 0
    assert np.all(((owner >= 0).astype(int) + inside)[free] == 1)

    def boxes_at(v):
        x, y, z = v % nx, (v // nx) % nx, v // (nx * nx)
        return {int(part[(x - dx) + n * ((y - dy) + n * (z - dz))])
                for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)}

    adj = lambda a, b: max(abs(a % nx - b % nx), abs((a // nx) % nx - (b // nx) % nx),
                           abs(a // (nx * nx) - b // (nx * nx))) <= 1
    for o in P.objects:
        for v in o["nodes"]:
            assert boxes_at(int(v)) == set(o["subs"])
        m = len(o["subs"])
        assert (o["kind"] == "face") == (m == 2)
        if o["kind"] != "face":
            assert (o["kind"] == "edge") == (o["nodes"].size >= 2)
        # connected
        nodes = [int(v) for v in o["nodes"]]
        reach, stack = {nodes[0]}, [nodes[0]]
        while stack:
            v = stack.pop()
            for w in nodes:
                if w not in reach and adj(v, w):
                    reach.add(w)
                    stack.append(w)
        assert len(reach) == len(nodes)
    # maximal: no two objects with one sharing set touch
    by_set = {}
    for k, o in enumerate(P.objects):
        by_set.setdefault(tuple(o["subs"]), []).append(k)
    for ks in by_set.values():
        for i in ks:
            for j in ks:
                if i < j:
                    A, B = P.objects[i]["nodes"], P.objects[j]["nodes"]
                    assert not any(adj(int(a), int(b)) for a in A for b in B)
    for s in range(N):
        boxes = np.flatnonzero(part == s)
        bx, by, bz = boxes % n, (boxes // n) % n, boxes // (n * n)
        nodes = set()
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    nodes |= set(((bx + dx) + nx * ((by + dy) + nx * (bz + dz))).tolist())
        nodes = {v for v in nodes if free[v]}
        local = set(P.sub[s]["interior"].tolist()) | set(P.iface_nodes[P.sub[s]["gamma"]].tolist())
        assert local == nodes


def test_irregular_subassembly_and_direct_solve():
    """sum_i R_i^T A^(i) R_i equals the global matrix, and BDDC-GMRES on the
    irregular partition reaches the sparse direct solution."""
    p = W.example_irregular(8, 8, 0)
    o = bddc.OracleBDDC(p)
    o.assemble()
    topo = o.topo
    M, b = fem.assemble_global(p, topo)
    acc = np.zeros((topo.n_dof, topo.n_dof))
    for s in range(topo.n_sub):
        loc = topo.dof_of_node[topo.local_nodes(s)]
        acc[np.ix_(loc, loc)] += o.A_loc[s]
    assert np.abs(acc - M.toarray()).max() <= 1e-12 * np.abs(M).max()
    o.setup_coarse_space({"theta_face": 1 + np.log(4), "theta_edge": 10.0})
    u, info = o.gmres_solve(30, 1e-10, 300)
    ud = spla.spsolve(M.tocsc(), b)
    assert info["relres_true"] <= 1e-10
    assert np.linalg.norm(u - ud) <= 1e-8 * np.linalg.norm(ud)


def test_irregular_all_primal_is_exact():
    p = W.example_irregular(8, 6, 3)
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 1e-12, "theta_edge": 1e-12})
    assert o.counts["n_primal"] == o.topo.n_gamma
    r = np.random.default_rng(1).standard_normal(o.topo.n_gamma)
    assert np.linalg.norm(o.apply_schur(o.apply_bddc(r)) - r) <= 1e-11 * np.linalg.norm(r)


def test_irregular_spd_lower_bound():
    """a = 0 on an irregular partition: lambda_min(M^{-1} Shat) >= 1, real."""
    p = W.example_irregular(8, 6, 2)
    p["a_nodal"] = np.zeros_like(p["a_nodal"])
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 3.0, "theta_edge": 3.0})
    n = o.topo.n_gamma
    S = np.stack([o.apply_schur(e) for e in np.eye(n)], 1)
    Mi = np.stack([o.apply_bddc(e) for e in np.eye(n)], 1)
    ev = np.linalg.eigvals(Mi @ S)
    assert np.abs(ev.imag).max() <= 1e-8
    assert ev.real.min() >= 1 - 1e-10
