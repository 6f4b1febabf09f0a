"""Box-partition topology: subdomains, interface classes and orderings.

Section 3 splits the mesh into non-overlapping subdomains whose interfaces
consist of faces, edges and vertices, with n(X) the set of subdomains sharing
an interface object X; the precise class definitions are deferred to another
paper.  For a tensor-product box partition of a box mesh they reduce to the
rule used here: a free (non-Dirichlet) grid node lying on an internal
subdomain cut plane in exactly one / two / three axes is a face / edge /
vertex node, and nodes with the same sharing set n(x) form one object.

Orderings (the library's interface vector layout uses the same rules):
  * grid node id      = ix + (nx+1) * (iy + (ny+1) * iz)
  * subdomain id      = sx + Nx * (sy + Ny * sz)
  * free dofs         = free grid nodes in increasing node id
  * interface objects = all faces, then all edges, then all vertices; inside
                        each kind by increasing smallest node id
  * interface vector  = objects in that order, nodes of an object by node id
  * subdomain i local = interior nodes by node id, then Gamma_i, which lists
                        the interface dofs of i by increasing interface index
"""
from __future__ import annotations

import numpy as np


class Topology:
    KINDS = ("face", "edge", "vertex")

    def __init__(self, nsub, widths):
        self.nsub = tuple(int(v) for v in nsub)
        self.widths = [np.asarray(w, dtype=np.int64) for w in widths]
        for a in range(3):
            assert len(self.widths[a]) == self.nsub[a]
            assert np.all(self.widths[a] >= 2), "every subdomain needs an interior node per axis"
        self.ne_axis = [int(w.sum()) for w in self.widths]
        self.cuts = [np.concatenate([[0], np.cumsum(w)]) for w in self.widths]
        self.nn_axis = [n + 1 for n in self.ne_axis]
        self.n_nodes = int(np.prod(self.nn_axis))
        self.n_elem = int(np.prod(self.ne_axis))
        self.n_sub = int(np.prod(self.nsub))
        self._classify()
        self._subdomains()

    # ----------------------------------------------------------------- ids
    def node_id(self, ix, iy, iz):
        nx, ny, _ = self.nn_axis
        return ix + nx * (iy + ny * iz)

    def node_coords(self, nid):
        nx, ny, _ = self.nn_axis
        return nid % nx, (nid // nx) % ny, nid // (nx * ny)

    def sub_id(self, sx, sy, sz):
        return sx + self.nsub[0] * (sy + self.nsub[1] * sz)

    def sub_coords(self, s):
        Nx, Ny, _ = self.nsub
        return s % Nx, (s // Nx) % Ny, s // (Nx * Ny)

    def _axis_subs(self, a, i):
        """Subdomain indices along axis a whose closed interval holds grid index i."""
        cuts = self.cuts[a]
        out = []
        for s in range(self.nsub[a]):
            if cuts[s] <= i <= cuts[s + 1]:
                out.append(s)
        return out

    # ------------------------------------------------------ classification
    def _classify(self):
        nx, ny, nz = self.nn_axis
        free = np.zeros(self.n_nodes, dtype=bool)
        ix = np.arange(self.n_nodes) % nx
        iy = (np.arange(self.n_nodes) // nx) % ny
        iz = np.arange(self.n_nodes) // (nx * ny)
        free = (ix > 0) & (ix < nx - 1) & (iy > 0) & (iy < ny - 1) & (iz > 0) & (iz < nz - 1)
        self.free = free
        self.free_nodes = np.nonzero(free)[0]
        self.n_dof = int(self.free_nodes.size)
        self.dof_of_node = -np.ones(self.n_nodes, dtype=np.int64)
        self.dof_of_node[self.free_nodes] = np.arange(self.n_dof)

        oncut = []
        for a, ii in enumerate((ix, iy, iz)):
            internal = self.cuts[a][1:-1]
            oncut.append(np.isin(ii, internal))
        count = oncut[0].astype(int) + oncut[1].astype(int) + oncut[2].astype(int)
        self.node_kind = np.where(free, count, -1)  # -1 Dirichlet, 0 interior

        # sharing set of every interface node
        groups = {}
        iface_nodes = np.nonzero(free & (count > 0))[0]
        axis_subs = [[self._axis_subs(a, i) for i in range(self.nn_axis[a])] for a in range(3)]
        for nid in iface_nodes:
            cx, cy, cz = int(ix[nid]), int(iy[nid]), int(iz[nid])
            subs = sorted(self.sub_id(sx, sy, sz)
                          for sz in axis_subs[2][cz]
                          for sy in axis_subs[1][cy]
                          for sx in axis_subs[0][cx])
            key = (int(count[nid]), tuple(subs))
            groups.setdefault(key, []).append(int(nid))

        objects = []
        for (cnt, subs), nodes in groups.items():
            kind = self.KINDS[cnt - 1]
            expected = {1: 2, 2: 4, 3: 8}[cnt]
            assert len(subs) == expected, (kind, subs)
            objects.append({"kind": kind, "subs": subs, "nodes": np.array(sorted(nodes), dtype=np.int64)})
        order = {"face": 0, "edge": 1, "vertex": 2}
        objects.sort(key=lambda o: (order[o["kind"]], int(o["nodes"][0])))
        self.objects = objects
        self.faces = [k for k, o in enumerate(objects) if o["kind"] == "face"]
        self.edges = [k for k, o in enumerate(objects) if o["kind"] == "edge"]
        self.vertices = [k for k, o in enumerate(objects) if o["kind"] == "vertex"]

        self.iface_of_node = -np.ones(self.n_nodes, dtype=np.int64)
        start = 0
        for o in objects:
            n = o["nodes"].size
            o["gstart"] = start
            o["gidx"] = np.arange(start, start + n)
            self.iface_of_node[o["nodes"]] = o["gidx"]
            start += n
        self.n_gamma = start
        self.iface_nodes = np.concatenate([o["nodes"] for o in objects]) if objects else np.zeros(0, np.int64)

    # ---------------------------------------------------------- subdomains
    def _subdomains(self):
        self.sub = []
        nx, ny, _ = self.nn_axis
        for s in range(self.n_sub):
            sx, sy, sz = self.sub_coords(s)
            x0, x1 = self.cuts[0][sx], self.cuts[0][sx + 1]
            y0, y1 = self.cuts[1][sy], self.cuts[1][sy + 1]
            z0, z1 = self.cuts[2][sz], self.cuts[2][sz + 1]
            gx, gy, gz = np.arange(x0 + 1, x1), np.arange(y0 + 1, y1), np.arange(z0 + 1, z1)
            Z, Y, X = np.meshgrid(gz, gy, gx, indexing="ij")
            interior = np.sort(self.node_id(X.ravel(), Y.ravel(), Z.ravel()))
            objs = [k for k, o in enumerate(self.objects) if s in o["subs"]]
            gamma = np.concatenate([self.objects[k]["gidx"] for k in objs]) if objs else np.zeros(0, np.int64)
            # objects are contiguous in the interface vector and listed in
            # interface order, so gamma is already sorted
            assert np.all(np.diff(gamma) > 0)
            loc = {}
            pos = 0
            for k in objs:
                n = self.objects[k]["nodes"].size
                loc[k] = np.arange(pos, pos + n)
                pos += n
            self.sub.append({
                "box": ((x0, x1), (y0, y1), (z0, z1)),
                "interior": interior,
                "gamma": gamma,
                "objects": objs,
                "obj_local": loc,
                "nI": int(interior.size),
                "nB": int(gamma.size),
            })

    # --------------------------------------------------------------- misc
    def elements_of(self, s):
        """Box ids of subdomain s (x-fastest)."""
        (x0, x1), (y0, y1), (z0, z1) = self.element_box(s)
        EZ, EY, EX = np.meshgrid(np.arange(z0, z1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        return self.elem_id(EX.ravel(), EY.ravel(), EZ.ravel())

    def element_box(self, s):
        """Element index ranges (ex0, ex1), (ey0, ey1), (ez0, ez1) of subdomain s."""
        sx, sy, sz = self.sub_coords(s)
        return tuple((int(self.cuts[a][c]), int(self.cuts[a][c + 1]))
                     for a, c in enumerate((sx, sy, sz)))

    def elem_id(self, ex, ey, ez):
        return ex + self.ne_axis[0] * (ey + self.ne_axis[1] * ez)

    def local_nodes(self, s):
        """Node ids of subdomain s in local order [interior; Gamma_s]."""
        sd = self.sub[s]
        return np.concatenate([sd["interior"], self.iface_nodes[sd["gamma"]]])


class PartitionTopology(Topology):
    """Topology of an arbitrary partition of the box grid into face-connected
    unions of boxes (Section 4's irregular subdomain partitions).

    The interface classes follow the same rule read from Section 3 for
    general partitions: n(x) = the subdomains holding a box incident to the
    free node x; a node with |n(x)| = 1 is interior to that subdomain; the
    nodes with one sharing set split into connected pieces (two nodes are
    adjacent when a box holds both), and each piece is one object: a face
    when |n(x)| = 2, an edge when |n(x)| >= 3 and the piece has two or more
    nodes, a vertex when |n(x)| >= 3 and it is a single node.  On a
    tensor-product box partition this gives the box classification.
    Orderings are those of Topology."""

    def __init__(self, widths, part, n_parts):
        self.nsub = (1, 1, 1)
        self.widths = [np.asarray(w, dtype=np.int64) for w in widths]
        self.ne_axis = [int(w.sum()) for w in self.widths]
        self.cuts = [np.concatenate([[0], np.cumsum(w)]) for w in self.widths]
        self.nn_axis = [n + 1 for n in self.ne_axis]
        self.n_nodes = int(np.prod(self.nn_axis))
        self.n_elem = int(np.prod(self.ne_axis))
        self.part = np.asarray(part, dtype=np.int64)
        assert self.part.size == self.n_elem
        self.n_sub = int(n_parts)
        assert self.part.min() >= 0 and self.part.max() < self.n_sub
        self._classify_general()
        self._subdomains_general()

    def _sharing_sets(self):
        nx, ny, nz = self.nn_axis
        ex, ey, ez = self.ne_axis
        nid = np.arange(self.n_nodes)
        ix, iy, iz = nid % nx, (nid // nx) % ny, nid // (nx * ny)
        cols = []
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    bx, by, bz = ix - dx, iy - dy, iz - dz
                    ok = (bx >= 0) & (bx < ex) & (by >= 0) & (by < ey) & (bz >= 0) & (bz < ez)
                    b = np.where(ok, bx + ex * (by + ey * bz), 0)
                    cols.append(np.where(ok, self.part[b], -1))
        P = np.sort(np.stack(cols, axis=1), axis=1)
        return [tuple(sorted(set(int(v) for v in row if v >= 0))) for row in P], (ix, iy, iz)

    def _classify_general(self):
        nx, ny, nz = self.nn_axis
        sets, (ix, iy, iz) = self._sharing_sets()
        free = (ix > 0) & (ix < nx - 1) & (iy > 0) & (iy < ny - 1) & (iz > 0) & (iz < nz - 1)
        self.free = free
        self.free_nodes = np.nonzero(free)[0]
        self.n_dof = int(self.free_nodes.size)
        self.dof_of_node = -np.ones(self.n_nodes, dtype=np.int64)
        self.dof_of_node[self.free_nodes] = np.arange(self.n_dof)
        self.sharing = sets
        groups = {}
        for v in self.free_nodes:
            if len(sets[v]) >= 2:
                groups.setdefault(sets[v], []).append(int(v))
        objects = []
        for subs, nodes in groups.items():
            member = set(nodes)
            seen = set()
            for v0 in nodes:            # node-id order, so pieces come out sorted by first node
                if v0 in seen:
                    continue
                piece, stack = [], [v0]
                seen.add(v0)
                while stack:
                    v = stack.pop()
                    piece.append(v)
                    x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                if dx == dy == dz == 0:
                                    continue
                                w = (x + dx) + nx * ((y + dy) + ny * (z + dz))
                                inside = 0 <= x + dx < nx and 0 <= y + dy < ny and 0 <= z + dz < nz
                                if inside and w in member and w not in seen:
                                    seen.add(w)
                                    stack.append(w)
                if len(subs) == 2:
                    kind = "face"
                else:
                    kind = "edge" if len(piece) >= 2 else "vertex"
                objects.append({"kind": kind, "subs": list(subs), "nodes": np.array(sorted(piece), dtype=np.int64)})
        order = {"face": 0, "edge": 1, "vertex": 2}
        objects.sort(key=lambda o: (order[o["kind"]], int(o["nodes"][0])))
        self.objects = objects
        self.faces = [k for k, o in enumerate(objects) if o["kind"] == "face"]
        self.edges = [k for k, o in enumerate(objects) if o["kind"] == "edge"]
        self.vertices = [k for k, o in enumerate(objects) if o["kind"] == "vertex"]
        self.iface_of_node = -np.ones(self.n_nodes, dtype=np.int64)
        start = 0
        for o in objects:
            n = o["nodes"].size
            o["gstart"] = start
            o["gidx"] = np.arange(start, start + n)
            self.iface_of_node[o["nodes"]] = o["gidx"]
            start += n
        self.n_gamma = start
        self.iface_nodes = np.concatenate([o["nodes"] for o in objects]) if objects else np.zeros(0, np.int64)

    def _subdomains_general(self):
        interior = [[] for _ in range(self.n_sub)]
        for v in self.free_nodes:
            if len(self.sharing[v]) == 1:
                interior[self.sharing[v][0]].append(int(v))
        self.sub = []
        for s in range(self.n_sub):
            objs = [k for k, o in enumerate(self.objects) if s in o["subs"]]
            gamma = np.concatenate([self.objects[k]["gidx"] for k in objs]) if objs else np.zeros(0, np.int64)
            assert np.all(np.diff(gamma) > 0)
            loc = {}
            pos = 0
            for k in objs:
                n = self.objects[k]["nodes"].size
                loc[k] = np.arange(pos, pos + n)
                pos += n
            self.sub.append({
                "interior": np.array(interior[s], dtype=np.int64),
                "gamma": gamma,
                "objects": objs,
                "obj_local": loc,
                "nI": len(interior[s]),
                "nB": int(gamma.size),
            })

    def elements_of(self, s):
        return np.flatnonzero(self.part == s)


def make_topology(problem):
    """The topology of a problem dict: a general partition when it carries
    per-box part ids, else the tensor-product box partition."""
    if problem.get("part") is not None:
        return PartitionTopology(problem["widths"], problem["part"], problem["n_parts"])
    return Topology(problem["nsub"], problem["widths"])
