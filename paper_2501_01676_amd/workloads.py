"""Seeded synthetic problem generators (inputs only, no method arithmetic).

Every workload is the model advection-diffusion problem of Section 2 on a
box grid split into a tensor-product box partition: the synthetic configs on
the unit cube with zero Dirichlet data and trilinear (Q1) boxes, Section 4's
example (``example_helicoid``, ``example_random``) with six linear
tetrahedra per box, a nodal velocity and lifted Dirichlet data.  A problem is
a plain dict that
both the GPU library binding and the test oracle read; nothing here computes
any part of the method.

Keys
----
nsub   : (nx, ny, nz) subdomains per axis
widths : three int lists, elements per subdomain along each axis
length : (Lx, Ly, Lz) box lengths (unit cube -> 1, 1, 1)
nu     : float64 array, one viscosity per element, x-fastest ordering
beta0, beta1 : affine velocity a(x) = beta0 + beta1 @ x (beta1 row-major 3x3)
c      : reaction coefficient (constant)
f_const / f_nodal : constant source, or source values at every grid node
                    (x-fastest, (nx_e+1)(ny_e+1)(nz_e+1) values) interpolated
                    trilinearly; f_nodal overrides f_const when not None
tau    : stabilisation constant of the GLS parameter (0.7 in the paper)
element: "q1" (trilinear boxes) or "p1" (six Kuhn tetrahedra per box; nu
         then holds six values per box, tetrahedra in the order of the axis
         permutations xyz, xzy, yxz, yzx, zxy, zyx)
origin : coordinates of grid node (0, 0, 0)
a_nodal: None (affine velocity) or the velocity at every grid node (3 per
         node, node-id order); "p1" only
u_dirichlet : None (zero data) or a value per grid node, of which the
         boundary nodes' are the Dirichlet data
part, n_parts : optional irregular partition: subdomain id per box
         (x-fastest, 0 .. n_parts - 1, each part a face-connected union of
         boxes); nsub is then (1, 1, 1) and widths give the grid

The random draws (viscosity fields, widths, channels) use
``numpy.random.default_rng(seed)`` so that both sides of any comparison see
the same arrays.
"""
from __future__ import annotations

import numpy as np

THETA_DEFAULT = 10.0


def _problem(nsub, widths, nu, beta0, beta1=None, c=0.0, f_const=1.0,
             f_nodal=None, tau=0.7, length=(1.0, 1.0, 1.0), name="", element="q1",
             origin=(0.0, 0.0, 0.0), a_nodal=None, u_dirichlet=None):
    widths = [np.asarray(w, dtype=np.int32) for w in widths]
    ne = [int(w.sum()) for w in widths]
    per = 6 if element == "p1" else 1
    nu = np.asarray(nu, dtype=np.float64)
    if nu.ndim == 0:
        nu = np.full(ne[0] * ne[1] * ne[2] * per, float(nu))
    assert nu.size == ne[0] * ne[1] * ne[2] * per
    if beta1 is None:
        beta1 = np.zeros((3, 3))
    return {
        "element": element,
        "origin": tuple(float(v) for v in origin),
        "a_nodal": None if a_nodal is None else np.ascontiguousarray(a_nodal, dtype=np.float64).reshape(-1),
        "u_dirichlet": None if u_dirichlet is None else np.ascontiguousarray(u_dirichlet, dtype=np.float64),
        "name": name,
        "nsub": tuple(int(v) for v in nsub),
        "widths": widths,
        "length": tuple(float(v) for v in length),
        "nu": np.ascontiguousarray(nu),
        "beta0": np.asarray(beta0, dtype=np.float64).reshape(3),
        "beta1": np.asarray(beta1, dtype=np.float64).reshape(3, 3),
        "c": float(c),
        "f_const": float(f_const),
        "f_nodal": None if f_nodal is None else np.ascontiguousarray(f_nodal, dtype=np.float64),
        "tau": float(tau),
    }


def element_centres(widths, length=(1.0, 1.0, 1.0)):
    """Centre coordinates (x, y, z) of every element, x-fastest flattening."""
    ne = [int(np.sum(w)) for w in widths]
    h = [length[a] / ne[a] for a in range(3)]
    cx = (np.arange(ne[0]) + 0.5) * h[0]
    cy = (np.arange(ne[1]) + 0.5) * h[1]
    cz = (np.arange(ne[2]) + 0.5) * h[2]
    Z, Y, X = np.meshgrid(cz, cy, cx, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def element_subdomain(widths):
    """Subdomain index triple (sx, sy, sz) of every element, x-fastest."""
    out = []
    for a in range(3):
        cuts = np.concatenate([[0], np.cumsum(widths[a])])
        e = np.arange(cuts[-1])
        out.append(np.searchsorted(cuts, e, side="right") - 1)
    Z, Y, X = np.meshgrid(out[2], out[1], out[0], indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def uniform(nsub, hh, nu=1.0, beta=(1.0, 1.0, 1.0), c=0.0, f=1.0, name="uniform"):
    """nsub^3-style box partition with H/h = hh elements per subdomain side."""
    if np.isscalar(nsub):
        nsub = (nsub, nsub, nsub)
    widths = [[hh] * n for n in nsub]
    return _problem(nsub, widths, nu, beta, c=c, f_const=f, name=name)


def config1a():
    """2x2x2 cubic subdomains, H/h = 4 (8^3 elements), nu = 1, a = (1,1,1)."""
    return uniform(2, 4, name="config1a")


def config1b():
    """2x2x2 cubic subdomains, H/h = 8 (16^3 elements), nu = 1, a = (1,1,1)."""
    return uniform(2, 8, name="config1b")


def config2():
    """4x4x4 subdomains, H/h = 8 (32^3 elements); nu = 1 on subdomains with
    even sx+sy+sz, 1e-3 on the others; a = (1, 0.5, 0.25)."""
    widths = [[8] * 4] * 3
    sx, sy, sz = element_subdomain(widths)
    nu = np.where((sx + sy + sz) % 2 == 0, 1.0, 1e-3)
    return _problem((4, 4, 4), widths, nu, (1.0, 0.5, 0.25), name="config2")


def config3(seed=0):
    """8x8x8 subdomains, H/h = 8 (64^3 elements); log10(nu) ~ U[-3, 0] per
    element; a = (10, 10, 10)."""
    rng = np.random.default_rng(seed)
    widths = [[8] * 8] * 3
    nu = 10.0 ** rng.uniform(-3.0, 0.0, 64 ** 3)
    return _problem((8, 8, 8), widths, nu, (10.0, 10.0, 10.0), name=f"config3_s{seed}")


def config4(seed=0):
    """6x6x6 subdomains with per-axis widths drawn from {6, 8, 10, 12};
    log10(nu) ~ U[-3, 0] per element; rotating a = 100 (0.5-y, x-0.5, 0.1)."""
    rng = np.random.default_rng(seed)
    w = rng.choice(np.array([6, 8, 10, 12]), size=(3, 6))
    widths = [list(w[a]) for a in range(3)]
    ne = int(np.prod([sum(x) for x in widths]))
    nu = 10.0 ** rng.uniform(-3.0, 0.0, ne)
    beta0 = (50.0, -50.0, 10.0)
    beta1 = [[0.0, -100.0, 0.0], [100.0, 0.0, 0.0], [0.0, 0.0, 0.0]]
    return _problem((6, 6, 6), widths, nu, beta0, beta1, name=f"config4_s{seed}")


def channel_field(widths, nchannels, seed, nu_out=1.0, nu_in=1e-4):
    """Straight axis-aligned channels of 2x2 elements cross-section spanning
    the whole domain; axis ~ U{x,y,z}, offsets uniform.  Returns nu."""
    rng = np.random.default_rng(seed)
    ne = [int(np.sum(w)) for w in widths]
    field = np.full((ne[2], ne[1], ne[0]), nu_out)
    for _ in range(nchannels):
        ax = int(rng.integers(0, 3))
        others = [a for a in range(3) if a != ax]
        o0 = int(rng.integers(0, ne[others[0]] - 1))
        o1 = int(rng.integers(0, ne[others[1]] - 1))
        sl = [slice(None)] * 3
        # field is indexed [z, y, x]
        sl[2 - others[0]] = slice(o0, o0 + 2)
        sl[2 - others[1]] = slice(o1, o1 + 2)
        field[tuple(sl)] = nu_in
    return field.ravel()


def config5(seed=0):
    """8x8x8 subdomains, H/h = 8; nu = 1e-4 in 32 seeded straight channels of
    2x2-element cross-section, 1 elsewhere; a = (50, 20, 10)."""
    widths = [[8] * 8] * 3
    nu = channel_field(widths, 32, seed)
    return _problem((8, 8, 8), widths, nu, (50.0, 20.0, 10.0), name=f"config5_s{seed}")


def random_field(nsub, hh, seed, lo=-3.0, hi=0.0, beta=(10.0, 10.0, 10.0), name="random"):
    """Box partition with log10(nu) ~ U[lo, hi] per element."""
    if np.isscalar(nsub):
        nsub = (nsub, nsub, nsub)
    widths = [[hh] * n for n in nsub]
    ne = int(np.prod([hh * n for n in nsub]))
    rng = np.random.default_rng(seed)
    nu = 10.0 ** rng.uniform(lo, hi, ne)
    return _problem(nsub, widths, nu, beta, name=name)


def ragged(nsub, choices, seed, beta0=(1.0, 0.5, 0.25), name="ragged"):
    """Box partition with per-axis widths drawn from ``choices``."""
    rng = np.random.default_rng(seed)
    widths = [list(rng.choice(np.array(choices), size=nsub[a])) for a in range(3)]
    ne = int(np.prod([sum(w) for w in widths]))
    nu = 10.0 ** rng.uniform(-2.0, 0.0, ne)
    return _problem(nsub, widths, nu, beta0, name=name)


def manufactured(hh, nsub=2):
    """Problem whose exact solution is sin(pi x) sin(pi y) sin(pi z) for
    nu = 1, a = (1, 1, 1), c = 0; the source is given at the grid nodes."""
    widths = [[hh] * nsub] * 3
    n = hh * nsub
    g = np.linspace(0.0, 1.0, n + 1)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    s, co = np.sin, np.cos
    pi = np.pi
    u = s(pi * X) * s(pi * Y) * s(pi * Z)
    f = 3 * pi ** 2 * u + pi * (co(pi * X) * s(pi * Y) * s(pi * Z)
                                + s(pi * X) * co(pi * Y) * s(pi * Z)
                                + s(pi * X) * s(pi * Y) * co(pi * Z))
    return _problem((nsub,) * 3, widths, 1.0, (1.0, 1.0, 1.0), f_nodal=f.ravel(), name=f"mms{hh}")


def grid_nodes(widths, length=(1.0, 1.0, 1.0), origin=(0.0, 0.0, 0.0)):
    """Coordinates X, Y, Z of every grid node, x-fastest flattening."""
    ne = [int(np.sum(w)) for w in widths]
    ax = [origin[a] + np.arange(ne[a] + 1) * (length[a] / ne[a]) for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


# Section 4's example: the 2x2x2 subdomains numbered anticlockwise (seen from
# +z) around the vertical axis, bottom layer first: (x-, y-), (x+, y-),
# (x+, y+), (x-, y+); value 0 marks the subdomains that take the first of the
# two viscosities of each test, 1 the others.
HELICOID = ((0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1))
EXAMPLE_TESTS = {
    1: (0, 1, 1, 0, 0, 1, 1, 0),   # nu_1 = nu_4 = nu_5 = nu_8
    2: (0, 1, 1, 1, 0, 0, 1, 0),   # nu_1 = nu_5 = nu_6 = nu_8
    3: (0, 1, 0, 1, 1, 0, 1, 0),   # nu_1 = nu_3 = nu_6 = nu_8
}


def _example_problem(n, m, nu_tet, name):
    """Section 4's model problem on (-0.5, 0.5)^2 x (0, 1), n^3 cubic
    subdomains of m^3 boxes, six linear tetrahedra per box: c = 1,
    a = (-2 pi y, 2 pi x, sin 2 pi x) given at the grid nodes, f = 0,
    u = 1 on z = 0 and 0 on the rest of the boundary."""
    widths = [[m] * n] * 3
    org = (-0.5, -0.5, 0.0)
    X, Y, Z = grid_nodes(widths, origin=org)
    a = np.stack([-2.0 * np.pi * Y, 2.0 * np.pi * X, np.sin(2.0 * np.pi * X)], axis=1)
    u0 = np.where(Z == 0.0, 1.0, 0.0)
    return _problem((n, n, n), widths, nu_tet, (0.0, 0.0, 0.0), c=1.0, f_const=0.0, name=name,
                    element="p1", origin=org, a_nodal=a, u_dirichlet=u0)


def example_helicoid(test, nu1, nu2, m):
    """Tests 1-3 of Section 4's uniform-mesh example: 8 subdomains of m^3
    boxes, nu piecewise constant per subdomain (two values, grouped by the
    test's pattern over the helicoidal numbering)."""
    widths = [[m] * 2] * 3
    sx, sy, sz = element_subdomain(widths)
    group = np.empty(8, dtype=np.int64)
    for k, (hx, hy, hz) in enumerate(HELICOID):
        group[hx + 2 * hy + 4 * hz] = EXAMPLE_TESTS[test][k]
    g = group[sx + 2 * sy + 4 * sz]
    nu_box = np.where(g == 0, float(nu1), float(nu2))
    return _example_problem(2, m, np.repeat(nu_box, 6), f"example_t{test}_m{m}")


def example_random(n, m, seed):
    """Section 4's random-viscosity example: n^3 subdomains of m^3 boxes,
    nu = 10^r with r ~ U(-3, 3) drawn per tetrahedron."""
    rng = np.random.default_rng(seed)
    ntet = 6 * (n * m) ** 3
    return _example_problem(n, m, 10.0 ** rng.uniform(-3.0, 3.0, ntet), f"example_random_n{n}_m{m}_s{seed}")


def aggregate_partition(ne, nparts, seed, jitter=0.6):
    """Irregular partition of the boxes of an ne[0] x ne[1] x ne[2] grid into
    nparts connected parts of nearly equal size, by seeded region growing
    (a stand-in for the load-balanced aggregation of a mesh that Section 4
    builds with METIS): seeds by farthest-point sampling from a random first
    box; then, round robin, every part below its quota ceil(n / nparts)
    takes the unassigned face neighbour of its region with the smallest
    squared distance to its seed times (1 + jitter u), u ~ U(0, 1) drawn once
    per box, so the interfaces are ragged; boxes no part could reach join a
    neighbouring part.  Returns part ids per box, x-fastest, int32."""
    import heapq
    rng = np.random.default_rng(seed)
    nx, ny, nz = (int(v) for v in ne)
    n = nx * ny * nz
    ids = np.arange(n)
    cx, cy, cz = ids % nx + 0.5, (ids // nx) % ny + 0.5, ids // (nx * ny) + 0.5
    noise = 1.0 + jitter * rng.uniform(0.0, 1.0, n)
    seeds = [int(rng.integers(0, n))]
    d2 = (cx - cx[seeds[0]]) ** 2 + (cy - cy[seeds[0]]) ** 2 + (cz - cz[seeds[0]]) ** 2
    for _ in range(1, nparts):
        nxt = int(np.argmax(d2))
        seeds.append(nxt)
        d2 = np.minimum(d2, (cx - cx[nxt]) ** 2 + (cy - cy[nxt]) ** 2 + (cz - cz[nxt]) ** 2)

    def neighbours(b):
        x, y, z = b % nx, (b // nx) % ny, b // (nx * ny)
        if x > 0: yield b - 1
        if x < nx - 1: yield b + 1
        if y > 0: yield b - nx
        if y < ny - 1: yield b + nx
        if z > 0: yield b - nx * ny
        if z < nz - 1: yield b + nx * ny

    part = -np.ones(n, dtype=np.int64)
    quota = -(-n // nparts)
    size = [0] * nparts
    heaps = [[] for _ in range(nparts)]

    def take(p, b):
        part[b] = p
        size[p] += 1
        for q in neighbours(b):
            if part[q] < 0:
                s0 = seeds[p]
                key = ((cx[q] - cx[s0]) ** 2 + (cy[q] - cy[s0]) ** 2 + (cz[q] - cz[s0]) ** 2) * noise[q]
                heapq.heappush(heaps[p], (key, q))

    for p, b in enumerate(seeds):
        take(p, b)
    active = True
    while active:
        active = False
        for p in range(nparts):
            if size[p] >= quota:
                continue
            while heaps[p] and part[heaps[p][0][1]] >= 0:
                heapq.heappop(heaps[p])
            if heaps[p]:
                take(p, heapq.heappop(heaps[p])[1])
                active = True
    while (part < 0).any():
        for b in np.flatnonzero(part < 0):
            owners = [part[q] for q in neighbours(b) if part[q] >= 0]
            if owners:
                part[b] = min(owners)
    return part.astype(np.int32)


def example_irregular(nparts, n, seed):
    """Section 4's irregular-partition example: the model problem of
    ``_example_problem`` on an n^3 box grid (h = 1/n, six tetrahedra per
    box) split by ``aggregate_partition`` into nparts subdomains;
    nu = 10^r, r ~ U(-3, 3) per tetrahedron."""
    rng = np.random.default_rng(seed)
    p = _example_problem(1, n, 10.0 ** rng.uniform(-3.0, 3.0, 6 * n ** 3), f"example_irregular_N{nparts}_n{n}_s{seed}")
    p["part"] = aggregate_partition((n, n, n), nparts, seed + 1)
    p["n_parts"] = int(nparts)
    return p


CONFIGS = {
    "config1a": config1a,
    "config1b": config1b,
    "config2": config2,
    "config3": config3,
    "config4": config4,
    "config5": config5,
}


def get(name, seed=0):
    fn = CONFIGS[name]
    if name in ("config3", "config4", "config5"):
        return fn(seed)
    return fn()


def mlp_init_params(seed):
    """Seeded initial parameters of the edge-constraint network (an input of
    the learned variant): Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights
    and biases of the layers 133 -> 128 -> 128 -> 28, packed as W1, b1, W2,
    b2, W3, b3 (row-major weights), float32."""
    rng = np.random.default_rng(seed)
    out = []
    for nout, nin in ((128, 133), (128, 128), (28, 128)):
        bound = 1.0 / np.sqrt(nin)
        out.append(rng.uniform(-bound, bound, (nout, nin)).ravel())
        out.append(rng.uniform(-bound, bound, nout))
    return np.concatenate(out).astype(np.float32)
