"""Seeded synthetic problem generators (inputs only, no method arithmetic).

Every workload is the model advection-diffusion problem of Section 2 on the
unit cube with zero Dirichlet data, discretised by trilinear (Q1) boxes and
split into a tensor-product box partition.  A problem is a plain dict that
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

The random draws (viscosity fields, widths, channels) use
``numpy.random.default_rng(seed)`` so that both sides of any comparison see
the same arrays.
"""
from __future__ import annotations

import numpy as np

THETA_DEFAULT = 10.0


def _problem(nsub, widths, nu, beta0, beta1=None, c=0.0, f_const=1.0,
             f_nodal=None, tau=0.7, length=(1.0, 1.0, 1.0), name=""):
    widths = [np.asarray(w, dtype=np.int32) for w in widths]
    ne = [int(w.sum()) for w in widths]
    nu = np.asarray(nu, dtype=np.float64)
    if nu.ndim == 0:
        nu = np.full(ne[0] * ne[1] * ne[2], float(nu))
    assert nu.size == ne[0] * ne[1] * ne[2]
    if beta1 is None:
        beta1 = np.zeros((3, 3))
    return {
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
