"""Write the oracle's results on the full-size workloads to tests/golden/.

    python tests/golden/make_fullsize.py [config3 config4 config5]
    python tests/golden/make_fullsize.py old [config3]

Calls only the CPU oracle (oracle/) on the seeded workload generators; the
GPU parity tests read the files this writes.  Per workload (seed 0,
Theta_F = Theta_E = 10, GMRES(30), rtol 1e-8, maxit 300), in
oracle_<workload>_seed0.npz:

  counts        n_vertex, pnum_face, pnum_edge, n_primal, n_near_ties
                (default reading: prior-selected primal unknowns shared)
  face_p/edge_r primal count per face / edge (interface order)
  face_mu_ptr, face_mu   concatenated ascending spectra mu = 1/lambda of the
  edge_mu_ptr, edge_mu   face and edge eigenproblems (interface order)
  u             the full solution (free grid nodes by node id)
  iters, restarts, relres_true, history      GMRES record
  ghat_norm     ||ghat||
  sep_counts, sep_edge_r, sep_iters          the same with the literal
                stacked (separate) prior-selected primal unknowns

and, for the earlier edge eigenproblem (eq. equ-4-8-E), in
oracle_<workload>_seed0_old.npz: counts, face_p, edge_r, edge_mu_ptr,
edge_mu, u, iters, restarts, relres_true, history.

The oracle needs ~1.5 minutes per workload on 8 cores (plus a second setup
and solve for the separate reading).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import bddc  # noqa: E402
from paper_2501_01676_amd import workloads as W  # noqa: E402

COUNT_KEYS = ("n_vertex", "pnum_face", "pnum_edge", "n_primal", "n_near_ties")


def path_for(name, seed=0):
    return os.path.join(HERE, f"oracle_{name}_seed{seed}.npz")


def _concat(mus):
    ptr = np.zeros(len(mus) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([m.size for m in mus])
    return ptr, (np.concatenate(mus) if mus else np.zeros(0))


def make(name, seed=0):
    p = W.get(name, seed)
    t0 = time.perf_counter()
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 10.0, "theta_edge": 10.0})
    u, info = o.gmres_solve(30, 1e-8, 300)
    topo = o.topo
    fptr, fmu = _concat([np.sort(o.face_mu[k]) for k in topo.faces])
    eptr, emu = _concat([np.sort(o.edge_mu[k]) for k in topo.edges])
    out = dict(
        counts=np.array([o.counts[k] for k in COUNT_KEYS], dtype=np.int64),
        face_p=np.array([o.face_p[k] for k in topo.faces], dtype=np.int32),
        edge_r=np.array([o.edge_r[k] for k in topo.edges], dtype=np.int32),
        face_mu_ptr=fptr, face_mu=fmu, edge_mu_ptr=eptr, edge_mu=emu,
        u=u, iters=np.int64(info["iters"]), restarts=np.int64(info["restarts"]),
        relres_true=np.float64(info["relres_true"]), history=np.array(info["history"]),
        ghat_norm=np.float64(np.linalg.norm(o.ghat)))
    print(f"[golden] {name} seed {seed}: counts {o.counts} iters {info['iters']} "
          f"({time.perf_counter() - t0:.0f} s)", flush=True)
    # the literal reading of the coupled edge matrix: stacked prior primals
    o.setup_coarse_space({"theta_face": 10.0, "theta_edge": 10.0, "edge_h_mode": "separate"})
    _, sinfo = o.gmres_solve(30, 1e-8, 300)
    out.update(sep_counts=np.array([o.counts[k] for k in COUNT_KEYS], dtype=np.int64),
               sep_edge_r=np.array([o.edge_r[k] for k in topo.edges], dtype=np.int32),
               sep_iters=np.int64(sinfo["iters"]))
    print(f"[golden] {name} seed {seed} separate: counts {o.counts} iters {sinfo['iters']} "
          f"({time.perf_counter() - t0:.0f} s)", flush=True)
    np.savez_compressed(path_for(name, seed), **out)


def make_old(name, seed=0):
    p = W.get(name, seed)
    t0 = time.perf_counter()
    o = bddc.OracleBDDC(p)
    o.assemble()
    o.setup_coarse_space({"theta_face": 10.0, "theta_edge": 10.0, "edge_variant": "old"})
    u, info = o.gmres_solve(30, 1e-8, 300)
    topo = o.topo
    eptr, emu = _concat([np.sort(o.edge_mu[k]) for k in topo.edges])
    np.savez_compressed(
        os.path.join(HERE, f"oracle_{name}_seed{seed}_old.npz"),
        counts=np.array([o.counts[k] for k in COUNT_KEYS], dtype=np.int64),
        face_p=np.array([o.face_p[k] for k in topo.faces], dtype=np.int32),
        edge_r=np.array([o.edge_r[k] for k in topo.edges], dtype=np.int32),
        edge_mu_ptr=eptr, edge_mu=emu, u=u, iters=np.int64(info["iters"]),
        restarts=np.int64(info["restarts"]), relres_true=np.float64(info["relres_true"]),
        history=np.array(info["history"]))
    print(f"[golden] {name} seed {seed} earlier edge eigenproblem: counts {o.counts} iters {info['iters']} "
          f"({time.perf_counter() - t0:.0f} s)", flush=True)


def load(name, seed=0):
    with np.load(path_for(name, seed)) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "old":
        for name in (args[1:] or ["config3"]):
            make_old(name)
    else:
        for name in (args or ["config3", "config4", "config5"]):
            make(name)
