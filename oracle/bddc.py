"""Adaptive BDDC for the NSPD Schur complement system (Section 3).

Steps, in the paper's order and notation:

  local Schur      S^(i) = A_BB - A_BI A_II^{-1} A_IB,  g^(i) = f_B - A_BI A_II^{-1} f_I
                   B^(i) = (S^(i) + S^(i)^T) / 2                 (Section 3)
  deluxe scaling   D_X^(k) = (sum_{j in n(X)} S_XX^(j))^{-1} S_XX^(k)
  face GEP         B_F v = lambda Btilde_F v                      (eq. equ-4-8)
                   B_F = D_j^T B_F^(i) D_j + D_i^T B_F^(j) D_i
                   Btilde_F = Btilde_F^(i) : Btilde_F^(j)  (parallel sum)
                   constraints (B_F v_l)^T (w_i,F - w_j,F) = 0   (eq. primal-constraints-F)
  edge GEP (old)   B_E v = lambda Btilde_E v, one constraint per selected
                   eigenvector (eq. equ-4-8-E, primal-constraints-E)
  edge GEP (new)   M_E vcheck = lambda Btilde~_E vcheck           (eq. equ-5-21)
                   M_E = That^T blockdiag(B_E^(k)) That           (eq. equ-5-20)
                   Btilde~_E = Schur complement onto the jumps of the matrix
                   coupling edge unknowns and prior-selected primal unknowns
                   (eq. equ-5-18 and the text after it)
                   constraints (M_E vcheck_l)^T wcheck = 0        (eq. equ-5-22)
                   realised by an SVD + QR change of basis (Remark after equ-5-22)
  preconditioner   M^{-1} = Rtilde^T Dtilde Stilde^{-1} Dtilde^T Rtilde
  Krylov           GMRES on Rtilde^T Stilde Rtilde u = Rtilde^T gtilde (eq. Schur-complex-sys)

Readings where the paper is silent (both the oracle and the library follow
them): the generalized eigenproblems are solved in reciprocal form with the
SPD matrix as metric, selecting mu = 1/lambda <= 1/Theta; pseudo-inverses
drop eigenvalues <= pinv_rtol * lambda_max; the edge rank uses the singular
values of the constraint block matrix with relative cut svd_rtol; vertices
carry the partition-of-unity weight 1/|n(V)|; prior-selected primal unknowns
H_k are all vertex dofs and all face-primal coordinates of Gamma_k, shared
between subdomains ("shared" mode) or stacked per subdomain ("separate").
"""
from __future__ import annotations

import numpy as np

from .topology import Topology, make_topology  # noqa: F401
from . import fem


DEFAULT_OPTIONS = {
    "theta_face": 10.0,
    "theta_edge": 10.0,
    "edge_h_mode": "shared",     # or "separate"
    "deluxe_source": "S",        # or "B"
    "pinv_rtol": 1e-10,
    "svd_rtol": 1e-8,
    "tie_rtol": 1e-9,
    "edge_ref": 0,               # which member of n(E) is the jump reference
    "edge_variant": "new",       # "new" (eq. equ-5-21) or "old" (eq. equ-4-8-E)
}


# ---------------------------------------------------------------- helpers
def sym(M):
    return 0.5 * (M + M.T)


def pinv_sym(M, rtol):
    """Moore-Penrose inverse of a symmetric PSD matrix from its eigenpairs,
    dropping eigenvalues <= rtol * lambda_max."""
    if M.size == 0:
        return M.copy()
    w, U = np.linalg.eigh(sym(M))
    top = max(float(w.max()), 0.0)
    keep = w > rtol * top if top > 0 else np.zeros_like(w, dtype=bool)
    Uk = U[:, keep]
    return (Uk / w[keep]) @ Uk.T


def parallel_sum(A, B, rtol):
    """A : B = A (A + B)^+ B (Anderson-Duffin), symmetrised."""
    return sym(A @ pinv_sym(A + B, rtol) @ B)


def parallel_sum_all(mats, rtol):
    """A_1 : A_2 : ... : A_m, folded left to right (the parallel sum of PSD
    matrices is commutative and associative)."""
    out = mats[0]
    for A in mats[1:]:
        out = parallel_sum(out, A, rtol)
    return out


def schur_onto(M, keep, rtol=None):
    """Schur complement of M onto index set ``keep`` (eliminating the rest).
    With rtol given, the eliminated block is inverted with pinv_sym."""
    keep = np.asarray(keep, dtype=np.int64)
    elim = np.setdiff1d(np.arange(M.shape[0]), keep)
    Mkk = M[np.ix_(keep, keep)]
    if elim.size == 0:
        return Mkk.copy()
    Mke = M[np.ix_(keep, elim)]
    Mek = M[np.ix_(elim, keep)]
    Mee = M[np.ix_(elim, elim)]
    if rtol is None:
        return Mkk - Mke @ np.linalg.solve(Mee, Mek)
    return Mkk - Mke @ pinv_sym(Mee, rtol) @ Mek


def gep_reciprocal(Bt, Bspd):
    """Eigenpairs of the pencil (Bt, Bspd): Bt y = mu Bspd y, Bspd SPD.

    Returns mu ascending and X = L Y where Bspd = L L^T and Y are the
    orthonormal eigenvectors of L^{-1} Bt L^{-T}.  The GEP vectors are
    v = L^{-T} y, so X[:, l] = Bspd v_l (the constraint vectors) and
    v_l^T Bspd v_m = delta_lm as the paper requires."""
    n = Bspd.shape[0]
    if n == 0:
        return np.zeros(0), np.zeros((0, 0))
    L = np.linalg.cholesky(sym(Bspd))
    Li = np.linalg.solve(L, np.eye(n))
    C = sym(Li @ Bt @ Li.T)
    mu, Y = np.linalg.eigh(C)
    return mu, L @ Y


def select(mu, theta, tie_rtol):
    """lambda >= Theta  <=>  mu <= 1/Theta (lambda = infinity included).
    Returns the selection mask and the number of near ties
    |lambda - Theta| <= tie_rtol * Theta."""
    sel = mu <= 1.0 / theta
    lam = np.where(mu > 0, 1.0 / np.maximum(mu, 1e-300), np.inf)
    ties = int(np.sum(np.abs(lam - theta) <= tie_rtol * theta))
    return sel, ties


def complete_basis(C, rank=None):
    """Orthonormal basis [Q | Qperp] of R^n whose first r columns span
    range(C) (Householder QR, complete mode)."""
    n = C.shape[0]
    r = C.shape[1] if rank is None else rank
    if r == 0:
        return np.eye(n), 0
    Q, _ = np.linalg.qr(C[:, :r] if rank is not None else C, mode="complete")
    return Q, r


# ------------------------------------------------------------------ class
class OracleBDDC:
    """Adaptive BDDC-GMRES with the new edge eigenproblem, FP64, on the CPU.

    Usage mirrors the library boundary: assemble -> setup_coarse_space ->
    apply_bddc / apply_schur / gmres_solve."""

    def __init__(self, problem):
        self.problem = problem
        self.topo = make_topology(problem)
        self.state = "created"

    # ------------------------------------------------------------ assemble
    def assemble(self, npts=3):
        """Local matrices and Schur complements (Section 3).

        S^(i) = A_BB - A_BI A_II^{-1} A_IB and g^(i) = f_B - A_BI A_II^{-1} f_I
        (the paper prints g^(i) = f_B - A_II^{-1} f_I, which does not
        type-check; the harmonic-extension form is used), B^(i) = sym(S^(i))."""
        topo = self.topo
        self.elem = fem.element_matrices(self.problem, topo, npts)
        local = fem.assemble_subdomains(self.problem, topo, npts, self.elem)
        self.A_loc, self.f_loc, self.S, self.g, self.B = [], [], [], [], []
        for s, (Al, fl) in enumerate(local):
            nI = topo.sub[s]["nI"]
            AII, AIB = Al[:nI, :nI], Al[:nI, nI:]
            ABI, ABB = Al[nI:, :nI], Al[nI:, nI:]
            X = np.linalg.solve(AII, np.concatenate([AIB, fl[:nI, None]], axis=1))
            S = ABB - ABI @ X[:, :-1]
            g = fl[nI:] - ABI @ X[:, -1]
            self.A_loc.append(Al)
            self.f_loc.append(fl)
            self.S.append(S)
            self.g.append(g)
            self.B.append(sym(S))
        # condensed right-hand side ghat = sum_i R_i^T g^(i)
        self.ghat = np.zeros(topo.n_gamma)
        for s in range(topo.n_sub):
            np.add.at(self.ghat, topo.sub[s]["gamma"], self.g[s])
        self.state = "assembled"

    # ---------------------------------------------------- operator pieces
    def apply_schur(self, x):
        """Shat x = sum_i R_i^T S^(i) R_i x."""
        topo = self.topo
        y = np.zeros(topo.n_gamma)
        for s in range(topo.n_sub):
            gam = topo.sub[s]["gamma"]
            np.add.at(y, gam, self.S[s] @ x[gam])
        return y

    def _block(self, M, s, k):
        loc = self.topo.sub[s]["obj_local"][k]
        return M[np.ix_(loc, loc)]

    # --------------------------------------------------------------- setup
    def setup_coarse_space(self, options=None):
        opt = dict(DEFAULT_OPTIONS)
        if options:
            opt.update(options)
        self.opt = opt
        self._deluxe()
        self._faces()
        if opt["edge_variant"] == "old":
            self._edges_old()
        else:
            self._edges()
        self._change_of_basis()
        self._coarse()
        self.state = "setup"
        return self.counts

    def _deluxe(self):
        """Deluxe weights D_X^(k) = (sum_j S_XX^(j))^{-1} S_XX^(k) for faces
        and edges (partition of unity, eq. partition-unity-cond); vertices
        get 1/|n(V)|.  deluxe_source = "B" uses B^(k) instead of S^(k)."""
        topo = self.topo
        src = self.S if self.opt["deluxe_source"] == "S" else self.B
        self.D = {}
        for k, o in enumerate(topo.objects):
            subs = o["subs"]
            if o["kind"] == "vertex":
                for s in subs:
                    self.D[(k, s)] = np.full((1, 1), 1.0 / len(subs))
                continue
            blocks = [self._block(src[s], s, k) for s in subs]
            tot = sum(blocks)
            for s, blk in zip(subs, blocks):
                self.D[(k, s)] = np.linalg.solve(tot, blk)

    def _faces(self):
        """Face eigenproblems (eq. equ-4-8) and face change of basis.

        Btilde_F^(nu) = B_FF - B_FC B_CC^{-1} B_CF with C = Gamma_nu minus F;
        Btilde_F is their parallel sum; B_F v = lambda Btilde_F v is solved
        in reciprocal form; the constraint vectors B_F v_l (lambda_l >= Theta_F)
        span range(Q_F), completed by QR to an orthonormal [Q_F | Q_F^perp]."""
        topo, opt = self.topo, self.opt
        self.face_mu, self.face_p, self.face_T = {}, {}, {}
        self.face_aux = {}
        self.n_ties = 0
        for k in topo.faces:
            i, j = topo.objects[k]["subs"]
            BFi, BFj = self._block(self.B[i], i, k), self._block(self.B[j], j, k)
            Di, Dj = self.D[(k, i)], self.D[(k, j)]
            BF = Dj.T @ BFi @ Dj + Di.T @ BFj @ Di
            Bti = schur_onto(self.B[i], topo.sub[i]["obj_local"][k])
            Btj = schur_onto(self.B[j], topo.sub[j]["obj_local"][k])
            Bt = parallel_sum(sym(Bti), sym(Btj), opt["pinv_rtol"])
            mu, X = gep_reciprocal(Bt, sym(BF))
            sel, ties = select(mu, opt["theta_face"], opt["tie_rtol"])
            self.n_ties += ties
            T, p = complete_basis(X[:, sel])
            self.face_mu[k], self.face_p[k], self.face_T[k] = mu, p, T
            self.face_aux[k] = {"BF": sym(BF), "Bt": Bt, "Bti": Bti, "Btj": Btj, "X": X, "sel": sel}

    def _primal_numbering_faces(self):
        """Global primal ids: vertices first, then face primal coordinates."""
        topo = self.topo
        self.vertex_pid = {k: n for n, k in enumerate(topo.vertices)}
        self.face_pid = {}
        nxt = len(topo.vertices)
        for k in topo.faces:
            self.face_pid[k] = np.arange(nxt, nxt + self.face_p[k])
            nxt += self.face_p[k]
        return nxt

    def _rotate_faces(self, M, s):
        """T^T M T for the face bases of Gamma_s (edges and vertices untouched),
        coordinates of each face ordered [primal (Q_F^T w), dual (Q_F^perp^T w)]."""
        topo = self.topo
        T = np.eye(M.shape[0])
        for k in topo.sub[s]["objects"]:
            if topo.objects[k]["kind"] == "face":
                loc = topo.sub[s]["obj_local"][k]
                T[np.ix_(loc, loc)] = self.face_T[k]
        return T.T @ M @ T

    def _H_positions(self, s):
        """Local positions (in the face-rotated basis) and global primal ids of
        the prior-selected primal unknowns H_s: vertex dofs and face primal
        coordinates of Gamma_s, ordered by global primal id."""
        topo = self.topo
        pos, pid = [], []
        for k in topo.sub[s]["objects"]:
            kind = topo.objects[k]["kind"]
            loc = topo.sub[s]["obj_local"][k]
            if kind == "vertex":
                pos.append(loc[0])
                pid.append(self.vertex_pid[k])
            elif kind == "face":
                for l in range(self.face_p[k]):
                    pos.append(loc[l])
                    pid.append(self.face_pid[k][l])
        order = np.argsort(pid, kind="stable")
        return np.asarray(pos, dtype=np.int64)[order], np.asarray(pid, dtype=np.int64)[order]

    def edge_operators(self, k):
        """M_E (eq. equ-5-20) and Btilde~_E (Schur complement of Btilde_E
        onto the jumps wcheck) for edge object k, plus the pieces.

        For n(E) = {k_1 < ... < k_m} the jumps are wcheck_j = w_kj - w_k1
        (j = 2..m) and what = sum_k D_E^(k) w_k (eq. equ-5-19), so that
        w_k = That_k wcheck + what with That_k = [-D^(k2) ... (I - D^(kj) in
        slot k) ... -D^(km)] (eq. equ-trans)."""
        topo, opt = self.topo, self.opt
        subs = list(topo.objects[k]["subs"])
        ref = int(opt.get("edge_ref", 0)) % len(subs)
        subs = [subs[ref]] + subs[:ref] + subs[ref + 1:]
        m = len(subs)
        nE = topo.objects[k]["nodes"].size
        Ds = [self.D[(k, s)] for s in subs]
        That = []
        for a in range(m):
            row = []
            for b in range(1, m):
                blk = -Ds[b]
                if a == b:
                    blk = blk + np.eye(nE)
                row.append(blk)
            That.append(np.concatenate(row, axis=1))                 # (nE, (m-1) nE)
        BE = [self._block(self.B[s], s, k) for s in subs]
        ME = sum(That[a].T @ BE[a] @ That[a] for a in range(m))

        # Btilde^(k): Schur complement of the face-rotated B^(k) onto (E, H_k)
        Hpos, Hpid, Bt = [], [], []
        for s in subs:
            Bbar = self._rotate_faces(self.B[s], s)
            pos, pid = self._H_positions(s)
            keep = np.concatenate([topo.sub[s]["obj_local"][k], pos])
            Bt.append(schur_onto(Bbar, keep))
            Hpos.append(pos)
            Hpid.append(pid)
        if opt["edge_h_mode"] == "shared":
            union = np.unique(np.concatenate(Hpid)) if Hpid else np.zeros(0, np.int64)
            R = [np.searchsorted(union, pid) for pid in Hpid]
            nH = union.size
        else:
            offs = np.cumsum([0] + [p.size for p in Hpid])
            R = [np.arange(offs[a], offs[a + 1]) for a in range(m)]
            nH = int(offs[-1])
        nw = (m - 1) * nE
        nv = nw + nE + nH
        BtE = np.zeros((nv, nv))
        for a in range(m):
            P = np.zeros((nE + R[a].size, nv))
            P[:nE, :nw] = That[a]
            P[:nE, nw:nw + nE] = np.eye(nE)
            P[nE + np.arange(R[a].size), nw + nE + R[a]] = 1.0
            BtE += P.T @ sym(Bt[a]) @ P
        BttE = sym(schur_onto(sym(BtE), np.arange(nw), rtol=opt["pinv_rtol"]))
        return {"ME": sym(ME), "BttE": BttE, "That": That, "BE": BE, "BtE": sym(BtE),
                "Bt": Bt, "R": R, "nH": nH, "m": m, "nE": nE, "subs": subs, "Ds": Ds}

    def _edges(self):
        """New edge eigenproblem (eq. equ-5-21) and the SVD + QR edge basis."""
        topo, opt = self.topo, self.opt
        self._primal_numbering_faces()
        self.edge_mu, self.edge_r, self.edge_T, self.edge_nsel = {}, {}, {}, {}
        self.edge_aux = {}
        for k in topo.edges:
            ops = self.edge_operators(k)
            mu, X = gep_reciprocal(ops["BttE"], ops["ME"])
            sel, ties = select(mu, opt["theta_edge"], opt["tie_rtol"])
            self.n_ties += ties
            nE, m = ops["nE"], ops["m"]
            # g_l = M_E vcheck_l split into m-1 blocks of length n_E
            G = np.concatenate([X[b * nE:(b + 1) * nE][:, sel] for b in range(m - 1)], axis=1)
            if G.shape[1] == 0:
                r = 0
                U = np.eye(nE)
            else:
                U, sv, _ = np.linalg.svd(G)
                r = int(np.sum(sv > opt["svd_rtol"] * sv[0])) if sv[0] > 0 else 0
            T, _ = complete_basis(U[:, :r], rank=r) if r > 0 else (np.eye(nE), 0)
            self.edge_mu[k], self.edge_r[k], self.edge_T[k] = mu, r, T
            self.edge_nsel[k] = int(sel.sum())
            self.edge_aux[k] = dict(ops, X=X, sel=sel, G=G)

    def _edges_old(self):
        """The earlier edge eigenproblem (eq. equ-4-8-E): B_E v = lambda Btilde_E v,

          B_E       = sum_{i in n(E)} sum_{k in n(E), k != i} D_E^(k)^T B_E^(i) D_E^(k),
                      B_E^(i) = (B^(i))_EE,
          Btilde_E  = Btilde_E^(1) : ... : Btilde_E^(m), the parallel sum of the
                      Schur complements of B^(nu) onto E (C = Gamma_nu minus E),

        solved in reciprocal form like the faces; one constraint
        (B_E v_l)^T (w_i,E - w_j,E) = 0 per lambda_l >= Theta_E
        (eq. primal-constraints-E), realised by an orthonormal basis of
        span{B_E v_l} completed by QR."""
        topo, opt = self.topo, self.opt
        self._primal_numbering_faces()
        self.edge_mu, self.edge_r, self.edge_T, self.edge_nsel = {}, {}, {}, {}
        self.edge_aux = {}
        for k in topo.edges:
            subs = list(topo.objects[k]["subs"])
            BEi = {s: self._block(self.B[s], s, k) for s in subs}
            BE = sum(self.D[(k, kk)].T @ BEi[i] @ self.D[(k, kk)] for i in subs for kk in subs if kk != i)
            Bts = [sym(schur_onto(self.B[s], topo.sub[s]["obj_local"][k])) for s in subs]
            Bt = parallel_sum_all(Bts, opt["pinv_rtol"])
            mu, X = gep_reciprocal(Bt, sym(BE))
            sel, ties = select(mu, opt["theta_edge"], opt["tie_rtol"])
            self.n_ties += ties
            T, p = complete_basis(X[:, sel])
            self.edge_mu[k], self.edge_r[k], self.edge_T[k] = mu, p, T
            self.edge_nsel[k] = int(sel.sum())
            self.edge_aux[k] = {"BE": sym(BE), "Bt": Bt, "Bts": Bts, "BEi": BEi, "X": X, "sel": sel,
                                "subs": subs, "Ds": [self.D[(k, s)] for s in subs]}

    def _change_of_basis(self):
        """T_i = blockdiag([Q_X | Q_X^perp]) over Gamma_i; Pi_i = primal
        coordinates (vertices, face and edge primal), Delta_i = the rest."""
        topo = self.topo
        npf = self._primal_numbering_faces()
        self.edge_pid = {}
        nxt = npf
        for k in topo.edges:
            self.edge_pid[k] = np.arange(nxt, nxt + self.edge_r[k])
            nxt += self.edge_r[k]
        self.n_primal = nxt
        self.T, self.Pi_loc, self.Pi_gid, self.Delta_loc, self.Dmat = [], [], [], [], []
        for s in range(topo.n_sub):
            sd = topo.sub[s]
            nB = sd["nB"]
            T = np.zeros((nB, nB))
            Dm = np.zeros((nB, nB))
            pi_loc, pi_gid, de_loc = [], [], []
            for k in sd["objects"]:
                loc = sd["obj_local"][k]
                kind = topo.objects[k]["kind"]
                if kind == "vertex":
                    TX, p, pid = np.eye(1), 1, [self.vertex_pid[k]]
                elif kind == "face":
                    TX, p, pid = self.face_T[k], self.face_p[k], list(self.face_pid[k])
                else:
                    TX, p, pid = self.edge_T[k], self.edge_r[k], list(self.edge_pid[k])
                T[np.ix_(loc, loc)] = TX
                Dm[np.ix_(loc, loc)] = self.D[(k, s)]
                pi_loc += list(loc[:p])
                pi_gid += pid
                de_loc += list(loc[p:])
            self.T.append(T)
            self.Dmat.append(Dm)
            self.Pi_loc.append(np.asarray(pi_loc, dtype=np.int64))
            self.Pi_gid.append(np.asarray(pi_gid, dtype=np.int64))
            self.Delta_loc.append(np.asarray(de_loc, dtype=np.int64))
        self.counts = {
            "n_vertex": len(topo.vertices),
            "pnum_face": int(sum(self.face_p.values())),
            "pnum_edge": int(sum(self.edge_r.values())),
            "n_primal": int(self.n_primal),
            "n_near_ties": int(self.n_ties),
        }

    def _coarse(self):
        """Sbar = T^T S T split into Delta/Pi blocks; Phi = -Sbar_DD^{-1} Sbar_DP,
        Psi^T = -Sbar_PD Sbar_DD^{-1}, S_Pi^(i) = Sbar_PP + Sbar_PD Phi;
        S_Pi = sum R_Pi^T S_Pi^(i) R_Pi."""
        topo = self.topo
        self.Sbar, self.Phi, self.PsiT, self.SPi_loc = [], [], [], []
        SPi = np.zeros((self.n_primal, self.n_primal))
        for s in range(topo.n_sub):
            Sb = self.T[s].T @ self.S[s] @ self.T[s]
            d, p = self.Delta_loc[s], self.Pi_loc[s]
            Sdd, Sdp = Sb[np.ix_(d, d)], Sb[np.ix_(d, p)]
            Spd, Spp = Sb[np.ix_(p, d)], Sb[np.ix_(p, p)]
            if d.size:
                Phi = -np.linalg.solve(Sdd, Sdp)
                PsiT = -np.linalg.solve(Sdd.T, Spd.T).T
            else:
                Phi = np.zeros((0, p.size))
                PsiT = np.zeros((p.size, 0))
            Sp = Spp + Spd @ Phi
            gid = self.Pi_gid[s]
            SPi[np.ix_(gid, gid)] += Sp
            self.Sbar.append(Sb)
            self.Phi.append(Phi)
            self.PsiT.append(PsiT)
            self.SPi_loc.append(Sp)
        self.SPi = SPi

    # ------------------------------------------------------------- apply
    def apply_bddc(self, r):
        """z = M^{-1} r = Rtilde^T Dtilde Stilde^{-1} Dtilde^T Rtilde r with the
        partially assembled inverse written by block elimination of the dual
        unknowns (primal unknowns assembled, dual unknowns local)."""
        topo = self.topo
        gbar, y = [], []
        gPi = np.zeros(self.n_primal)
        bPi = np.zeros(self.n_primal)
        for s in range(topo.n_sub):
            gam = topo.sub[s]["gamma"]
            gb = self.T[s].T @ (self.Dmat[s].T @ r[gam])
            d, p = self.Delta_loc[s], self.Pi_loc[s]
            np.add.at(gPi, self.Pi_gid[s], gb[p])
            ys = np.linalg.solve(self.Sbar[s][np.ix_(d, d)], gb[d]) if d.size else np.zeros(0)
            np.add.at(bPi, self.Pi_gid[s], -self.Sbar[s][np.ix_(p, d)] @ ys)
            gbar.append(gb)
            y.append(ys)
        bPi += gPi
        xPi = np.linalg.solve(self.SPi, bPi) if self.n_primal else np.zeros(0)
        z = np.zeros(topo.n_gamma)
        for s in range(topo.n_sub):
            gam = topo.sub[s]["gamma"]
            d, p = self.Delta_loc[s], self.Pi_loc[s]
            xp = xPi[self.Pi_gid[s]]
            xd = y[s] + self.Phi[s] @ xp
            w = np.zeros(topo.sub[s]["nB"])
            w[d] = xd
            w[p] = xp
            np.add.at(z, gam, self.Dmat[s] @ (self.T[s] @ w))
        return z

    # ------------------------------------------------------------ GMRES
    def gmres_solve(self, restart=30, rtol=1e-8, maxit=300):
        """Right-preconditioned restarted GMRES (flexible form, stored Z) with
        classical Gram-Schmidt applied twice and Givens rotations, x0 = 0.
        Stops when the true residual ||ghat - Shat x|| <= rtol ||ghat|| or
        after maxit Arnoldi steps; then recovers the interior unknowns."""
        x, info = gmres(self.apply_schur, self.apply_bddc, self.ghat, restart, rtol, maxit)
        self.uhat = x
        self.u = self.recover(x)
        return self.u, info

    def recover(self, uhat):
        """u_I^(i) = A_II^{-1} (f_I - A_IB u_B^(i)); full free-dof vector."""
        topo = self.topo
        u = np.zeros(topo.n_dof)
        u[topo.dof_of_node[topo.iface_nodes]] = uhat
        for s in range(topo.n_sub):
            nI = topo.sub[s]["nI"]
            Al, fl = self.A_loc[s], self.f_loc[s]
            uB = uhat[topo.sub[s]["gamma"]]
            uI = np.linalg.solve(Al[:nI, :nI], fl[:nI] - Al[:nI, nI:] @ uB)
            u[topo.dof_of_node[topo.sub[s]["interior"]]] = uI
        return u


def gmres(Aop, Mop, b, restart, rtol, maxit, keep_basis=False):
    """Restarted right-preconditioned flexible GMRES with CGS2 and Givens
    rotations.  Returns (x, info) with info = {iters, restarts, relres_true,
    history (Arnoldi residual estimates / ||b||)}; keep_basis stores the
    last cycle's orthonormal Arnoldi vectors in info["basis"]."""
    n = b.size
    x = np.zeros(n)
    bnorm = float(np.linalg.norm(b))
    info = {"iters": 0, "restarts": 0, "history": [], "relres_true": 0.0}
    if bnorm == 0.0:
        return x, info
    r = b.copy()
    beta = bnorm
    while True:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs, sn = np.zeros(restart), np.zeros(restart)
        gv = np.zeros(restart + 1)
        gv[0] = beta
        V[0] = r / beta
        jend = 0
        for j in range(restart):
            Z[j] = Mop(V[j])
            w = Aop(Z[j])
            info["iters"] += 1
            Vj = V[:j + 1]
            h = Vj @ w
            w = w - Vj.T @ h
            h2 = Vj @ w
            w = w - Vj.T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            col = np.zeros(restart + 1)
            col[:j + 1] = h
            col[j + 1] = hn
            for i in range(j):
                t = cs[i] * col[i] + sn[i] * col[i + 1]
                col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1]
                col[i] = t
            a, bb = col[j], col[j + 1]
            rr = float(np.hypot(a, bb))
            if rr == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = a / rr, bb / rr
            col[j] = rr
            col[j + 1] = 0.0
            gv[j + 1] = -sn[j] * gv[j]
            gv[j] = cs[j] * gv[j]
            H[:, j] = col
            res = abs(gv[j + 1])
            info["history"].append(res / bnorm)
            jend = j + 1
            if hn == 0.0 or res <= rtol * bnorm or info["iters"] >= maxit:
                break
            V[j + 1] = w / hn
        if keep_basis:
            info["basis"] = V[:jend].copy()
        y = np.zeros(jend)
        for i in range(jend - 1, -1, -1):
            y[i] = (gv[i] - H[i, i + 1:jend] @ y[i + 1:jend]) / H[i, i]
        x = x + Z[:jend].T @ y
        r = b - Aop(x)
        beta = float(np.linalg.norm(r))
        info["relres_true"] = beta / bnorm
        if beta <= rtol * bnorm or info["iters"] >= maxit:
            break
        info["restarts"] += 1
    return x, info


def solve(problem, options=None, restart=30, rtol=1e-8, maxit=300):
    """assemble + setup_coarse_space + gmres_solve; returns the oracle object
    (solution in .u, counts in .counts) and the GMRES info."""
    o = OracleBDDC(problem)
    o.assemble()
    o.setup_coarse_space(options)
    _, info = o.gmres_solve(restart, rtol, maxit)
    return o, info
