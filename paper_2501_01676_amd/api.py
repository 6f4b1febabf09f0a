"""Thin Python binding of the C ABI (argument marshalling only).

torch supplies device memory and the HIP stream; every step of the method
runs in the library's kernels.  Names follow include/abddc.h.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L

ELEMENTS = {"q1": 0, "p1": 1}   # ABDDC_ELEM_Q1, ABDDC_ELEM_P1

DEFAULT_OPTIONS = {
    "theta_face": 10.0,
    "theta_edge": 10.0,
    "edge_variant": 0,
    "edge_h_mode": 0,
    "deluxe_source": 0,
    "pinv_rtol": 1e-10,
    "svd_rtol": 1e-8,
    "tie_rtol": 1e-9,
    "precision": 0,
    "constraint_source": 0,
    "mlp": None,
    "judge_iters": 0,
    "judge_ratio": 0.0,
}


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


class TorchAllocator:
    """Device allocation hooks of abddc_device backed by torch's caching
    allocator on one stream (blocks are reused in that stream's order).
    Counts the library's calls and the bytes it holds."""

    def __init__(self, device, stream):
        self.device, self.stream = device, stream
        self.n_alloc = self.n_free = 0
        self.bytes_total = 0
        self.live = {}

        def _alloc(nbytes, user):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:   # out of memory: the library reports ENOMEM
                return None
            self.n_alloc += 1
            self.bytes_total += int(nbytes)
            self.live[int(p)] = int(nbytes)
            return p

        def _free(p, user):
            self.n_free += 1
            self.live.pop(int(p), None)
            torch.cuda.caching_allocator_delete(int(p))

        # the C function pointers must live as long as any buffer they made
        self.alloc_fn = L.ALLOC_FN(_alloc)
        self.free_fn = L.FREE_FN(_free)

    def bind(self, dev):
        dev.alloc = self.alloc_fn
        dev.free = self.free_fn
        return dev


class Solver:
    """One assembled problem on one GPU (abddc_ctx).  allocator: None (the
    library's caching allocator), "torch" (torch's caching allocator on the
    solver's stream) or a TorchAllocator."""

    def __init__(self, problem, device=0, stream=None, allocator=None):
        self.lib = L.load()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        if allocator == "torch":
            allocator = TorchAllocator(device, self.stream)
        self.allocator = allocator
        p = L.Problem()
        self._keep = []
        for a in range(3):
            p.nsub[a] = int(problem["nsub"][a])
            w = np.ascontiguousarray(problem["widths"][a], dtype=np.int32)
            self._keep.append(w)
            p.width[a] = w.ctypes.data_as(C.POINTER(C.c_int32))
            p.length[a] = float(problem["length"][a])
            p.beta0[a] = float(problem["beta0"][a])
        for i in range(9):
            p.beta1[i] = float(np.asarray(problem["beta1"]).reshape(9)[i])
        p.element = ELEMENTS[problem.get("element", "q1")]
        if problem.get("part") is not None:
            part = np.ascontiguousarray(problem["part"], dtype=np.int32)
            self._keep.append(part)
            p.part = part.ctypes.data_as(C.POINTER(C.c_int32))
            p.n_parts = int(problem["n_parts"])
        for a, v in enumerate(problem.get("origin", (0.0, 0.0, 0.0))):
            p.origin[a] = float(v)
        nu = problem["nu"]
        if isinstance(nu, torch.Tensor):
            # device-resident coefficient arrays (copied on the device)
            assert nu.is_cuda and nu.dtype == torch.float64 and nu.is_contiguous()
            p.nu = self._device_array(nu)
            for key in ("f_nodal", "a_nodal", "u_dirichlet"):
                if problem.get(key) is not None:
                    setattr(p, key, self._device_array(problem[key]))
            p.arrays_on_device = 1
        else:
            p.nu = self._host_array(nu)
            for key in ("f_nodal", "a_nodal", "u_dirichlet"):
                if problem.get(key) is not None:
                    setattr(p, key, self._host_array(problem[key]))
        p.f_const = float(problem["f_const"])
        p.c = float(problem["c"])
        p.tau = float(problem["tau"])
        dev = L.Device(device, _stream_handle(self.stream))
        if allocator is not None:
            allocator.bind(dev)
        ctx = C.c_void_p()
        L.check(self.lib.abddc_assemble(C.byref(p), C.byref(dev), C.byref(ctx)))
        self.ctx = ctx
        nd, ng = C.c_int64(), C.c_int64()
        ns, nf, ne = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(self.lib.abddc_query(ctx, C.byref(nd), C.byref(ng), C.byref(ns), C.byref(nf), C.byref(ne)))
        self.n_dof, self.n_gamma = nd.value, ng.value
        self.n_sub, self.n_face, self.n_edge = ns.value, nf.value, ne.value
        self.counts = None

    def _device_array(self, t):
        assert isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        self._keep.append(t)
        return C.cast(C.c_void_p(t.data_ptr()), C.POINTER(C.c_double))

    def _host_array(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
        self._keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    def setup_coarse_space(self, **opts):
        o = dict(DEFAULT_OPTIONS)
        o.update(opts)
        s = L.Options()
        for k, v in o.items():
            if k == "mlp":
                s.mlp = None if v is None else v.handle
                self._mlp = v   # the network must outlive the setup call
            else:
                setattr(s, k, v)
        cnt = L.Counts()
        L.check(self.lib.abddc_setup_coarse_space(self.ctx, C.byref(s), C.byref(cnt)))
        self.counts = cnt.as_dict()
        return self.counts

    def _vec(self, n):
        return torch.empty(n, dtype=torch.float64, device=f"cuda:{self.device}")

    def edge_features(self):
        """(features n_edge x 133 float32, eligible n_edge int32), device tensors."""
        X = torch.empty((self.n_edge, L.MLP_FEATURES), dtype=torch.float32, device=f"cuda:{self.device}")
        el = torch.empty(self.n_edge, dtype=torch.int32, device=f"cuda:{self.device}")
        if self.n_edge:
            L.check(self.lib.abddc_edge_features(self.ctx, _dptr(X), _dptr(el)))
        return X, el

    def edge_projectors(self):
        """Training targets of the last setup (n_edge x 28 float32, device)."""
        Y = torch.empty((self.n_edge, L.MLP_OUTPUTS), dtype=torch.float32, device=f"cuda:{self.device}")
        if self.n_edge:
            L.check(self.lib.abddc_edge_projectors(self.ctx, _dptr(Y)))
        return Y

    def learned_stats(self):
        a, b = C.c_int32(), C.c_int32()
        L.check(self.lib.abddc_learned_stats(self.ctx, C.byref(a), C.byref(b)))
        return {"predicted": a.value, "exact": b.value}

    def apply_bddc(self, r, out=None):
        z = self._vec(self.n_gamma) if out is None else out
        L.check(self.lib.abddc_apply_bddc(self.ctx, _dptr(r), _dptr(z)))
        return z

    def apply_bddc_noalloc(self, r, out):
        """z = M^{-1} r through the entry point that allocates nothing (work
        vectors in the library's fixed per-GPU array); out is required."""
        L.check(self.lib.abddc_apply_bddc_noalloc(self.ctx, _dptr(r), _dptr(out)))
        return out

    def apply_schur(self, x, out=None):
        y = self._vec(self.n_gamma) if out is None else out
        L.check(self.lib.abddc_apply_schur(self.ctx, _dptr(x), _dptr(y)))
        return y

    def rhs(self):
        g = self._vec(self.n_gamma)
        L.check(self.lib.abddc_get_rhs(self.ctx, _dptr(g)))
        return g

    def gmres_solve(self, restart=30, rtol=1e-8, maxit=300, out=None, history=True):
        u = self._vec(self.n_dof) if out is None else out
        info = L.SolveInfo()
        hist = np.zeros(maxit + 1) if history else None
        if history:
            info.resid_history = hist.ctypes.data_as(C.POINTER(C.c_double))
            info.resid_cap = hist.size
        rc = L.check(self.lib.abddc_gmres_solve(self.ctx, int(restart), float(rtol), int(maxit), _dptr(u),
                                                C.byref(info)))
        res = {"iters": info.iters, "restarts": info.restarts, "relres_true": info.relres_true,
               "t_setup_s": info.t_setup_s, "t_iter_s": info.t_iter_s, "converged": rc == L.OK,
               "redone": bool(info.redone), "first_iters": info.first_iters}
        if history:
            res["history"] = hist[:info.iters].copy()
        return u, res

    def stage(self, stage, index=0):
        n = self.lib.abddc_get_stage(self.ctx, stage, index, None, 0)
        L.check(n)
        buf = np.zeros(max(int(n), 1))
        L.check(self.lib.abddc_get_stage(self.ctx, stage, index, buf.ctypes.data_as(C.POINTER(C.c_double)), n))
        return buf[:n]

    def phase_times(self):
        t = np.zeros(9)
        L.check(self.lib.abddc_phase_times(self.ctx, t.ctypes.data_as(C.POINTER(C.c_double)), 9))
        return t

    def kernel_stats(self, kernel):
        """(seconds, launches, work) accumulated for a tracked kernel class
        (0: partial-LU trailing Schur product, flops; 1: batched GEMV, bytes;
        2: partial-LU per-group update, flops; 3: diagonal-block LU, flops;
        4: panel triangular solves, bytes; 5: in-group band update, flops).
        Only classes in the process-wide mask (set_kernel_stats) are timed."""
        sec, n, w = C.c_double(), C.c_int64(), C.c_double()
        L.check(self.lib.abddc_kernel_stats(self.ctx, kernel, C.byref(sec), C.byref(n), C.byref(w)))
        return sec.value, n.value, w.value

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.abddc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MLP:
    """Edge-constraint network (abddc_mlp) on one GPU."""

    def __init__(self, params, device=0, stream=None):
        self.lib = L.load()
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == L.MLP_PARAMS
        dev = L.Device(device, _stream_handle(self.stream))
        h = C.c_void_p()
        L.check(self.lib.abddc_mlp_create(p.ctypes.data_as(C.POINTER(C.c_float)), p.size, C.byref(dev), C.byref(h)))
        self.handle = h

    def params(self):
        out = np.zeros(L.MLP_PARAMS, dtype=np.float32)
        L.check(self.lib.abddc_mlp_get_params(self.handle, out.ctypes.data_as(C.POINTER(C.c_float)), out.size))
        return out

    def forward(self, X):
        X = X.contiguous()
        Y = torch.empty((X.shape[0], L.MLP_OUTPUTS), dtype=torch.float32, device=X.device)
        L.check(self.lib.abddc_mlp_forward(self.handle, _dptr(X), X.shape[0], _dptr(Y)))
        return Y

    def loss_grad(self, X, T):
        g = torch.empty(L.MLP_PARAMS, dtype=torch.float32, device=X.device)
        loss = C.c_float()
        L.check(self.lib.abddc_mlp_loss_grad(self.handle, _dptr(X.contiguous()), _dptr(T.contiguous()), X.shape[0],
                                             _dptr(g), C.byref(loss)))
        return loss.value, g

    def train_step(self, X, T, lr, want_loss=False):
        loss = C.c_float()
        L.check(self.lib.abddc_mlp_train_step(self.handle, _dptr(X), _dptr(T), X.shape[0], float(lr),
                                              C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def set_ranges(self, X):
        L.check(self.lib.abddc_mlp_set_ranges(self.handle, _dptr(X.contiguous()), X.shape[0]))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.abddc_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- test hooks
def set_kernel_stats(mask):
    """Time the kernel classes whose bits are set in `mask` (bit k: class k
    of Solver.kernel_stats), process-wide; returns the previous mask."""
    return int(L.load().abddc_set_kernel_stats(int(mask) & 0xFFFFFFFF))


def _pack(mats, dtype, device):
    offs, flat = [], []
    pos = 0
    for m in mats:
        offs.append(pos)
        flat.append(np.ascontiguousarray(m, dtype=dtype).ravel())
        pos += m.size
        pad = (-pos) % 64
        flat.append(np.zeros(pad, dtype=dtype))
        pos += pad
    buf = torch.from_numpy(np.concatenate(flat) if flat else np.zeros(1, dtype)).to(device)
    return buf, offs


def partial_lu(mats, ks, precision=0, device="cuda"):
    """Batched in-place partial LU (library primitive) on host matrices."""
    lib = L.load()
    dtype = np.float64 if precision == 0 else np.float32
    buf, offs = _pack(mats, dtype, device)
    rc = lib.abddc_test_partial_lu(len(mats), _dptr(buf), L.i64(offs), L.i32([m.shape[0] for m in mats]),
                                   L.i32([m.shape[1] for m in mats]), L.i32([m.shape[1] for m in mats]),
                                   L.i32(ks), precision, _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    return [h[o:o + m.size].reshape(m.shape) for o, m in zip(offs, mats)]


def gemm(As, Bs, Cs, transA=False, transB=False, alpha=1.0, beta=0.0, device="cuda"):
    lib = L.load()
    buf, offs = _pack(list(As) + list(Bs) + list(Cs), np.float64, device)
    nb = len(As)
    oA, oB, oC = offs[:nb], offs[nb:2 * nb], offs[2 * nb:]
    m = [a.shape[1] if transA else a.shape[0] for a in As]
    k = [a.shape[0] if transA else a.shape[1] for a in As]
    n = [b.shape[0] if transB else b.shape[1] for b in Bs]
    rc = lib.abddc_test_gemm(nb, _dptr(buf), L.i64(oA), L.i64(oB), L.i64(oC), L.i32(m), L.i32(n), L.i32(k),
                             L.i32([a.shape[1] for a in As]), L.i32([b.shape[1] for b in Bs]),
                             L.i32([c.shape[1] for c in Cs]), int(transA), int(transB), alpha, beta,
                             _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    return [h[o:o + c.size].reshape(c.shape) for o, c in zip(oC, Cs)]


def schur_pinv(mats, ks, rtol=1e-10, device="cuda"):
    """Batched M22 - M21 (sym M11)^+ M12 (library primitive); returns the
    trailing blocks."""
    lib = L.load()
    buf, offs = _pack(mats, np.float64, device)
    rc = lib.abddc_test_schur_pinv(len(mats), _dptr(buf), L.i64(offs), L.i32([m.shape[0] for m in mats]),
                                   L.i32(ks), float(rtol), _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    return [h[o:o + m.size].reshape(m.shape)[k:, k:].copy() for o, m, k in zip(offs, mats, ks)]


def parallel_sum(As, Bs, rtol=1e-10, device="cuda"):
    """Batched sym(A (A + B)^+ B) (library primitive) on host matrices."""
    lib = L.load()
    n = [a.shape[0] for a in As]
    outs = [np.zeros((k, k)) for k in n]
    buf, offs = _pack(list(As) + list(Bs) + outs, np.float64, device)
    nb = len(As)
    rc = lib.abddc_test_parallel_sum(nb, _dptr(buf), L.i64(offs[:nb]), L.i64(offs[nb:2 * nb]),
                                     L.i64(offs[2 * nb:]), L.i32(n), float(rtol), _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    return [h[o:o + k * k].reshape(k, k) for o, k in zip(offs[2 * nb:], n)]


def sygv_select(As, Bs, sel, device="cuda"):
    """Every eigenvalue of A y = mu B y (ascending) and X = B Y for the
    eigenvalues <= sel (the first columns; the others are returned as 0)."""
    lib = L.load()
    n = [a.shape[0] for a in As]
    Ws = [np.zeros(k) for k in n]
    Xs = [np.zeros((k, k)) for k in n]
    buf, offs = _pack(list(As) + list(Bs) + Ws + Xs, np.float64, device)
    nb = len(As)
    rc = lib.abddc_test_sygv_select(nb, _dptr(buf), L.i64(offs[:nb]), L.i64(offs[nb:2 * nb]),
                                    L.i64(offs[2 * nb:3 * nb]), L.i64(offs[3 * nb:]), L.i32(n), float(sel),
                                    _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    w = [h[o:o + k].copy() for o, k in zip(offs[2 * nb:3 * nb], n)]
    X = [h[o:o + k * k].reshape(k, k).copy() for o, k in zip(offs[3 * nb:], n)]
    return w, X


def sygv(As, Bs, device="cuda"):
    lib = L.load()
    n = [a.shape[0] for a in As]
    Ws = [np.zeros(k) for k in n]
    Xs = [np.zeros((k, k)) for k in n]
    buf, offs = _pack(list(As) + list(Bs) + Ws + Xs, np.float64, device)
    nb = len(As)
    rc = lib.abddc_test_sygv(nb, _dptr(buf), L.i64(offs[:nb]), L.i64(offs[nb:2 * nb]),
                             L.i64(offs[2 * nb:3 * nb]), L.i64(offs[3 * nb:]), L.i32(n), _stream_handle())
    L.check(rc)
    h = buf.cpu().numpy()
    w = [h[o:o + k] for o, k in zip(offs[2 * nb:3 * nb], n)]
    X = [h[o:o + k * k].reshape(k, k) for o, k in zip(offs[3 * nb:], n)]
    return w, X
