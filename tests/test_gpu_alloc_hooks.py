"""Caller-supplied device memory (abddc_device alloc / free / user): a
context bound to torch's caching allocator takes every device allocation of
assemble, setup and solve through the hooks (the library's own cache serves
none meanwhile), returns every block at destroy, and gives bit-identical
results to a context on the library's allocator."""
import ctypes as C
import gc

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2501_01676_amd import workloads as W  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cache_allocs():
    from paper_2501_01676_amd import _lib as L
    n, b = C.c_int64(), C.c_int64()
    L.check(L.load().abddc_cache_stats(torch.cuda.current_device(), C.byref(n), C.byref(b)))
    return n.value


def _solve(p, allocator, **opts):
    from paper_2501_01676_amd import api
    g = api.Solver(p, allocator=allocator)
    counts = g.setup_coarse_space(**opts)
    u, info = g.gmres_solve(restart=30, rtol=1e-8, maxit=300)
    r = torch.from_numpy(np.random.default_rng(1).standard_normal(g.n_gamma)).cuda()
    z = g.apply_bddc(r)
    torch.cuda.synchronize()
    g.close()
    return counts, u.cpu(), info, z.cpu()   # no device tensor outlives the call


@pytest.mark.parametrize("precision", [0, 1])
def test_torch_allocator_hooks(precision):
    _need_gpu()
    from paper_2501_01676_amd import api
    p = W.config2()
    opts = dict(precision=precision)
    # the library's allocator first (it also sizes the process-wide work
    # space the partial LU keeps in the library's own cache)
    c0, u0, i0, z0 = _solve(p, None, **opts)
    gc.collect()   # device tensors left by earlier tests
    before = _cache_allocs()
    mem0 = torch.cuda.memory_allocated()
    hooks = api.TorchAllocator(torch.cuda.current_device(), torch.cuda.current_stream())
    c1, u1, i1, z1 = _solve(p, hooks, **opts)
    after = _cache_allocs()
    print(f"[hooks] precision {precision}: {hooks.n_alloc} allocations ({hooks.bytes_total / 2**20:.1f} MiB) "
          f"through the hooks, {after - before} from the library cache", flush=True)
    assert hooks.n_alloc > 0
    assert after == before                       # nothing bypassed the hooks
    assert hooks.n_free == hooks.n_alloc and not hooks.live
    gc.collect()
    assert torch.cuda.memory_allocated() == mem0   # every block went back to torch
    assert c1 == c0 and i1["iters"] == i0["iters"]
    assert np.array_equal(i1["history"], i0["history"])
    assert torch.equal(u1, u0) and torch.equal(z1, z0)


def test_hook_failure_is_enomem():
    """An allocator that refuses (alloc returns NULL) makes the call fail
    with ENOMEM and releases what it had taken."""
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api

    class Refusing(api.TorchAllocator):
        def __init__(self, device, stream, budget):
            super().__init__(device, stream)
            inner = self.alloc_fn
            self.budget = budget

            def _alloc(nbytes, user):
                if self.n_alloc >= self.budget:
                    return None
                return inner(nbytes, user)
            self.alloc_fn = L.ALLOC_FN(_alloc)
            self._inner = inner

    hooks = Refusing(torch.cuda.current_device(), torch.cuda.current_stream(), budget=5)
    with pytest.raises(L.AbddcError) as e:
        api.Solver(W.config1b(), allocator=hooks)
    assert e.value.code == L.ENOMEM
    torch.cuda.synchronize()
    assert hooks.n_free == hooks.n_alloc and not hooks.live
