"""abddc_apply_bddc_noalloc (work vectors in the library's fixed per-GPU
array) against abddc_apply_bddc (work vectors the library allocates at
setup), through the C ABI: bit-identical results on consecutive calls, the
second on a smaller problem (whose work vectors occupy less of the shared
array that still holds the first call's values), and in mixed precision."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2501_01676_amd import workloads as W  # noqa: E402


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(g, rng):
    r = torch.from_numpy(rng.standard_normal(g.n_gamma)).cuda()
    z_ref = g.apply_bddc(r)
    z = torch.full_like(z_ref, float("nan"))
    g.apply_bddc_noalloc(r, z)
    torch.cuda.synchronize()
    return z, z_ref


def test_noalloc_matches_apply_bddc():
    _need_gpu()
    from paper_2501_01676_amd import api
    rng = np.random.default_rng(7)
    big = api.Solver(W.config2())
    big.setup_coarse_space()
    small = api.Solver(W.ragged((2, 2, 2), [3, 4, 5], 4))
    small.setup_coarse_space(theta_face=2.0, theta_edge=2.0)
    assert small.n_gamma < big.n_gamma
    print(f"[noalloc] config2 n_gamma {big.n_gamma}, then ragged n_gamma {small.n_gamma}", flush=True)
    for g in (big, small, big):
        z, z_ref = _pair(g, rng)
        assert torch.equal(z, z_ref)
    big.close()
    small.close()


def test_noalloc_mixed_precision():
    _need_gpu()
    from paper_2501_01676_amd import api
    rng = np.random.default_rng(8)
    g = api.Solver(W.config1b())
    g.setup_coarse_space(precision=1)
    print(f"[noalloc] config1b mixed n_gamma {g.n_gamma}", flush=True)
    for _ in range(2):
        z, z_ref = _pair(g, rng)
        assert torch.equal(z, z_ref)
    g.close()


def test_noalloc_before_setup_is_rejected():
    _need_gpu()
    from paper_2501_01676_amd import _lib as L
    from paper_2501_01676_amd import api
    g = api.Solver(W.config1a())
    r = torch.zeros(g.n_gamma, dtype=torch.float64, device="cuda")
    z = torch.empty_like(r)
    with pytest.raises(L.AbddcError) as e:
        g.apply_bddc_noalloc(r, z)
    assert e.value.code == L.ESTATE
    g.close()
