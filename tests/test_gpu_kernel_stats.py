"""Live kernel statistics: the process-wide class mask chooses which kernel
classes carry timing events, untimed classes report no launches, and timing
changes no result."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2501_01676_amd import workloads as W  # noqa: E402

ALL = (1 << 6) - 1
TRSM, DIAG = 4, 3


def _solve(p):
    from paper_2501_01676_amd import api
    g = api.Solver(p)
    g.setup_coarse_space()
    u, info = g.gmres_solve()
    stats = [g.kernel_stats(k) for k in range(6)]
    g.close()
    return u, info, stats


def test_kernel_stats_mask():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2501_01676_amd import api
    p = W.uniform(2, 8)
    prev = api.set_kernel_stats(0)
    try:
        u0, i0, s0 = _solve(p)
        assert all(s[1] == 0 and s[0] == 0.0 for s in s0)
        assert api.set_kernel_stats(ALL) == 0
        u1, i1, s1 = _solve(p)
        assert s1[TRSM][1] > 0 and s1[DIAG][1] > 0
        assert all(s[0] > 0 and s[2] > 0 for s in s1 if s[1] > 0)
        assert i0["iters"] == i1["iters"] and torch.equal(u0, u1)
        api.set_kernel_stats(1 << TRSM)
        u2, _, s2 = _solve(p)
        assert [k for k in range(6) if s2[k][1] > 0] == [TRSM]
        assert s2[TRSM][1] == s1[TRSM][1] and torch.equal(u0, u2)
        # bits beyond the last class are ignored
        api.set_kernel_stats(0xFFFFFFFF)
        assert api.set_kernel_stats(ALL) == ALL
    finally:
        api.set_kernel_stats(prev)
