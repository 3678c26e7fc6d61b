"""The allocation-free A v (wh_apply_A_noalloc, state levels and accumulator in
the library's fixed device scratch) against wh_apply_A (the same kernels on
the caller's workspace), through the C ABI: a full-size call, then smaller
grids on the same scratch (whose contents the previous call left), and the
size limit."""
import sys

import numpy as np
import pytest

from oracle import core as oc
import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU test run without a GPU: the HIP path has no CPU fallback")
    return _t


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _solver(torch, dim, n, order, prec, seed, omega):
    from paper_2504_03074_amd import Solver
    grid = oc.Grid(dim, n, order)
    c2 = 0.6 + 0.9 * np.abs(np.tanh(wl.random_field(grid.shape, seed=seed, zero_walls=False)))
    s = Solver(dim, n, order=order, precision=prec, restart=2)
    s.set_c2(c2)
    s.set_source(wl.random_field(grid.shape, seed=seed + 1))
    s.set_frequency(omega)
    return s, grid, c2


# (dim, cells, order, precision, omega, bar): the first is the largest 2-D FP64
# grid of the configurations (168 MB of scratch), then smaller ones
CASES = [
    (2, (2048, 2048), 4, "fp64", 200.0, 1e-11),
    (2, (130, 67), 4, "fp64", 23.0, 1e-11),
    (3, (96, 80, 72), 2, "fp32", 30.0, 1e-5),
    (2, (61, 45), 2, "fp32", 12.0, 1e-5),
]


def test_noalloc_matches_apply_A_then_smaller_grids(torch):
    for dim, n, order, prec, omega, bar in CASES:
        _say(f"[noalloc] {dim}-D {n} p={order} {prec} omega={omega}")
        s, grid, c2 = _solver(torch, dim, n, order, prec, 11, omega)
        v = torch.from_numpy(wl.random_field(s.shape, seed=21)).cuda()
        want = s.apply_A(v).cpu().numpy()
        got = s.apply_A_noalloc(v, s.new()).cpu().numpy()
        err = _rel(got, want)
        _say(f"[noalloc]   rel L2 against wh_apply_A {err:.2e}, bitwise equal {np.array_equal(got, want)}")
        assert err <= bar
        # the same kernels on the same inputs: identical results
        assert np.array_equal(got, want)
        if np.prod([m + 1 for m in n]) <= 20000 and prec == "fp64":
            tp = oc.time_params(grid, c2, omega)
            ref = oc.apply_A(grid, c2, v.cpu().numpy(), tp)
            assert _rel(got, ref) <= 1e-11
        del s, v
        torch.cuda.synchronize()


def test_noalloc_twice_in_a_row_second_smaller(torch):
    _say("[noalloc] two calls in a row, the second on a smaller grid")
    big, _, _ = _solver(torch, 2, (1024, 1024), 4, "fp64", 5, 120.0)
    small, grid, c2 = _solver(torch, 2, (77, 90), 2, "fp64", 6, 17.0)
    vb = torch.from_numpy(wl.random_field(big.shape, seed=31)).cuda()
    vs = torch.from_numpy(wl.random_field(small.shape, seed=32)).cuda()
    out_b = big.apply_A_noalloc(vb, big.new())
    out_s = small.apply_A_noalloc(vs, small.new())
    torch.cuda.synchronize()
    assert np.array_equal(out_b.cpu().numpy(), big.apply_A(vb).cpu().numpy())
    got = out_s.cpu().numpy()
    assert np.array_equal(got, small.apply_A(vs).cpu().numpy())
    ref = oc.apply_A(grid, c2, vs.cpu().numpy(), oc.time_params(grid, c2, 17.0))
    assert _rel(got, ref) <= 1e-11


def test_noalloc_rejects_grids_beyond_the_scratch(torch):
    from paper_2504_03074_amd import WhError, wh
    _say("[noalloc] size limit")
    # 2-D 4096^2 FP64: 4 levels + accumulator of 134 MB each, above 192 MiB
    s, _, _ = _solver(torch, 2, (4096, 4096), 2, "fp64", 7, 60.0)
    v = torch.zeros(s.shape, dtype=torch.float64, device="cuda")
    out = s.new()
    with pytest.raises(WhError) as ei:
        s.apply_A_noalloc(v, out)
    assert ei.value.status == wh.WH_EINVAL
    assert "static scratch holds" in wh.wh_last_error(s.ctx)
    # the context still works through its workspace
    s.apply_A(v, out=out)
    assert float(out.abs().max()) == 0.0
