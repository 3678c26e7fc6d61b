"""The C ABI's validation and error reporting on a GPU, through the raw
binding: grid limits, call order, workspace size and alignment, host and
device pointers, aliasing, non-finite data; and the degenerate grids (one
interior node) through every kernel family against the oracle."""
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


def _status(fn, *args):
    from paper_2504_03074_amd import WhError
    try:
        fn(*args)
    except WhError as e:
        return e.status
    return 0


def test_grid_limits(torch):
    from paper_2504_03074_amd import wh
    _say("[abi] grid limits")
    ctx = wh.wh_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        for dim, n, order, prec in [(1, (8, 8, 8), 2, wh.WH_FP64), (4, (8, 8, 8), 2, wh.WH_FP64),
                                    (2, (8, 8), 3, wh.WH_FP64), (2, (1, 8), 2, wh.WH_FP64),
                                    (2, (65536, 8), 2, wh.WH_FP64), (3, (2048, 2048, 2048), 2, wh.WH_FP64),
                                    (2, (8, 8), 2, 7)]:
            assert _status(wh.wh_set_grid, ctx, dim, n, order, prec) == wh.WH_EINVAL, (dim, n, order, prec)
        # at most 65535 cells per axis and 2^33 nodes (2049^3 is above it)
        assert _status(wh.wh_set_grid, ctx, 2, (65535, 2), 4, wh.WH_FP64) == 0
        assert wh.wh_last_error(ctx) == ""
    finally:
        wh.wh_destroy(ctx)


def test_call_order_workspace_and_pointers(torch):
    from paper_2504_03074_amd import wh
    _say("[abi] call order, workspace, pointers")
    ctx = wh.wh_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        n = (20, 18)
        shape = (n[1] + 1, n[0] + 1)
        # nothing before the grid
        assert _status(wh.wh_set_c2_constant, ctx, 1.0) == wh.WH_ESTATE
        wh.wh_set_grid(ctx, 2, n, 2, wh.WH_FP64)
        # no workspace yet
        assert _status(wh.wh_set_c2_constant, ctx, 1.0) == wh.WH_ENOMEM
        need = wh.wh_workspace_size(ctx, 2)
        ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        assert _status(wh.wh_bind_workspace, ctx, ws.data_ptr(), need - 256, 2) == wh.WH_ENOMEM
        assert _status(wh.wh_bind_workspace, ctx, ws.data_ptr() + 8, need, 2) == wh.WH_EINVAL
        host = np.zeros(need // 8 + 64)
        hp = (host.ctypes.data + 255) // 256 * 256
        assert _status(wh.wh_bind_workspace, ctx, hp, need, 2) == wh.WH_EINVAL
        wh.wh_bind_workspace(ctx, ws.data_ptr(), need, 2)
        # frequency before c^2, solve before frequency
        assert _status(wh.wh_set_frequency, ctx, 9.0) == wh.WH_ESTATE
        assert _status(wh.wh_set_c2_constant, ctx, -1.0) == wh.WH_EINVAL
        assert _status(wh.wh_set_c2_constant, ctx, float("nan")) == wh.WH_EINVAL
        wh.wh_set_c2_constant(ctx, 1.2)
        assert _status(wh.wh_set_frequency, ctx, -3.0) == wh.WH_EINVAL
        v = torch.zeros(shape, dtype=torch.float64, device="cuda")
        out = torch.zeros_like(v)
        assert _status(wh.wh_apply_A, ctx, v.data_ptr(), out.data_ptr()) == wh.WH_ESTATE
        wh.wh_set_frequency(ctx, 9.0)
        # forcing without a source
        assert _status(wh.wh_apply, ctx, v.data_ptr(), out.data_ptr(), True) == wh.WH_ESTATE
        # aliasing and host pointers
        assert _status(wh.wh_apply_A, ctx, v.data_ptr(), v.data_ptr()) == wh.WH_EINVAL
        hv = np.zeros(shape)
        assert _status(wh.wh_apply_A, ctx, hv.ctypes.data, out.data_ptr()) == wh.WH_EINVAL
        assert _status(wh.wh_apply_A, ctx, v.data_ptr(), hv.ctypes.data) == wh.WH_EINVAL
        # a valid call works after all the rejected ones, and A 0 = 0
        wh.wh_apply_A(ctx, v.data_ptr(), out.data_ptr())
        assert float(out.abs().max()) == 0.0
        assert wh.wh_status_string(wh.WH_EINVAL) == "WH_EINVAL"
    finally:
        wh.wh_destroy(ctx)


def test_non_finite_source_is_reported(torch):
    from paper_2504_03074_amd import Solver, WhError
    from paper_2504_03074_amd import wh
    _say("[abi] non-finite")
    s = Solver(2, (24, 20), order=2, restart=4)
    s.set_c2(1.0)
    f = np.zeros(s.shape)
    f[5, 7] = np.nan
    s.set_source(f)
    s.set_frequency(8.0)
    for method in ("gmres", "cg"):
        with pytest.raises(WhError) as e:
            s.solve(method=method, rtol=1e-8, maxit=20)
        assert e.value.status == wh.WH_ENONFINITE, method


@pytest.mark.parametrize("dim,n,order,kernel,kblock", [
    (2, (2, 2), 2, "node", 0), (2, (2, 2), 4, "blocked_2d", 4), (2, (2, 3), 4, "blocked_2d", 2),
    (3, (2, 2, 2), 2, "node", 0), (3, (2, 2, 2), 4, "zcol_3d", 0), (3, (2, 3, 2), 4, "blocked_3d", 2),
    (3, (2, 2, 2), 2, "blocked_3d", 4)])
def test_single_interior_node_grids(torch, dim, n, order, kernel, kblock):
    """The smallest grids (one or two interior nodes) through every kernel
    family, FP64, against the oracle."""
    from paper_2504_03074_amd import Solver
    _say(f"[abi] tiny grid {dim}D n={n} p={order} {kernel} K={kblock}")
    grid = oc.Grid(dim, n, order)
    c2 = 0.9 + 0.2 * wl.random_field(grid.shape, seed=901, zero_walls=False) ** 2
    f = wl.random_field(grid.shape, seed=902)
    v = wl.random_field(grid.shape, seed=903)
    s = Solver(dim, n, order=order)
    s.set_tuning(kernel, kblock, 0)
    s.set_c2(c2)
    s.set_source(f)
    s.set_frequency(3.0)
    tp = oc.time_params(grid, c2, 3.0)
    got = s.apply(torch.from_numpy(v).cuda(), with_forcing=True).cpu().numpy()
    want = oc.apply(grid, c2, f, v, tp, with_forcing=True)
    assert np.linalg.norm(got - want) <= 1e-11 * np.linalg.norm(want)


def test_stream_bandwidth_reference_kernels(torch):
    """The streaming-bandwidth reference (used only to read rooflines): each
    kind moves what it says, and bad sizes, kinds and overlaps are rejected."""
    from paper_2504_03074_amd import wh
    _say("[abi] streaming reference kernels")
    dev = torch.device("cuda:0")
    nodes = 4096
    g = torch.Generator(device="cpu").manual_seed(11)
    a = torch.rand(nodes, generator=g, dtype=torch.float32).to(dev)
    b = torch.empty_like(a)
    ms = wh.wh_stream_bandwidth(0, a.data_ptr(), b.data_ptr(), nodes * 4, 0, 2)
    torch.cuda.synchronize()
    assert ms > 0 and torch.equal(a, b)
    wh.wh_stream_bandwidth(2, 0, b.data_ptr(), nodes * 4, 0, 1)
    torch.cuda.synchronize()
    assert torch.equal(b.view(-1, 4).cpu(), torch.tensor([[1.0, 2.0, 3.0, 4.0]]).expand(nodes // 4, 4))
    wh.wh_stream_bandwidth(1, a.data_ptr(), 0, nodes * 4, 0, 1)
    # kind 3: src = (W^{n-1}, W^n, c^2), dst = (out_prev, out_cur, FP64 acc)
    src = torch.rand(3 * nodes, generator=g, dtype=torch.float32).to(dev)
    acc0 = torch.rand(nodes, generator=g, dtype=torch.float64)
    dst = torch.zeros(4 * nodes, dtype=torch.float32, device=dev)
    dst.view(torch.float64)[nodes:] = acc0.to(dev)
    reps = 3  # one untimed launch and three timed ones: the accumulator gains four increments
    wh.wh_stream_bandwidth(3, src.data_ptr(), dst.data_ptr(), 36 * nodes, 0, reps)
    torch.cuda.synchronize()
    ip, ic, c2 = src.cpu().view(3, nodes)
    out_cur = dst[nodes:2 * nodes].cpu()
    assert torch.equal(dst[:nodes].cpu(), ic)
    # (2 W^n - W^{n-1}) + c^2 W^n in FP32 (the device may fuse the last multiply-add)
    assert torch.allclose(out_cur, (ic + ic - ip) + c2 * ic, rtol=1e-6, atol=1e-6)
    want = acc0.clone()
    for _ in range(reps + 1):
        want += 0.5 * out_cur.double()
    assert torch.allclose(dst.view(torch.float64)[nodes:].cpu(), want, rtol=0, atol=1e-12)
    # rejected: unknown kind, a size that is not whole vectors (or 144-byte
    # groups for kind 3), overlapping buffers, too many repetitions
    for args in ((4, a.data_ptr(), b.data_ptr(), nodes * 4, 0, 1),
                 (0, a.data_ptr(), b.data_ptr(), 8, 0, 1),
                 (3, src.data_ptr(), dst.data_ptr(), 36 * nodes + 36, 0, 1),
                 (3, src.data_ptr(), src.data_ptr() + 512, 36 * 64, 0, 1),
                 (0, a.data_ptr(), a.data_ptr() + 64, 1024, 0, 1),
                 (0, a.data_ptr(), b.data_ptr(), nodes * 4, 0, 10001)):
        assert _status(wh.wh_stream_bandwidth, *args) == wh.WH_EINVAL, args
