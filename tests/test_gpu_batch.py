"""GPU parity of batched solves: many independent 2-D problems (different
grids, frequencies and speeds) advanced by one launch per blocked pass, with
the CG iteration captured in a HIP graph and replayed.

Each problem is checked against the FP64 CPU oracle (bars as for single
problems: 1e-11 FP64, 1e-5 FP32 state) and against the single-problem path
of the library with the same kernel configuration.
"""
import sys

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-11, "fp32": 1e-5}

# n, c2 kind, omega, periods
MIX = [
    ((61, 47), "var", 25.0, 1),
    ((44, 37), "const", 12.0, 1),
    ((130, 67), "var", 41.0, 1),
    ((26, 21), "var", 9.0, 2),
    ((5, 7), "var", 3.0, 1),
]


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.fail("GPU test run without a GPU: the HIP path has no CPU fallback")
    return _t


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _err(prec, got, want, inp):
    scale = np.linalg.norm(want)
    if prec == "fp32":
        scale = max(scale, np.linalg.norm(inp))
    return float(np.linalg.norm(got - want) / scale)


class Prob:
    def __init__(self, n, c2kind, omega, periods, order, seed):
        self.grid = oc.Grid(2, n, order)
        if c2kind == "const":
            self.c2 = 1.3
        else:
            g = wl.random_field(self.grid.shape, seed=seed, zero_walls=False)
            self.c2 = 0.6 + 1.2 / (1.0 + np.exp(-g))
        self.f = wl.random_field(self.grid.shape, seed=seed + 1)
        self.v = wl.random_field(self.grid.shape, seed=seed + 2)
        self.omega, self.periods = omega, periods
        self.tp = oc.time_params(self.grid, self.c2, omega, periods=periods) if omega else None

    def solver(self, prec, order):
        from paper_2504_03074_amd import Solver
        s = Solver(2, self.grid.n, order=order, precision=prec, restart=2)
        s.set_c2(self.c2)
        s.set_source(self.f)
        s.set_frequency(self.omega, periods=self.periods)
        return s


def _mix(order, seed0=500):
    return [Prob(n, k, om, npd, order, seed0 + 10 * i) for i, (n, k, om, npd) in enumerate(MIX)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("forcing", [True, False])
def test_batch_apply(torch, prec, order, forcing):
    from paper_2504_03074_amd import Batch
    _say(f"[batch apply] {prec} p={order} forcing={forcing}")
    probs = _mix(order)
    solvers = [p.solver(prec, order) for p in probs]
    batch = Batch(solvers)
    vs = [_to_dev(torch, p.v) for p in probs]
    outs = batch.apply(vs, with_forcing=forcing)
    torch.cuda.synchronize()
    for p, s, v, o in zip(probs, solvers, vs, outs):
        got = o.cpu().numpy()
        want = oc.apply(p.grid, p.c2, p.f, p.v, p.tp, with_forcing=forcing)
        assert _err(prec, got, want, p.v) <= TOL[prec], p.grid.n
        single = s.apply(v, with_forcing=forcing).cpu().numpy()
        # same kernel body and tile configuration as the single-problem path
        assert _err(prec, got, single, p.v) <= (1e-14 if prec == "fp64" else 1e-6), p.grid.n


def test_batch_full_size_members_sampled(torch):
    """Batch members at the batched configuration's full sizes (256^2, 512^2
    and 1024^2, c = 1, 2nd order, Gaussian sources drawn as in the batched
    workload) together with the small mixed problems, the default tuning:
    W_h(v, f) of every full-size member at sampled nodes (corners, edges,
    the source peak, inner nodes) against the oracle on the domain of
    dependence, relative L2 over the samples <= 1e-11, and the
    single-problem path's result within 1e-14."""
    from paper_2504_03074_amd import Batch, Solver
    _say("[batch full-size members] 256^2, 512^2, 1024^2")
    draws = wl.batched_problems(64)
    picks = []
    for size in (256, 512, 1024):
        picks.append(next(p for p in draws if p["n"] == size))
    small = _mix(2, seed0=700)
    solvers, members = [], []
    for i, p in enumerate(picks):
        n = p["n"]
        grid = oc.Grid(2, (n, n), 2)
        f = wl.materialise_source(2, n, p["source"])
        v = wl.random_field(grid.shape, seed=900 + i)
        s = Solver(2, (n, n), order=2, precision="fp64", restart=2)
        s.set_c2(1.0)
        s.set_source(f)
        s.set_frequency(p["omega"], periods=p["periods"], cfl_frac=p["cfl"])
        solvers.append(s)
        members.append((grid, f, v, p))
    solvers += [q.solver("fp64", 2) for q in small]
    batch = Batch(solvers)
    vs = [_to_dev(torch, m[2]) for m in members] + [_to_dev(torch, q.v) for q in small]
    outs = batch.apply(vs, with_forcing=True)
    torch.cuda.synchronize()
    for (grid, f, v, p), s, vd, o in zip(members, solvers, vs, outs):
        n = grid.n[0]
        tp = oc.time_params(grid, 1.0, p["omega"], periods=p["periods"], cfl_frac=p["cfl"])
        assert s.time_params["nt"] == tp["nt"]
        peak = np.unravel_index(int(np.argmax(np.abs(f))), f.shape)
        pts = [(1, 1), (n - 1, n - 1), (2, n // 2), (n // 2, n - 3), (int(peak[1]), int(peak[0])),
               (n // 3, n // 4), (3 * n // 4, 2 * n // 3)]
        want = oc.apply_at_points(grid, 1.0, f, v, tp, pts, with_forcing=True)
        got = o.cpu().numpy()
        g = np.array([got[q[1], q[0]] for q in pts])
        err = _rel(g, want)
        _say(f"    {n}^2 omega {p['omega']:.1f} nt {tp['nt']}: rel L2 over {len(pts)} samples {err:.2e}")
        assert err <= TOL["fp64"]
        assert _rel(got, s.apply(vd, with_forcing=True).cpu().numpy()) <= 1e-14
    for q, o in zip(small, outs[len(members):]):
        want = oc.apply(q.grid, q.c2, q.f, q.v, q.tp, with_forcing=True)
        assert _rel(o.cpu().numpy(), want) <= TOL["fp64"], q.grid.n


@pytest.mark.parametrize("order,kblock,tile", [(4, 2, 40), (4, 3, 80), (4, 4, 40), (4, 6, 80), (2, 4, 32),
                                               (2, 8, 64)])
def test_batch_apply_tunings(torch, order, kblock, tile):
    from paper_2504_03074_amd import Batch
    _say(f"[batch apply tuning] p={order} K={kblock} rows={tile}")
    probs = _mix(order, seed0=600)
    batch = Batch([p.solver("fp64", order) for p in probs], kblock=kblock, tile=tile)
    outs = batch.apply([_to_dev(torch, p.v) for p in probs], with_forcing=True)
    for p, o in zip(probs, outs):
        want = oc.apply(p.grid, p.c2, p.f, p.v, p.tp, with_forcing=True)
        assert _rel(o.cpu().numpy(), want) <= TOL["fp64"], p.grid.n


def test_batch_autotune_then_apply(torch):
    from paper_2504_03074_amd import Batch
    _say("[batch autotune]")
    probs = _mix(4, seed0=620)
    batch = Batch([p.solver("fp64", 4) for p in probs])
    best = batch.autotune(1)
    assert best["kblock"] in (2, 3, 4, 5, 6) and best["tile"] in (40, 80) and best["ms_per_apply"] > 0
    assert batch.tuning() == dict(kblock=best["kblock"], tile=best["tile"])
    outs = batch.apply([_to_dev(torch, p.v) for p in probs], with_forcing=True)
    for p, o in zip(probs, outs):
        want = oc.apply(p.grid, p.c2, p.f, p.v, p.tp, with_forcing=True)
        assert _rel(o.cpu().numpy(), want) <= TOL["fp64"], p.grid.n


def test_batch_apply_repeated_with_other_inputs(torch):
    """The descriptor tables are rebuilt per call: a second call with other
    inputs must not see the first call's pointers."""
    from paper_2504_03074_amd import Batch
    _say("[batch apply repeated]")
    probs = _mix(2, seed0=650)
    batch = Batch([p.solver("fp64", 2) for p in probs])
    first = batch.apply([_to_dev(torch, p.v) for p in probs], with_forcing=False)
    second_in = [_to_dev(torch, 2.0 * p.f) for p in probs]
    second = batch.apply(second_in, with_forcing=False)
    for p, a, b in zip(probs, first, second):
        assert _rel(a.cpu().numpy(), oc.apply(p.grid, p.c2, p.f, p.v, p.tp, with_forcing=False)) <= 1e-11
        assert _rel(b.cpu().numpy(), oc.apply(p.grid, p.c2, p.f, 2.0 * p.f, p.tp, with_forcing=False)) <= 1e-11


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("iters", [1, 3, 12])
def test_batch_cg_fixed_iterations(torch, prec, iters):
    """k replays of the captured CG iteration against k eager oracle CG
    iterations, for every problem of the batch."""
    from paper_2504_03074_amd import Batch
    _say(f"[batch cg fixed] {prec} iters={iters}")
    probs = _mix(4, seed0=700)
    batch = Batch([p.solver(prec, 4) for p in probs])
    xs, infos = batch.solve(rtol=1e-300, maxit=iters)
    tol = 1e-11 if prec == "fp64" else 2e-5
    for p, x, inf in zip(probs, xs, infos):
        want, oinfo = oc.cg(p.grid, p.c2, p.f, p.tp, fixed_iters=iters)
        assert inf["iters"] == iters
        assert not inf["converged"]
        assert _rel(x.cpu().numpy(), want) <= tol, p.grid.n
        # reported residual is the true residual of the returned iterate,
        # evaluated in the state precision: with FP32 state it carries that
        # rounding (absolute, relative to ||b||)
        b = oc.apply(p.grid, p.c2, p.f, np.zeros(p.grid.shape), p.tp, with_forcing=True)
        r = b - oc.apply_A(p.grid, p.c2, want, p.tp)
        true_rel = np.linalg.norm(r) / np.linalg.norm(b)
        if prec == "fp64":
            assert inf["rel_res"] == pytest.approx(true_rel, rel=1e-8)
        else:
            assert abs(inf["rel_res"] - true_rel) <= TOL["fp32"]


@pytest.mark.parametrize("iters", [1, 7])
def test_batch_cg_with_given_rhs_fixed_iterations(torch, iters):
    """Batched CG on (I - S_h) x_i = b_i with given right-hand sides
    (wh_batch_solve_rhs), k iterations against k oracle CG iterations on the
    same b_i; a zero right-hand side leaves its problem at x = 0."""
    from paper_2504_03074_amd import Batch
    _say(f"[batch cg rhs] iters={iters}")
    probs = _mix(2, seed0=800)
    batch = Batch([p.solver("fp64", 2) for p in probs])
    bs = [wl.random_field(p.grid.shape, seed=810 + i) for i, p in enumerate(probs)]
    bs[1] = np.zeros(probs[1].grid.shape)
    xs, infos = batch.solve(rtol=1e-300, maxit=iters, b=[_to_dev(torch, b) for b in bs])
    for i, (p, x, inf, b) in enumerate(zip(probs, xs, infos, bs)):
        got = x.cpu().numpy()
        if i == 1:
            assert not got.any() and inf["rel_res"] == 0.0
            continue
        want, _ = oc.cg(p.grid, p.c2, p.f, p.tp, fixed_iters=iters, b=b)
        assert inf["iters"] == iters
        assert _rel(got, want) <= TOL["fp64"], p.grid.n


def test_batch_mixed_precision_refinement(torch):
    """Batched residual correction (wh_batch_solve_mixed): FP64 residuals of
    every problem, corrections by the batched FP32-state CG, reaching each
    problem's FP64 discrete Helmholtz solution (sparse direct solve) while
    the plain FP32-state batched solve does not."""
    from paper_2504_03074_amd import Batch
    _say("[batch mixed]")
    probs = []
    for i, (n, om_range) in enumerate([((40, 31), (5.0, 15.0)), ((33, 45), (6.0, 14.0)), ((52, 27), (4.0, 12.0))]):
        p = Prob(n, "var", 0.0, 1, 4, seed=850 + 10 * i)
        p.omega = _best_omega(p.grid, p.c2, np.linspace(*om_range, 17))
        p.tp = oc.time_params(p.grid, p.c2, p.omega)
        probs.append(p)
    hi = Batch([p.solver("fp64", 4) for p in probs])
    lo = Batch([p.solver("fp32", 4) for p in probs])
    xs, infos = hi.solve_mixed(lo, rtol=1e-11, maxit=40, inner_rtol=1e-4, inner_maxit=5000)
    x32, _ = lo.solve(rtol=1e-6, maxit=5000)
    for p, x, inf, y in zip(probs, xs, infos, x32):
        assert inf["converged"], inf
        U = cf.dhs_direct(p.grid, p.c2, p.f, p.omega)
        err = _rel(x.cpu().numpy(), U)
        err32 = _rel(y.cpu().numpy(), U)
        _say(f"    {p.grid.n} omega {p.omega:.2f}: {inf['iters']} corrections, mixed error {err:.2e}, "
             f"FP32-state solve error {err32:.2e}")
        assert err <= 1e-9
        assert err32 > 10 * err


def _best_omega(grid, c2, candidates):
    import scipy.sparse as sp
    inner = (slice(1, -1),) * grid.dim
    L = cf.laplacian_matrix(grid)
    c2i = (np.full(grid.shape, c2) if np.isscalar(c2) else c2)[inner].ravel()
    ev = np.linalg.eigvals((sp.diags(c2i) @ L).toarray())
    lam = np.sqrt(np.maximum(-ev.real, 0))
    best = None
    for om in candidates:
        tp = oc.time_params(grid, c2, om)
        gap = float(np.min(np.abs(1 - cf.beta_d_tp(cf.lambda_tilde(lam, tp["dt"]), tp))))
        if best is None or gap > best[1]:
            best = (om, gap)
    return best[0]


def test_batch_cg_converges_to_direct_solves(torch):
    """Problems that converge after different iteration counts leave the
    batch one by one (tables rebuilt, iteration recaptured); each solution
    matches the direct solve of its discrete Helmholtz problem."""
    from paper_2504_03074_amd import Batch
    _say("[batch cg converged]")
    probs = []
    for i, (n, order) in enumerate([((26, 21), 4), ((30, 19), 4), ((18, 24), 4), ((22, 22), 4)]):
        p = Prob(n, "var", 0.0, 1, order, seed=800 + 10 * i)
        p.omega = _best_omega(p.grid, p.c2, np.linspace(5.0 + i, 15.0 + i, 21))
        p.tp = oc.time_params(p.grid, p.c2, p.omega)
        probs.append(p)
    solvers = [p.solver("fp64", 4) for p in probs]
    batch = Batch(solvers)
    xs, infos = batch.solve(rtol=1e-12, maxit=5000)
    iters = [inf["iters"] for inf in infos]
    assert len(set(iters)) > 1, iters  # the subset path is exercised
    for p, s, x, inf in zip(probs, solvers, xs, infos):
        assert inf["converged"] and inf["rel_res"] <= 1e-12, inf
        U = cf.dhs_direct(p.grid, p.c2, p.f, p.omega)
        assert _rel(x.cpu().numpy(), U) <= 1e-9
        xs1, inf1 = s.solve(method="cg", rtol=1e-12, maxit=5000)
        assert abs(inf1["iters"] - inf["iters"]) <= max(2, inf1["iters"] // 50)


def test_batch_zero_source_and_resolve(torch):
    """A problem with zero source converges at once (x stays 0); a second
    solve started from the first solution stops after at most one iteration."""
    from paper_2504_03074_amd import Batch
    _say("[batch zero source / resolve]")
    probs = _mix(2, seed0=900)[:3]
    probs[1].f = np.zeros(probs[1].grid.shape)
    solvers = [p.solver("fp64", 2) for p in probs]
    batch = Batch(solvers)
    xs, infos = batch.solve(rtol=1e-9, maxit=3000)
    assert infos[1]["iters"] == 0 and infos[1]["converged"]
    assert float(xs[1].abs().max()) == 0.0
    for p, x, inf in zip(probs, xs, infos):
        if p is probs[1]:
            continue
        assert inf["converged"], inf
        b = oc.apply(p.grid, p.c2, p.f, np.zeros(p.grid.shape), p.tp, with_forcing=True)
        r = b - oc.apply_A(p.grid, p.c2, x.cpu().numpy(), p.tp)
        assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-9 * 1.01
    xs2, infos2 = batch.solve(rtol=1e-9, maxit=3000, x0=xs)
    for x, x2, inf in zip(xs, xs2, infos2):
        assert inf["iters"] <= 1
        assert float((x - x2).abs().max()) <= 1e-6 * max(float(x.abs().max()), 1e-300)


def test_batch_errors(torch):
    from paper_2504_03074_amd import Solver, WhError
    from paper_2504_03074_amd import wh
    _say("[batch errors]")
    p2 = Prob((20, 18), "var", 8.0, 1, 2, seed=950)
    p4 = Prob((20, 18), "var", 8.0, 1, 4, seed=960)
    s2, s4 = p2.solver("fp64", 2), p4.solver("fp64", 4)
    b = wh.wh_batch_create(0, None)
    try:
        wh.wh_batch_add(b, s2.ctx)
        with pytest.raises(WhError) as e:
            wh.wh_batch_add(b, s4.ctx)  # order differs
        assert e.value.status == wh.WH_EINVAL
        with pytest.raises(WhError) as e:
            wh.wh_batch_add(b, s2.ctx)  # added twice
        assert e.value.status == wh.WH_EINVAL
        s3 = Solver(3, (6, 6, 6), order=2, restart=2)
        s3.set_c2(1.0)
        s3.set_source(np.zeros(s3.shape))
        s3.set_frequency(3.0)
        with pytest.raises(WhError) as e:
            wh.wh_batch_add(b, s3.ctx)
        assert e.value.status == wh.WH_EINVAL
        s0 = Solver(2, (20, 18), order=2, restart=0)
        s0.set_c2(1.0)
        s0.set_source(np.zeros(s0.shape))
        s0.set_frequency(3.0)
        with pytest.raises(WhError) as e:
            wh.wh_batch_add(b, s0.ctx)
        assert e.value.status == wh.WH_ENOMEM
        v = s2.new()
        with pytest.raises(WhError) as e:
            wh.wh_batch_apply(b, [v.data_ptr()], [s2.new().data_ptr()], True)
        assert e.value.status == wh.WH_ESTATE
        with pytest.raises(WhError) as e:
            wh.wh_batch_set_tuning(b, 1, 0)
        assert e.value.status == wh.WH_EINVAL
        nbytes = wh.wh_batch_workspace_size(b)
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        with pytest.raises(WhError) as e:
            wh.wh_batch_finalize(b, ws.data_ptr(), nbytes - 1)
        assert e.value.status == wh.WH_ENOMEM
        wh.wh_batch_finalize(b, ws.data_ptr(), nbytes)
        opts, _ = wh.make_opts("gmres", 1e-8, 10)
        with pytest.raises(WhError) as e:
            wh.wh_batch_solve(b, opts, [v.data_ptr()])
        assert e.value.status == wh.WH_EINVAL
        with pytest.raises(WhError) as e:
            wh.wh_batch_apply(b, [v.data_ptr()], [v.data_ptr()], True)  # aliasing
        assert e.value.status == wh.WH_EINVAL
    finally:
        wh.wh_batch_destroy(b)
