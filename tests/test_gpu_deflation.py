"""GPU parity of WaveHoltz with deflation (Alg. 3) against the oracle:
the selected modes and predicted deflated rate, deflated fixed-point
iterates at fixed iteration counts (FP64 1e-11), the measured deflated rate,
and deflated Krylov solves against the discrete Helmholtz solution."""
import sys

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
from oracle import deflation as od
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _solver(grid, c2, f, omega, restart=2, precision="fp64"):
    from paper_2504_03074_amd import Solver
    s = Solver(grid.dim, grid.n, order=grid.order, restart=restart, precision=precision)
    s.set_c2(c2)
    s.set_source(f)
    s.set_frequency(omega)
    return s


CASES = [
    # dim, n, order, c2, omega, count
    (2, (40, 33), 2, 1.0, 14.0, 8),
    (2, (36, 30), 4, 1.7, 16.0, 20),
    (3, (10, 9, 11), 2, 1.2, 7.0, 6),
]


@pytest.mark.parametrize("dim,n,order,c2,omega,count", CASES)
def test_selected_modes_and_deflated_fpi(torch, dim, n, order, c2, omega, count):
    _say(f"[deflation fpi] dim={dim} n={n} p={order} c2={c2} omega={omega} count={count}")
    grid = oc.Grid(dim, n, order)
    f = wl.random_field(grid.shape, seed=520 + dim + order)
    s = _solver(grid, c2, f, omega)
    tp = oc.time_params(grid, c2, omega)
    modes, mu = s.set_deflation(count=count)
    want_modes, want_mu = od.select_modes(grid, c2, tp, count)
    assert set(modes) == set(want_modes)
    assert mu == pytest.approx(want_mu, rel=1e-10)
    for k in (1, 5, 12):
        v, info = s.solve(method="fpi", rtol=0.0, maxit=k)
        assert info["iters"] == k
        want, _ = od.fpi_deflated(grid, c2, f, tp, want_modes, k)
        assert _rel(v.cpu().numpy(), want) <= 1e-11, k
        assert info["mu_pred"] == pytest.approx(want_mu, rel=1e-10)


def test_c1_workload_deflated(torch):
    """The 128^2 single-Gaussian configuration, 30 deflated iterations."""
    _say("[deflation C1]")
    w = wl.single_gaussian_source()
    grid = oc.Grid(2, (w["n"], w["n"]), w["order"])
    s = _solver(grid, w["c2"], w["f"], w["omega"])
    tp = oc.time_params(grid, w["c2"], w["omega"])
    modes, mu = s.set_deflation(count=16)
    mu_full, _ = cf.predicted_rate(grid, w["c2"], tp)
    assert mu < mu_full
    v, info = s.solve(method="fpi", rtol=0.0, maxit=w["fpi_iters"])
    want, _ = od.fpi_deflated(grid, w["c2"], w["f"], tp, modes, w["fpi_iters"])
    assert _rel(v.cpu().numpy(), want) <= 1e-11


def test_measured_rate_is_the_deflated_rate(torch):
    _say("[deflation rate]")
    grid = oc.Grid(2, (48, 40), 2)
    f = wl.random_field(grid.shape, seed=531)
    s = _solver(grid, 1.0, f, 15.0)
    modes, mu = s.set_deflation(count=10)
    v, info = s.solve(method="fpi", rtol=0.0, maxit=80)
    assert info["cr_last"] == pytest.approx(mu, rel=5e-3)
    tp = oc.time_params(grid, 1.0, 15.0)
    U = cf.helmholtz_closed_form(grid, 1.0, f, 15.0)
    assert _rel(v.cpu().numpy(), U) <= 2.0 * mu ** 80 + 1e-12


@pytest.mark.parametrize("method", ["cg", "gmres"])
def test_deflated_krylov_reaches_dhs(torch, method):
    _say(f"[deflation {method}]")
    grid = oc.Grid(2, (44, 38), 4)
    c2 = 1.3
    f = wl.random_field(grid.shape, seed=541)
    omega = 17.0
    s = _solver(grid, c2, f, omega, restart=40)
    plain, pinfo = s.solve(method=method, rtol=1e-11, maxit=5000, restart=40)
    s.set_deflation(count=30)
    v, info = s.solve(method=method, rtol=1e-11, maxit=5000, restart=40)
    assert info["converged"] and pinfo["converged"]
    assert info["iters"] < pinfo["iters"]
    U = cf.helmholtz_closed_form(grid, c2, f, omega)
    assert _rel(v.cpu().numpy(), U) <= 1e-8
    assert _rel(v.cpu().numpy(), plain.cpu().numpy()) <= 1e-8


def test_deflation_errors_and_clearing(torch):
    from paper_2504_03074_amd import WhError
    from paper_2504_03074_amd import wh
    _say("[deflation errors]")
    grid = oc.Grid(2, (20, 18), 2)
    f = wl.random_field(grid.shape, seed=551)
    s = _solver(grid, 1.0, f, 8.0)
    with pytest.raises(WhError) as e:
        s.set_deflation(modes=[(1, 1), (1, 1)])
    assert e.value.status == wh.WH_EINVAL
    with pytest.raises(WhError) as e:
        s.set_deflation(modes=[(20, 1)])
    assert e.value.status == wh.WH_EINVAL
    s.set_deflation(count=4)
    b = s.new()
    with pytest.raises(WhError) as e:
        s.solve(method="cg", rtol=1e-8, maxit=10, b=b)
    assert e.value.status == wh.WH_EINVAL
    _, info_d = s.solve(method="fpi", rtol=0.0, maxit=2)
    s.set_c2(1.0)  # clears deflation
    s.set_frequency(8.0)
    _, info_p = s.solve(method="fpi", rtol=0.0, maxit=2)
    tp = oc.time_params(grid, 1.0, 8.0)
    assert info_p["mu_pred"] == pytest.approx(cf.predicted_rate(grid, 1.0, tp)[0], rel=1e-10)
    assert info_d["mu_pred"] < info_p["mu_pred"]
    from paper_2504_03074_amd import wh as whm
    s2 = _solver(grid, 1.0, f, 8.0)
    s2.set_deflation(count=2)
    b = whm.wh_batch_create(0, None)
    try:
        with pytest.raises(WhError) as e:
            whm.wh_batch_add(b, s2.ctx)  # the batched solve does not deflate
        assert e.value.status == wh.WH_EINVAL
    finally:
        whm.wh_batch_destroy(b)
    g = wl.random_field(grid.shape, seed=552, zero_walls=False)
    s.set_c2(0.8 + 0.1 * g ** 2)
    s.set_frequency(8.0)
    with pytest.raises(WhError) as e:
        s.set_deflation(count=3)
    assert e.value.status == wh.WH_EINVAL
