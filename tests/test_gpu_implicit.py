"""GPU parity of implicit time stepping (Sec. 4.2.2) against the oracle:
one application W_h(v, f) and A v with variable c^2 (FP64 1e-11), sine modes
filtered by beta_d(lambda~_i) and the predicted implicit rate, fixed-count
FPI iterates, a Krylov solve reaching the discrete Helmholtz solution, a grid
without coarsening, and the error paths."""
import math
import sys

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
from oracle import implicit as oi
import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-11
INNER = 1e-14


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


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _solver(n, order, c2, f, omega, nits, periods=1, restart=2):
    from paper_2504_03074_amd import Solver
    s = Solver(2, n, order=order, restart=restart)
    s.set_c2(c2)
    s.set_source(f)
    s.set_implicit(nits, INNER)
    s.set_frequency(omega, periods=periods)
    return s


def _var_c2(grid, seed):
    g = wl.random_field(grid.shape, seed=seed, zero_walls=False)
    return 0.7 + 0.8 / (1.0 + np.exp(-g))


@pytest.mark.parametrize("n,order,nits,periods", [((64, 48), 2, 10, 1), ((64, 48), 4, 7, 1), ((96, 40), 4, 10, 2),
                                                  ((37, 30), 2, 6, 1)])
def test_implicit_apply_matches_oracle(torch, n, order, nits, periods):
    _say(f"[implicit apply] n={n} p={order} nits={nits} periods={periods}")
    grid = oc.Grid(2, n, order)
    c2 = _var_c2(grid, 801 + order)
    f = wl.random_field(grid.shape, seed=802)
    v = wl.random_field(grid.shape, seed=803)
    omega = 14.0
    s = _solver(n, order, c2, f, omega, nits, periods)
    tp = oi.time_params_implicit(omega, nits, periods)
    got_tp = s.time_params
    assert got_tp["nt"] == nits and got_tp["dt"] == pytest.approx(tp["dt"], rel=1e-14)
    assert got_tp["omega_e"] == pytest.approx(tp["omega_e"], rel=1e-14)
    st = oi.ImplicitStepper(grid, c2, tp["dt"])
    vd = _dev(torch, v)
    got = s.apply(vd, with_forcing=True).cpu().numpy()
    assert _rel(got, oi.apply_implicit(grid, c2, f, v, tp, stepper=st)) <= TOL
    gotA = s.apply_A(vd).cpu().numpy()
    assert _rel(gotA, oi.apply_A_implicit(grid, c2, v, tp, stepper=st)) <= TOL
    fin, fil = s.run_periods(vd, with_forcing=True)
    want_fil, want_fin = oi.apply_implicit(grid, c2, f, v, tp, return_final=True, stepper=st)
    assert _rel(fin.cpu().numpy(), want_fin) <= TOL
    stats = s.implicit_stats()
    assert stats["steps"] == 3 * nits * periods and stats["inner_iters"] >= stats["steps"]
    # levels: halve while both axes are even, and only while theta n^2 > 1/2
    theta = 0.5 * tp["dt"] ** 2
    levels, (nx, ny) = 1, n
    while nx % 2 == 0 and ny % 2 == 0 and nx >= 4 and ny >= 4 and theta * max(nx, ny) ** 2 > 0.5:
        nx, ny, levels = nx // 2, ny // 2, levels + 1
    assert stats["levels"] == levels


@pytest.mark.parametrize("order", [2, 4])
def test_implicit_sine_modes_and_rate(torch, order):
    _say(f"[implicit sine] p={order}")
    n = (48, 40)
    grid = oc.Grid(2, n, order)
    c2, omega, nits = 1.3, 12.5, 8
    s = _solver(n, order, c2, np.zeros(grid.shape), omega, nits)
    tp = oi.time_params_implicit(omega, nits)
    for k in [(1, 1), (3, 5), (47, 39), (20, 2)]:
        phi = np.multiply.outer(np.sin(k[1] * math.pi * np.arange(n[1] + 1) / n[1]),
                                np.sin(k[0] * math.pi * np.arange(n[0] + 1) / n[0]))
        lam = math.sqrt(c2 * sum(float(cf.lambda_h_sq_1d(km * math.pi, 1.0 / nm, order)) for km, nm in zip(k, n)))
        beta = float(cf.beta_d_tp(oi.lambda_tilde_implicit(lam, tp["dt"]), tp))
        got = s.apply(_dev(torch, phi), with_forcing=False).cpu().numpy()
        assert np.abs(got - beta * phi).max() <= TOL * max(1.0, abs(beta)), k
    _, info = s.solve(method="fpi", rtol=0.0, maxit=1)
    mu, _ = oi.predicted_rate_implicit(grid, c2, tp)
    assert info["mu_pred"] == pytest.approx(mu, rel=1e-10)


def test_implicit_fpi_iterates(torch):
    _say("[implicit fpi]")
    n = (40, 36)
    grid = oc.Grid(2, n, 4)
    c2 = _var_c2(grid, 811)
    f = wl.random_field(grid.shape, seed=812)
    s = _solver(n, 4, c2, f, 10.0, 9)
    tp = oi.time_params_implicit(10.0, 9)
    _, hist = oi.fpi_implicit(grid, c2, f, tp, 6)
    for k in (1, 6):
        v, info = s.solve(method="fpi", rtol=0.0, maxit=k)
        assert info["iters"] == k
        assert _rel(v.cpu().numpy(), hist[k - 1]) <= TOL, k


@pytest.mark.parametrize("method", ["cg", "gmres"])
def test_implicit_krylov_reaches_dhs(torch, method):
    _say(f"[implicit {method}]")
    n = (64, 56)
    grid = oc.Grid(2, n, 4)
    c2 = _var_c2(grid, 821)
    f = wl.random_field(grid.shape, seed=822)
    s = _solver(n, 4, c2, f, 16.0, 10, restart=60)
    v, info = s.solve(method=method, rtol=1e-11, maxit=3000, restart=60)
    assert info["converged"]
    U = cf.dhs_direct(grid, c2, f, 16.0)
    assert _rel(v.cpu().numpy(), U) <= 1e-8


def test_implicit_errors_and_switching(torch):
    from paper_2504_03074_amd import Solver, WhError
    from paper_2504_03074_amd import wh
    _say("[implicit errors]")
    grid = oc.Grid(2, (32, 32), 2)
    f = wl.random_field(grid.shape, seed=831)
    v = wl.random_field(grid.shape, seed=832)
    s3 = Solver(3, (8, 8, 8), order=2)
    with pytest.raises(WhError):
        s3.set_implicit(10)
    s32 = Solver(2, (32, 32), order=2, precision="fp32")
    with pytest.raises(WhError):
        s32.set_implicit(10)
    s = Solver(2, (32, 32), order=2, restart=2)
    s.set_c2(1.0)
    s.set_source(f)
    with pytest.raises(WhError):
        s.set_implicit(4)
    with pytest.raises(WhError):
        s.set_implicit(10, 0.5)
    # without its workspace the implicit apply fails cleanly
    wh.wh_set_implicit(s.ctx, 10, 1e-12)
    s.set_frequency(9.0)
    with pytest.raises(WhError) as e:
        s.apply(_dev(torch, v), with_forcing=True)
    assert e.value.status == wh.WH_ESTATE
    s.set_implicit(10, INNER)
    s.set_frequency(9.0)
    got = s.apply(_dev(torch, v), with_forcing=True).cpu().numpy()
    tp = oi.time_params_implicit(9.0, 10)
    assert _rel(got, oi.apply_implicit(grid, 1.0, f, v, tp)) <= TOL
    with pytest.raises(WhError):
        s.autotune(1)
    with pytest.raises(WhError):
        s.gradient(_dev(torch, v), _dev(torch, v))
    b = wh.wh_batch_create(0, None)
    try:
        with pytest.raises(WhError):
            wh.wh_batch_add(b, s.ctx)
    finally:
        wh.wh_batch_destroy(b)
    # back to explicit: the explicit oracle again
    s.set_implicit(0)
    s.set_frequency(9.0)
    tpe = oc.time_params(grid, 1.0, 9.0)
    got = s.apply(_dev(torch, v), with_forcing=True).cpu().numpy()
    assert _rel(got, oc.apply(grid, 1.0, f, v, tpe)) <= TOL


def test_implicit_with_deflation(torch):
    """Alg. 3 on top of implicit stepping (constant c^2): the modes chosen are
    the slowest under the implicit mode map, and every inflated iterate is the
    DST-I closed form (1 - beta_i^k) U on kept modes, U on deflated ones."""
    _say("[implicit deflation]")
    n = (40, 36)
    grid = oc.Grid(2, n, 2)
    c2, omega, nits = 1.1, 12.0, 8
    f = wl.random_field(grid.shape, seed=841)
    s = _solver(n, 2, c2, f, omega, nits)
    tp = oi.time_params_implicit(omega, nits)
    modes, mu = s.set_deflation(count=10)
    inner = (slice(1, -1),) * 2
    lam2 = cf.mode_eigenvalues(grid, c2)
    beta = cf.beta_d_tp(oi.lambda_tilde_implicit(np.sqrt(lam2), tp["dt"]), tp)
    keep = np.ones(beta.shape, dtype=bool)
    for m in modes:
        keep[m[1] - 1, m[0] - 1] = False
    assert np.abs(beta[~keep]).min() >= np.abs(beta[keep]).max()
    assert mu == pytest.approx(float(np.abs(beta[keep]).max()), rel=1e-10)
    U = cf._dst(f[inner]) / (omega ** 2 - lam2)
    for k in (1, 5):
        v, info = s.solve(method="fpi", rtol=0.0, maxit=k)
        V = np.where(keep, (1.0 - beta ** k) * U, U)
        want = np.zeros(grid.shape)
        want[inner] = cf._idst(V)
        assert _rel(v.cpu().numpy(), want) <= TOL, k


def test_implicit_sine_modes_square_2048(torch):
    """The implicit rate theorem at the full 2048^2 size (p = 4, constant c^2,
    omega = 200, N_ITS = 10), through the whole multigrid hierarchy: sine
    modes come back scaled by beta_d(lambda~_i).  Inner tolerance 1e-12: the
    step operator's condition number here is about 350, so a tighter
    relative residual is near the rounding floor; the error budget of each
    solve is then about 1e-12 relative for these low and middle modes."""
    _say("[implicit sine 2048]")
    n = (2048, 2048)
    order, c2, omega, nits = 4, 1.3, 200.0, 10
    from paper_2504_03074_amd import Solver
    s = Solver(2, n, order=order, restart=2)
    s.set_c2(c2)
    s.set_source(np.zeros((n[1] + 1, n[0] + 1)))
    s.set_implicit(nits, 1e-12)
    s.set_frequency(omega)
    tp = oi.time_params_implicit(omega, nits)
    for k in [(1, 1), (5, 3), (200, 150)]:
        phi = np.multiply.outer(np.sin(k[1] * math.pi * np.arange(n[1] + 1) / n[1]),
                                np.sin(k[0] * math.pi * np.arange(n[0] + 1) / n[0]))
        lam = math.sqrt(c2 * sum(float(cf.lambda_h_sq_1d(km * math.pi, 1.0 / nm, order)) for km, nm in zip(k, n)))
        beta = float(cf.beta_d_tp(oi.lambda_tilde_implicit(lam, tp["dt"]), tp))
        got = s.apply(_dev(torch, phi), with_forcing=False).cpu().numpy()
        err = float(np.abs(got - beta * phi).max())
        _say(f"  mode {k}: beta {beta:.6f} max error {err:.2e}")
        assert err <= 1e-10 * max(1.0, abs(beta)), k
    stats = s.implicit_stats()
    theta = 0.5 * tp["dt"] ** 2
    levels, m = 1, n[0]
    while m % 2 == 0 and m >= 4 and theta * m ** 2 > 0.5:
        m, levels = m // 2, levels + 1
    assert stats["levels"] == levels and levels >= 4
    # multigrid-preconditioned CG: the inner count does not grow with the grid
    assert stats["max_inner"] <= 20, stats
