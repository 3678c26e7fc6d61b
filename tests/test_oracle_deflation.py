"""Pins of the deflation oracle (Alg. 3) against the DST-I closed forms of the
sine basis: every deflated iterate, the deflated convergence rate of the
theorem on deflated convergence, the converged inflated result equal to the
discrete Helmholtz solution, orthonormality of the modes; planted mistakes in
a copy of the deflation source must fail one of these pins."""
import importlib.util
import os

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import core as oc
from oracle import deflation as od
import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "deflation.py")


def _closed_form_deflated(grid, c2, f, tp, modes, k):
    """Iterate k of Alg. 3 (inflated) by DST-I: each kept coefficient is
    (1 - beta^k) U, each deflated one U after inflation."""
    inner = (slice(1, -1),) * grid.dim
    fh = cf._dst(np.asarray(f, dtype=np.float64)[inner])
    lam2 = cf.mode_eigenvalues(grid, c2)
    U = fh / (tp["omega"] ** 2 - lam2)
    beta = cf.beta_d_tp(cf.lambda_tilde(np.sqrt(lam2), tp["dt"]), tp)
    V = (1.0 - beta ** k) * U
    for m in modes:
        V[tuple(km - 1 for km in reversed(m))] = U[tuple(km - 1 for km in reversed(m))]
    out = np.zeros(grid.shape)
    out[inner] = cf._idst(V)
    return out


CASES = [
    # dim, n, order, c2, omega, count
    (2, (24, 20), 2, 1.0, 10.3, 6),
    (2, (18, 22), 4, 1.7, 12.0, 10),
    (3, (8, 7, 9), 2, 1.2, 6.0, 5),
]


def _check(mod, case, iters=(1, 4, 15)):
    dim, n, order, c2, omega, count = case
    grid = oc.Grid(dim, n, order)
    f = wl.random_field(grid.shape, seed=510 + dim)
    tp = oc.time_params(grid, c2, omega)
    modes, mu_after = mod.select_modes(grid, c2, tp, count)
    err = {}
    _, hist = mod.fpi_deflated(grid, c2, f, tp, modes, max(iters), inflate_result=False)
    worst = 0.0
    for k in iters:
        got = mod.inflate(grid, c2, f, tp["omega"], modes, hist[k - 1])
        want = _closed_form_deflated(grid, c2, f, tp, modes, k)
        worst = max(worst, float(np.linalg.norm(got - want) / np.linalg.norm(want)))
    err["iterates"] = worst
    # the deflated modes are those with the largest |beta_d|
    lam2 = cf.mode_eigenvalues(grid, c2)
    beta = np.abs(cf.beta_d_tp(cf.lambda_tilde(np.sqrt(lam2), tp["dt"]), tp))
    mask = np.ones(beta.shape, dtype=bool)
    for m in modes:
        mask[tuple(km - 1 for km in reversed(m))] = False
    err["selection"] = float(max(0.0, beta[mask].max() - min(beta[tuple(km - 1 for km in reversed(m))]
                                                               for m in modes)))
    err["mu"] = abs(mu_after - float(beta[mask].max()))
    return err, grid, f, tp, modes, mu_after


@pytest.mark.parametrize("case", CASES)
def test_deflated_iterates_match_closed_form(case):
    err, *_ = _check(od, case)
    assert err["iterates"] <= 1e-12, err
    assert err["selection"] == 0.0 and err["mu"] == 0.0, err


def test_sine_modes_orthonormal():
    grid = oc.Grid(2, (9, 7), 4)
    modes = [(1, 1), (2, 1), (8, 6), (3, 5)]
    G = np.array([[np.sum(od.sine_mode(grid, a) * od.sine_mode(grid, b)) for b in modes] for a in modes])
    assert np.allclose(G, np.eye(len(modes)), atol=1e-14)
    # and they are eigenvectors of the oracle's operator with the stated eigenvalue
    for k in modes:
        phi = od.sine_mode(grid, k)
        Lphi = oc.laplacian(grid, 1.3, phi)
        assert np.linalg.norm(Lphi + od.mode_eigenvalue(grid, 1.3, k) * phi) <= 1e-12 * np.linalg.norm(Lphi)


def test_deflated_rate_and_converged_solution():
    """Theorem (deflated convergence): the iterate differences contract by
    max |beta_d| over the kept modes; the inflated limit is the DHS."""
    case = (2, (24, 20), 2, 1.0, 10.3, 6)
    err, grid, f, tp, modes, mu_after = _check(od, case, iters=(1,))
    mu_full, _ = cf.predicted_rate(grid, 1.0, tp)
    assert mu_after < mu_full
    _, hist = od.fpi_deflated(grid, 1.0, f, tp, modes, 60, inflate_result=False)
    d = [np.linalg.norm(hist[k + 1] - hist[k]) for k in range(len(hist) - 1)]
    rate = d[-1] / d[-2]
    assert rate == pytest.approx(mu_after, rel=2e-3)
    k = int(np.ceil(np.log(1e-13) / np.log(mu_after)))
    out, _ = od.fpi_deflated(grid, 1.0, f, tp, modes, k)
    U = cf.helmholtz_closed_form(grid, 1.0, f, tp["omega"])
    assert np.linalg.norm(out - U) <= 1e-10 * np.linalg.norm(U)


MUTATIONS = [
    ("mode normalization dropped", "axes.append(math.sqrt(2.0 / nm) * np.sin(", "axes.append(np.sin("),
    ("inflation with the wrong sign", "/ (omega ** 2 - mode_eigenvalue(grid, c2, k))",
     "/ (mode_eigenvalue(grid, c2, k) - omega ** 2)"),
    ("fastest modes deflated instead of slowest", "order = np.argsort(-beta, kind=\"stable\")",
     "order = np.argsort(beta, kind=\"stable\")"),
    ("eigenvalue without c^2", "return float(c2) * sum(", "return sum("),
]


@pytest.mark.parametrize("desc,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_deflation_mistake_is_caught(tmp_path, desc, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    path = tmp_path / "deflation_mutant.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("oracle.deflation_mutant", str(path))
    mod = importlib.util.module_from_spec(spec)
    mod.__package__ = "oracle"
    spec.loader.exec_module(mod)
    caught = False
    for case in CASES[:2]:
        try:
            err, *_ = _check(mod, case)
        except Exception:
            caught = True
            break
        if err["iterates"] > 1e-12 or err["selection"] != 0.0 or err["mu"] != 0.0:
            caught = True
            break
    assert caught, desc
