"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point the header declares, reports status codes, rejects bad
arguments, and computes the time parameters exactly as the oracle does (two
independent implementations of the explicit correction recipe, Appendix A.1).
"""
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wh.h")


def _lib():
    from paper_2504_03074_amd import wh
    return wh


def test_library_exports_every_declared_symbol():
    wh = _lib()
    wh.library()
    declared = set(re.findall(r"^WH_API[^\n(]*?\b(wh_\w+)\s*\(", open(HEADER).read(), re.M))
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", wh.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = declared - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"
    extra = {s for s in exported if s.startswith("wh_")} - declared
    assert not extra, f"exported but not declared: {sorted(extra)}"


def test_status_strings_and_version():
    wh = _lib()
    assert wh.wh_version() >= 10000
    names = {s: wh.wh_status_string(s) for s in range(-7, 1)}
    assert names[0] == "WH_OK" and names[-4] == "WH_EUNSTABLE" and names[-7] == "WH_ESTATE"
    assert wh.wh_status_string(-99) == "unknown wh_status"


CASES = [
    (2, (128, 128), 2, 1.0, 10.3, 1), (2, (2048, 2048), 4, 2.0, 200.0, 1), (3, (512, 512, 512), 2, 2.25, 80.0, 1),
    (3, (512, 512, 512), 4, 2.25, 80.0, 1), (2, (61, 47), 4, 1.7, 33.3, 2), (3, (21, 18, 15), 2, 1.3, 12.5, 3),
    (2, (1024, 1024), 2, 1.0, 60.0, 1), (2, (256, 512), 2, 1.0, 149.9, 1), (2, (4, 4), 2, 1.0, 1.0, 1),
]


@pytest.mark.parametrize("dim,n,order,c2max,omega,periods", CASES)
def test_time_params_agree_with_oracle(dim, n, order, c2max, omega, periods):
    from oracle import core as oc
    wh = _lib()
    tp = wh.wh_compute_time_params(dim, n, order, c2max, omega, periods).as_dict()
    ref = oc.time_params(oc.Grid(dim, tuple(n), order), c2max, omega, periods=periods)
    assert tp["nt"] == ref["nt"]
    assert tp["periods"] == periods
    for key in ("dt", "omega_e", "alpha"):
        assert tp[key] == pytest.approx(ref[key], rel=1e-14)
    assert tp["cfl"] == pytest.approx(ref["nu"], rel=1e-14)
    assert tp["cfl"] <= 0.9 * oc.stability_constant(order) * (1 + 1e-14)


def test_time_params_overrides_and_errors():
    wh = _lib()
    base = wh.wh_compute_time_params(2, (64, 64), 2, 1.0, 10.0).as_dict()
    forced = wh.wh_compute_time_params(2, (64, 64), 2, 1.0, 10.0, nt_override=base["nt"] + 7, alpha=0.5).as_dict()
    assert forced["nt"] == base["nt"] + 7 and forced["alpha"] == 0.5
    with pytest.raises(wh.WhError) as e:  # too few steps for the stability limit
        wh.wh_compute_time_params(2, (64, 64), 2, 1.0, 10.0, nt_override=6)
    assert e.value.status == wh.WH_EUNSTABLE
    bad = [dict(dim=1), dict(order=3), dict(c2max=0.0), dict(c2max=float("nan")), dict(omega=-1.0),
           dict(periods=0), dict(cfl_frac=1.5), dict(cfl_frac=0.0), dict(nt_override=4), dict(n=(1, 64)),
           dict(alpha=float("inf"))]
    for kw in bad:
        args = dict(dim=2, n=(64, 64), order=2, c2max=1.0, omega=10.0, periods=1, cfl_frac=0.9, nt_override=0,
                    alpha=-1.0)
        args.update(kw)
        with pytest.raises(wh.WhError) as e:
            wh.wh_compute_time_params(**args)
        assert e.value.status == wh.WH_EINVAL, kw


def test_cfl_is_stable_limit_fraction():
    """The chosen dt is the largest dt = (2/omega) sin(pi/Nt) within the limit:
    one step fewer would exceed it (Nt minimal)."""
    wh = _lib()
    for order in (2, 4):
        limit = 1.0 if order == 2 else math.sqrt(3) / 2
        tp = wh.wh_compute_time_params(2, (300, 200), order, 1.8, 41.0).as_dict()
        root = math.sqrt(300 ** 2 + 200 ** 2)
        dt_less = (2 / 41.0) * math.sin(math.pi / (tp["nt"] - 1))
        assert math.sqrt(1.8) * dt_less * root > 0.9 * limit


def test_create_without_device_fails_cleanly():
    """On a machine without a GPU wh_create must report WH_EDEVICE, not crash."""
    wh = _lib()
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        pytest.skip("a GPU is present")
    with pytest.raises(wh.WhError) as e:
        wh.wh_create(0)
    assert e.value.status == wh.WH_EDEVICE


def test_null_context_is_rejected():
    wh = _lib()
    lib = wh.library()
    assert lib.wh_set_grid(None, 2, wh._n3((8, 8)), 2, 0) == wh.WH_EINVAL
    assert lib.wh_last_error(None) == b"no context"
    lib.wh_destroy(None)  # accepted
