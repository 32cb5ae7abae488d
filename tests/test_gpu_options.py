"""Parity of the HIP path's later options with the oracle, through the C ABI:
the HLLE flux and the WENO5 / PPM reconstructions (Sec. 2.3, 2.4), the full
8x8 / 10x10 Newton system (Sec. 8.2's comparison form), the chi = phi cs^2
tau_R, nu = psi cs^2 tau_R closure and the DeltaP saturation (Sec. 4, 8.1,
9), and the paper's firehose and Table 1 tests run on the GPU.

Bounds are those of the plain method's parity tests: the explicit stage to
1e-11 of its scale (1e-9 in Kerr, where the two sides difference the metric
with different stencils) plus face-flux rounding, stage roots to 1e-6 of
max(|P_v|, family RMS) or what the tolerance leaves open (bench.compare_stage)
with the oracle's residual at the GPU root below 2 tol."""
import numpy as np
import pytest

import bench
from paper_1702_01106_amd import workloads as W
from tests.helpers import prim_rel_err
from tests.test_gpu_parity import _flux_scale, _perturbed, _say, _state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(wl):
    from paper_1702_01106_amd import grim

    return grim.Context(wl)


def _emhd2d(**kw):
    return dict(W.small("emhd2d_modes_256", [70, 45]), **kw)


CASES = {
    # name: (workload, state generator name of test_gpu_parity._state)
    "hlle_emhd2d": (lambda: _emhd2d(riemann="hlle"), "emhd2d_ragged"),
    "weno5_emhd2d": (lambda: _emhd2d(recon="weno5", ng=3), "emhd2d_ragged"),
    "ppm_ideal2d": (lambda: dict(W.small("emhd2d_modes_256", [33, 20]), nvar=8, recon="ppm", ng=3), "ideal2d"),
    "closure_emhd2d": (lambda: _emhd2d(closure=True, phi=0.7, psi=1.9), "emhd2d_ragged"),
    "sat_emhd2d": (lambda: _emhd2d(closure=True, phi=0.7, psi=1.9, dp_saturation=True), "sat"),
    "hlle_weno5_emhd3d": (lambda: dict(W._BASE, ndim=3, n=[12, 10, 7], x_start=[0, 0, 0], x_end=[1, 1, 1], nvar=10,
                                       gamma=4 / 3, tau_R=1.0, chi=0.01, nu=0.01, riemann="hlle", recon="weno5",
                                       ng=3, name="hw3d"), "emhd3d"),
    "ppm_kerr_emhd": (lambda: W.small("emhd3d_kerr_192", [28, 24, 6], recon="ppm", ng=3), "kerr_emhd"),
    "hlle_kerr_ideal": (lambda: W.small("grmhd3d_kerr_128", [28, 24, 6], riemann="hlle"), "kerr_ideal"),
    "full_emhd2d": (lambda: _emhd2d(system="full"), "emhd2d_ragged"),
    "full_ideal1d": (lambda: W.small("srmhd1d_alfven_128", [300], system="full"), "srmhd1d_300"),
    "full_kerr_emhd": (lambda: W.small("emhd3d_kerr_192", [28, 24, 6], system="full"), "kerr_emhd"),
}
KERR = ("ppm_kerr_emhd", "hlle_kerr_ideal", "full_kerr_emhd")


def _case(name):
    mk, st = CASES[name]
    wl = mk()
    if st == "sat":
        # DeltaP up to three times past the thresholds in most zones
        P = _state("emhd2d_ragged", wl)
        rng = np.random.default_rng(17)
        b2 = P[5] ** 2 + P[6] ** 2 + P[7] ** 2
        P[9] = b2 * rng.uniform(-3.0, 1.5, P[9].shape)
        return wl, P
    return wl, _state(st, wl)


@pytest.mark.parametrize("name", [n for n in CASES if not n.startswith("full")])
def test_explicit_stage_options(torch_cuda, oracle_mod, name):
    wl, P = _case(name)
    _say(f"explicit stage {name} n={wl['n']}")
    o = oracle_mod.Oracle(wl)
    dF, src, sp = o.explicit(P)
    gdF, gsrc, gsp = (x.cpu().numpy() for x in _ctx(wl).explicit(P))
    kerr = name in KERR
    tdf, tsrc = (1e-9, 1e-7) if kerr else (1e-11, 1e-12)
    fmax = _flux_scale(o, wl, P)
    idx = sum(wl["n"][d] / (wl["x_end"][d] - wl["x_start"][d]) for d in range(wl["ndim"]))
    for v in range(wl["nvar"]):
        scale = max(np.abs(dF[v]).max(), 1e-300)
        floor = 32 * np.finfo(float).eps * fmax[v] * idx
        err = np.abs(gdF[v] - dF[v]).max()
        assert err <= tdf * scale + floor, (v, err, scale, floor)
    assert np.abs(gsrc - src).max() <= tsrc * max(np.abs(src).max(), 1.0)
    if wl["nvar"] == 10:
        for q in range(3):
            scale = max(np.abs(sp[:, q]).max(), 1e-300)
            assert np.abs(gsp[:, q] - sp[:, q]).max() <= (1e-7 if kerr else 1e-11) * scale + 1e-14, q


@pytest.mark.parametrize("jac", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_stage_solve_options(torch_cuda, oracle_mod, name, jac):
    """One stage solve from P_n with a perturbed P^E: every zone converges and
    the root is the oracle's within the tolerance-implied bound."""
    wl, Pn = _case(name)
    wl = dict(wl, jac=jac)
    o = oracle_mod.Oracle(wl)
    dtp = 0.5 * o.cfl_dt(Pn, 0.5)
    PE = _perturbed(Pn, 4, 1e-4, 1e-3)
    _say(f"stage solve {name} jac={jac}")
    ref, it, rr, fl = o.stage(Pn, PE, dtp)
    assert np.all(fl == 0), np.unique(fl, return_counts=True)
    gP, git, grr, gfl = (x.cpu().numpy() for x in _ctx(wl).stage_solve(Pn, PE, dtp))
    assert np.all((gfl & ~np.uint8(32)) == 0), np.unique(gfl)
    assert jac == "f32" or np.all(gfl == 0)
    rep = bench.compare_stage(o, wl, Pn, o.fill_ghosts(PE), dtp, gP, ref, rr)
    _say(f"  rel {rep['rel']}")
    assert rep["within"], rep
    if jac == "f64" and name not in KERR:
        assert np.abs(git.astype(int) - it).max() <= 1
        assert np.mean(git == it) >= 0.9, np.mean(git == it)


@pytest.mark.parametrize("name", ["hlle_emhd2d", "weno5_emhd2d", "ppm_ideal2d", "sat_emhd2d", "ppm_kerr_emhd",
                                  "full_emhd2d", "full_kerr_emhd"])
def test_steps_options(torch_cuda, oracle_mod, name):
    """Three full steps in the benchmark's launch configuration
    (graph replay), which exercise each stage's ghost images (three layers
    for WENO5 / PPM, with the outflow and polar maps in Kerr) and the flux
    stage on the GPU's own half step; against the oracle's three steps."""
    wl, P0 = _case(name)
    o = oracle_mod.Oracle(wl)
    dt = o.cfl_dt(P0, 0.5)
    nst = 3
    _say(f"steps {name} x{nst}")
    ref, st = o.step(P0, dt, nst)
    g = _ctx(wl)
    g.set_prims(P0)
    assert abs(g.cfl_dt(0.5) - dt) <= 1e-13 * dt
    gst = g.run(dt, nst, use_graph=True)
    gP = g.get_prims()
    assert gst["n_fail"] == st["n_fail"] == 0
    err = prim_rel_err(gP, ref).reshape(wl["nvar"], -1).max(axis=1)
    _say(f"  max err {np.array2string(err, precision=1)}")
    # three steps of the parity bound: per-stage roots agree to what the
    # tolerance leaves open, which the next stages carry forward
    bound = 1e-6 if name not in KERR else 1e-5
    assert np.all(err[:5] < bound), err
    assert np.all(err[5:8] < 1e-9), err
    if wl["nvar"] == 10 and name not in KERR:
        assert np.all(err[8:] < 1e-4), err


def test_full_system_matches_reduced_on_the_gpu(torch_cuda):
    """Sec. 8.2: the GPU's 10x10 and 7x7 solves of one stage land on the same
    root (both within the tolerance), with B at its explicit update."""
    wl, Pn = _case("full_emhd2d")
    dtp = 2e-3
    a = _ctx(dict(wl, system="reduced"))
    b = _ctx(wl)
    Pa, ia, ra, fa = (x.cpu().numpy() for x in a.stage_solve(Pn, Pn, dtp))
    Pb, ib, rb, fb = (x.cpu().numpy() for x in b.stage_solve(Pn, Pn, dtp))
    assert np.all(fa == 0) and np.all(fb == 0)
    assert prim_rel_err(Pb, Pa).max() < 1e-8
    assert np.abs(Pb[5:8] - Pa[5:8]).max() < 1e-12 * np.abs(Pa[5:8]).max()


def test_firehose_growth_on_the_gpu(torch_cuda, oracle_mod):
    """Sec. 8.1, firehose test, on the GPU (256 zones, t = 3): the mode grows
    at the paper's Gamma = 0.1036 within 4%, and the final state matches the
    oracle's run to the accumulated tolerance."""
    N = 256
    wl = dict(W._BASE, ndim=1, n=[N], x_start=[0.0], x_end=[1.0], nvar=10, gamma=4 / 3, tau_R=1e6, chi=0.01,
              nu=0.01, plm_theta=1.5, tol=1e-12, name="firehose")
    P0 = W.firehose_1d(wl, alpha=1e-4)
    X1 = (np.arange(N) + 0.5) / N
    g = _ctx(wl)
    g.set_prims(P0)
    dt = g.cfl_dt(0.5)
    ts, amps, t = [], [], 0.0
    while t < 3.0:
        st = g.run(dt, 16, use_graph=True)
        assert st["n_fail"] == 0
        t += 16 * dt
        P = g.get_prims()
        ts.append(t)
        amps.append(2.0 / N * np.sum(P[6, 0, 0] * np.cos(2 * np.pi * X1)))
    ts, amps = np.array(ts), np.array(amps)
    keep = ts >= 0.5
    gam = np.polyfit(ts[keep], np.log(amps[keep]), 1)[0]
    _say(f"firehose growth rate {gam:.5f} (paper 0.1036)")
    assert abs(gam - 0.1036) < 0.04 * 0.1036, gam
    ref, _ = oracle_mod.Oracle(wl).step(P0, dt, 16 * len(ts))
    assert np.abs(P[6] - ref[6]).max() < 1e-6 * np.abs(ref[6]).max()


def _table1_error(wl_base, N):
    from paper_1702_01106_amd import grim  # noqa: F401

    wl = dict(wl_base, n=[N, N])
    amp = 1e-6
    P = W.table1_mode(wl, 0.0, amp)
    g = _ctx(wl)
    g.set_prims(P)
    tend = 0.5
    n = int(np.ceil(tend / g.cfl_dt(0.5)))
    st = g.run(tend / n, n, use_graph=True)
    assert st["n_fail"] == 0
    P1 = g.get_prims()
    ex = W.table1_mode(wl, tend, amp)
    return np.array([np.abs(P1[v] - ex[v]).mean() / amp for v in range(10)])


def test_table1_sweep_on_the_gpu(torch_cuda):
    """Sec. 8.1.1, Table 1: the EMHD linear mode with the paper's closure
    (chi = nu = cs^2 tau_R, tau_R = 1) from 32^2 to 512^2 to t = 0.5: the L1
    error of rho, u, q and DeltaP falls at second order over the sweep (the
    least-squares order over 64^2..512^2 at least 1.8, and no doubling gains
    less than 2.8) and ends below 1e-4 of the amplitude."""
    base = dict(W._BASE, ndim=2, n=[32, 32], x_start=[0, 0], x_end=[1, 1], nvar=10, gamma=4 / 3, tau_R=1.0,
                closure=True, phi=1.0, psi=1.0, tol=1e-13, plm_theta=2.0, name="table1")
    errs = []
    for N in (32, 64, 128, 256, 512):
        errs.append(_table1_error(base, N))
        _say(f"table 1 N={N}: " + " ".join(f"{errs[-1][v]:.2e}" for v in (0, 1, 8, 9)))
    E = np.array(errs)
    Ns = np.array([32, 64, 128, 256, 512])
    for v in (0, 1, 8, 9):
        ratios = E[:-1, v] / E[1:, v]
        order = -np.polyfit(np.log(Ns[1:]), np.log(E[1:, v]), 1)[0]
        _say(f"  v={v}: order {order:.2f}, ratios {np.array2string(ratios, precision=2)}")
        assert order >= 1.8 and np.all(ratios > 2.8), (v, order, ratios)
        assert E[-1, v] < 1e-4, (v, E[-1, v])
