"""Pins of the oracle's later options against what the paper and the
mathematics fix: the HLLE flux and the WENO5 / PPM reconstructions (Sec. 2.3,
2.4), the full 8x8 / 10x10 Newton system against the paper's reduced one
(Sec. 8.2), the chi = phi cs^2 tau_R, nu = psi cs^2 tau_R closure (Sec. 4,
4.1), the DeltaP saturation (Sec. 8.1, 9) and the firehose growth rate
(Sec. 8.1)."""
import numpy as np
import pytest

from paper_1702_01106_amd import workloads as W
from tests.helpers import prim_rel_err

XMID = np.array([0.0, 0.5, 0.5, 0.5])


def base(**kw):
    d = dict(W._BASE, ndim=1, n=[32], x_start=[0.0], x_end=[1.0], nvar=10, gamma=4.0 / 3.0, tau_R=1.0,
             chi=0.01, nu=0.01, name="next")
    d.update(kw)
    return d


# ---------------------------------------------------------------- HLLE

def _rest_state(n, seed):
    rng = np.random.default_rng(seed)
    P = np.zeros((10, 1, 1, n))
    P[0] = 1.0 + 0.1 * rng.uniform(-1, 1, n)
    P[1] = 1.0 + 0.1 * rng.uniform(-1, 1, n)
    P[5] = 0.1
    P[6] = 0.2 + 0.05 * rng.uniform(-1, 1, n)
    P[8] = 1e-3 * rng.uniform(-1, 1, n)
    P[9] = 1e-3 * rng.uniform(-1, 1, n)
    return P


def test_hlle_equals_llf_when_speeds_are_symmetric(oracle_mod):
    """Sec. 2.4.2: the two fluxes agree when the largest left- and right-going
    speeds are equal, as at every face of a fluid at rest (each state's
    speeds are +-v_max)."""
    P = _rest_state(32, 1)
    dl, _, _ = oracle_mod.Oracle(base()).explicit(P)
    dh, _, _ = oracle_mod.Oracle(base(riemann="hlle")).explicit(P)
    for v in range(10):
        scale = max(np.abs(dl[v]).max(), 1e-300)
        assert np.abs(dh[v] - dl[v]).max() <= 1e-12 * scale, v


def test_hlle_upwinds_supersonic_flow(oracle_mod):
    """Sec. 2.4.2: when every speed on both sides is positive the HLLE flux
    is the left state's flux.  Two uniform regions moving at 0.95 and 0.9
    with cold gas: the PLM slopes vanish next to the jump, so the zone right
    of it sees F(P_right) - F(P_left) exactly; LLF adds dissipation there."""
    n = 16
    wl = base(nvar=8, n=[n], bc=["outflow"] * 3)
    P = np.zeros((8, 1, 1, n))
    for sl, (rho, u, v) in ((slice(0, 8), (1.0, 0.01, 0.95)), (slice(8, 16), (2.0, 0.02, 0.9))):
        P[0, 0, 0, sl] = rho
        P[1, 0, 0, sl] = u
        P[2, 0, 0, sl] = v / np.sqrt(1 - v * v)
    oh = oracle_mod.Oracle(dict(wl, riemann="hlle"))
    pl, pr = P[:, 0, 0, 7], P[:, 0, 0, 8]
    for p in (pl, pr):
        assert oh.speeds(p, XMID, 1)[1] > 0.5  # the left-going speed is positive too
    dh, _, _ = oh.explicit(P)
    exp = (oh.flux(pr, XMID, 1) - oh.flux(pl, XMID, 1)) * n
    got = dh[:, 0, 0, 8]
    assert np.allclose(got, exp, rtol=1e-12, atol=1e-12 * np.abs(exp).max())
    dl, _, _ = oracle_mod.Oracle(wl).explicit(P)
    assert np.abs(dl[:, 0, 0, 8] - exp).max() > 1e-3 * np.abs(exp).max()
    # away from the jump nothing changes
    assert np.abs(dh[:, 0, 0, 3]).max() < 1e-12 and np.abs(dh[:, 0, 0, 12]).max() < 1e-12


# ---------------------------------------------------------------- WENO5 / PPM

@pytest.mark.parametrize("recon", ["plm", "weno5", "ppm"])
def test_reconstruction_exact_for_linear_data(oracle_mod, recon):
    """Every reconstruction returns the face value of linear data on both sides."""
    o = oracle_mod.Oracle(base(recon=recon, ng=3))
    s = 0.7 + 0.3 * np.arange(6)  # cells i-3..i+2
    lo, hi = o.reconstruct(s)
    face = 0.7 + 0.3 * 2.5
    assert abs(lo - face) < 1e-14 and abs(hi - face) < 1e-14


@pytest.mark.parametrize("recon", ["weno5", "ppm"])
def test_reconstruction_exact_for_quadratic_averages(oracle_mod, recon):
    """WENO5's three candidate stencils and PPM's fourth-order interface value
    are exact for the cell averages of a quadratic (here x^2 on unit cells
    away from its minimum, where PPM's monotonicity steps do nothing)."""
    o = oracle_mod.Oracle(base(recon=recon, ng=3))
    x = 10.0 + np.arange(6)           # cell centres of cells i-3..i+2
    s = x * x + 1.0 / 12.0            # averages of x^2 over [x - 1/2, x + 1/2]
    lo, hi = o.reconstruct(s)
    face = (x[2] + 0.5) ** 2
    assert abs(lo - face) < 1e-11 and abs(hi - face) < 1e-11


@pytest.mark.parametrize("recon", ["weno5", "ppm"])
def test_reconstruction_at_a_step(oracle_mod, recon):
    """Next to a jump neither operator overshoots: PPM's monotonicity
    constraint returns the cell values exactly; WENO5 puts its weight on the
    smooth stencil (within its epsilon-sized leak).  Reversing the data
    swaps the two states."""
    o = oracle_mod.Oracle(base(recon=recon, ng=3))
    s = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0])
    lo, hi = o.reconstruct(s)
    tol = 0.0 if recon == "ppm" else 1e-5
    assert abs(lo) <= tol and abs(hi - 1.0) <= tol, (lo, hi)
    rng = np.random.default_rng(3)
    r = rng.uniform(-1, 1, 6)
    a, b = o.reconstruct(r)
    c, d = o.reconstruct(r[::-1].copy())
    assert abs(a - d) < 1e-15 and abs(b - c) < 1e-15


def _alfven_error(oracle_mod, N, recon):
    wl = W.workload("srmhd1d_alfven_128", n=[N], plm_theta=2.0, tol=1e-13, recon=recon,
                    ng=3 if recon != "plm" else 2)
    o = oracle_mod.Oracle(wl)
    amp = 1e-5
    P = W.alfven_1d(wl, seed=0, amp=amp)
    tend = 1.0
    n = int(np.ceil(tend / o.cfl_dt(P, 0.5)))
    P1, st = o.step(P, tend / n, n)
    assert st["n_fail"] == 0
    vA = 0.1 / np.sqrt(1 + 8 / 3 + 0.1)
    phi = np.random.default_rng(0).uniform(0.0, 2.0 * np.pi)
    X1 = (np.arange(N) + 0.5) / N
    ex = amp * np.cos(2 * np.pi * (X1 - vA * tend) + phi)
    return np.abs(P1[4, 0, 0] - ex).mean() / amp


def test_weno5_and_ppm_alfven_convergence(oracle_mod):
    """The 1-D Alfven wave converges at second order (the scheme's order,
    Sec. 2.2) with either five-point reconstruction, and WENO5 is more
    accurate than PLM on the same grid."""
    e = {r: [_alfven_error(oracle_mod, N, r) for N in (64, 128)] for r in ("plm", "weno5", "ppm")}
    for r in ("weno5", "ppm"):
        assert e[r][0] / e[r][1] > 3.0, e
        assert e[r][1] < 1e-3, e
    assert e["weno5"][0] < e["plm"][0], e


# ---------------------------------------------------------------- full system

def test_full_system_has_the_same_root(oracle_mod):
    """Sec. 8.2: B is fixed by its explicit update, so Newton over all nvar
    primitives (B among the unknowns, started at that update) finds the root
    of the reduced system: the answers agree to what the tolerance leaves
    open, and B stays at its update."""
    rng = np.random.default_rng(11)
    wl = dict(W._BASE, ndim=2, n=[12, 10], x_start=[0, 0], x_end=[1, 1], nvar=10, gamma=4 / 3, tau_R=1.0,
              chi=0.01, nu=0.01, name="full")
    P = np.zeros((10, 1, 10, 12))
    P[0] = 1 + 0.1 * rng.uniform(-1, 1, P[0].shape)
    P[1] = 1 + 0.1 * rng.uniform(-1, 1, P[0].shape)
    P[2:5] = 0.1 * rng.uniform(-1, 1, P[2:5].shape)
    P[5:8] = 0.1 + 0.05 * rng.uniform(-1, 1, P[5:8].shape)
    P[8:10] = 1e-3 * rng.uniform(-1, 1, P[8:10].shape)
    o_r = oracle_mod.Oracle(wl)
    o_f = oracle_mod.Oracle(dict(wl, system="full"))
    dtp = 0.5 * o_r.cfl_dt(P, 0.5)
    Pr, itr, rrr, flr = o_r.stage(P, P, dtp)
    Pf, itf, rrf, flf = o_f.stage(P, P, dtp)
    assert np.all(flr == 0) and np.all(flf == 0)
    assert rrf.max() < wl["tol"] and rrr.max() < wl["tol"]
    assert prim_rel_err(Pf, Pr).max() < 1e-8
    # the B rows' residual at the update is rounding, so B moves by rounding
    assert np.abs(Pf[5:8] - Pr[5:8]).max() < 1e-12 * np.abs(Pr[5:8]).max()
    assert abs(itf.mean() - itr.mean()) <= 0.2 * itr.mean()


# ---------------------------------------------------------------- closure

@pytest.mark.parametrize("gam", [4.0 / 3.0, 5.0 / 3.0])
@pytest.mark.parametrize("phi,psi", [(1.0, 1.0), (5.0, 3.0), (0.3, 0.7)])
def test_closure_speed_is_the_simplified_form(oracle_mod, gam, phi, psi):
    """Sec. 4.1: with chi = phi cs^2 tau_R and nu = psi cs^2 tau_R, eq. modcs
    reduces to ct^2 = cs^2/2 (1 + (gamma-1) phi + sqrt(1 + (gamma-1)^2 phi^2)
    + 8 psi/3), whatever tau_R is."""
    rho, u = 1.3, 0.8
    cs2 = gam * (gam - 1) * u / (rho + gam * u)
    ct2 = 0.5 * cs2 * (1 + (gam - 1) * phi + np.sqrt(1 + (gam - 1) ** 2 * phi ** 2) + 8 * psi / 3)
    P = np.array([rho, u, 0, 0, 0, 0, 0, 0, 0, 0.0])
    for tau in (0.37, 20.0):
        o = oracle_mod.Oracle(base(gamma=gam, tau_R=tau, closure=True, phi=phi, psi=psi))
        assert abs(o.vmax2(P, XMID) - ct2) < 1e-14


def test_closure_scales_the_relaxation_targets(oracle_mod):
    """Sec. 4: with q = DeltaP = 0 and P = P_n = P^E, the q and DeltaP rows of
    the residual are -qtilde_0 / tau_R and -DPtilde_0 / tau_R, which are
    sqrt(rho chi / tau_R) and sqrt(rho nu / tau_R) times P^E-only factors.
    With the closure, chi / tau_R = phi cs^2 of each zone's P^E, so against
    constant chi_0, nu_0 each zone's rows change by sqrt(phi cs^2 tau_R /
    chi_0) and sqrt(psi cs^2 tau_R / nu_0).  (Their flux terms vanish: the
    face q and DeltaP are zero, and so is every rescaled U_q, U_DP jump.)"""
    rng = np.random.default_rng(5)
    n = [12, 10]
    wl = dict(W._BASE, ndim=2, n=n, x_start=[0, 0], x_end=[1, 1], nvar=10, gamma=4 / 3, tau_R=0.5,
              chi=0.02, nu=0.03, name="closure")
    P = np.zeros((10, 1, 10, 12))
    X1, X2, _ = W.zone_centres(wl)
    P[0] = 1 + 0.2 * np.sin(2 * np.pi * X1)
    P[1] = 1 + 0.3 * np.cos(2 * np.pi * X2)
    P[2] = 0.05 * np.sin(2 * np.pi * X2)
    P[3] = 0.05 * np.cos(2 * np.pi * X1)
    P[5], P[6] = 0.1, 0.05
    phi, psi = 0.7, 1.9
    o0 = oracle_mod.Oracle(wl)
    oc = oracle_mod.Oracle(dict(wl, closure=True, phi=phi, psi=psi))
    dtp = 1e-3
    R0, _ = o0.residual(P, P, dtp, P)
    Rc, _ = oc.residual(P, P, dtp, P)
    g = 4 / 3
    cs2 = g * (g - 1) * P[1] / (P[0] + g * P[1])
    for row, coef, c0 in ((8, phi, 0.02), (9, psi, 0.03)):
        ok = np.abs(R0[row]) > 1e-8 * np.abs(R0[row]).max()
        assert ok.mean() > 0.5
        ratio = Rc[row][ok] / R0[row][ok]
        assert np.allclose(ratio, np.sqrt(coef * cs2[ok] * 0.5 / c0), rtol=1e-12)


# ---------------------------------------------------------------- saturation

@pytest.mark.parametrize("side", ["firehose", "mirror"])
def test_dp_saturates_at_the_instability_thresholds(oracle_mod, side):
    """Sec. 8.1 and 9: DeltaP saturates near -b^2 (firehose) and b^2/2
    (mirror) through a smooth reduction of tau_R.  A uniform magnetised state
    at rest with DeltaP five times past the threshold and tau_R = 100 relaxes
    to within 35% past the threshold by t = 4 and stops there; without the
    saturation it barely moves."""
    n = 16
    b2 = 0.01
    thr = -b2 if side == "firehose" else 0.5 * b2
    P = np.zeros((10, 1, 1, n))
    P[0], P[1], P[5] = 1.0, 1.0, 0.1
    P[9] = 5.0 * thr
    wl = base(n=[n], tau_R=100.0, closure=True, phi=1.0, psi=1.0)
    res = {}
    for sat in (False, True):
        o = oracle_mod.Oracle(dict(wl, dp_saturation=sat))
        dt = o.cfl_dt(P, 0.5)
        nst = int(np.ceil(4.0 / dt))
        P1, st = o.step(P.copy(), 4.0 / nst, nst)
        assert st["n_fail"] == 0
        res[sat] = P1[9] / thr
        assert np.ptp(P1[9]) < 1e-12 * abs(thr)
    assert np.all(res[False] > 4.5), res[False]
    assert np.all((res[True] > 1.0) & (res[True] < 1.35)), res[True]


# ---------------------------------------------------------------- firehose

def test_firehose_growth_rate(oracle_mod):
    """Sec. 8.1, firehose test: the Alfven mode with DeltaP = -0.011 < -b^2
    grows at Gamma = 0.1036 (tau_R = 1e6 freezes DeltaP).  256 zones, t in
    [0.5, 3]: the fitted rate is within 4% of the paper's (numerical
    dissipation slows it slightly)."""
    N = 256
    wl = dict(W._BASE, ndim=1, n=[N], x_start=[0.0], x_end=[1.0], nvar=10, gamma=4 / 3, tau_R=1e6,
              chi=0.01, nu=0.01, plm_theta=1.5, tol=1e-12, name="firehose")
    o = oracle_mod.Oracle(wl)
    P = W.firehose_1d(wl, alpha=1e-4)
    X1 = (np.arange(N) + 0.5) / N
    dt = o.cfl_dt(P, 0.5)
    ts, amps = [], []
    t, chunk = 0.0, 16
    while t < 3.0:
        P, st = o.step(P, dt, chunk)
        assert st["n_fail"] == 0
        t += chunk * dt
        ts.append(t)
        amps.append(2.0 / N * np.sum(P[6, 0, 0] * np.cos(2 * np.pi * X1)))
    ts, amps = np.array(ts), np.array(amps)
    keep = ts >= 0.5
    gam = np.polyfit(ts[keep], np.log(amps[keep]), 1)[0]
    assert abs(gam - 0.1036) < 0.04 * 0.1036, gam
