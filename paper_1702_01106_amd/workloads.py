"""Seeded synthetic workloads: configuration presets and initial data.

This module is shared by the GPU path and the CPU oracle's tests.  It holds
no arithmetic of the method (no residual, flux, reconstruction, wave speed,
solver or geometry of the solve): only the shapes and parameters of the
workloads and the seeded initial states, drawn with
``numpy.random.default_rng(seed)`` (PCG64).

Arrays are float64, structure of arrays [nvar][n3][n2][n1] (interior zones,
i fastest).  Primitive order: rho, u, utilde^1..3, B^1..3[, q, DeltaP].
"""
from __future__ import annotations

import copy

import numpy as np

GAMMA_43 = 4.0 / 3.0

_BASE = {
    "ng": 2,
    "plm_theta": 1.0,
    "tol": 1e-10,
    "eps_fd": 1.4901161193847656e-08,
    "eps_bt": 1e-4,
    "k_max": 20,
    "ls_max": 10,
    "metric": "minkowski",
    "bc": ["periodic", "periodic", "periodic"],
    "jac": "f64",
    "guess": "pn",
    "cfl": 0.5,
    "floors": False,
}

WORKLOADS = {
    # 1D special-relativistic ideal MHD, 128 zones, one linear wave, 10 steps
    "srmhd1d_alfven_128": dict(
        ndim=1, n=[128], x_start=[0.0], x_end=[1.0], nvar=8, gamma=GAMMA_43, steps=10),
    # 2D EMHD, 256^2, 16 random Fourier modes in rho and u, 50 steps
    "emhd2d_modes_256": dict(
        ndim=2, n=[256, 256], x_start=[0.0, 0.0], x_end=[1.0, 1.0], nvar=10, gamma=GAMMA_43,
        tau_R=1.0, chi=0.01, nu=0.01, steps=50),
    # the same 2D EMHD setup at 512^2 (learned-guess workload), 50 steps
    "emhd2d_modes_512": dict(
        ndim=2, n=[512, 512], x_start=[0.0, 0.0], x_end=[1.0, 1.0], nvar=10, gamma=GAMMA_43,
        tau_R=1.0, chi=0.01, nu=0.01, steps=50),
}


# The line search keeps each new lambda within [0.1, 0.5] of the previous one
# on the torus: with the update as printed, a full Newton step far worse than
# f(0) gives lambda ~ f(0)/f(1) and Newton crawls in the atmosphere next to
# the torus (seen on a 28 x 24 x 6 EMHD torus in the CPU tests).
# Atmosphere floors rho >= 1e-3 r^-3/2, u >= 1e-3 r^-5/2: on r <= 40 they keep
# u above the finite-difference rule's absolute threshold 5 eps ~ 7.5e-8 for
# "small" primitives (Sec. 3.1), where the u column of the Jacobian would be
# taken with a step of half of u and the EMHD rescalings (~u^-1/2) make it
# inaccurate enough to stall Newton.
_KERR = dict(
    metric="mks", spin=0.9375, hslope=0.3, gamma=13.0 / 9.0,
    x_start=[float(np.log(1.3)), 0.0, 0.0], x_end=[float(np.log(40.0)), 1.0, float(2.0 * np.pi)],
    bc=["outflow", "polar", "periodic"], floors=True, rho_floor=1e-3, u_floor=1e-3, ls_safeguard=1,
    torus=dict(r_in=6.0, r_max=12.0, kappa=1e-3, beta=100.0, noise=0.04),
)

WORKLOADS.update({
    # 3D ideal GRMHD, Kerr a=0.9375 in modified Kerr-Schild, FM torus, 20 steps
    "grmhd3d_kerr_128": dict(_KERR, ndim=3, n=[128, 128, 64], nvar=8, steps=20, ic="kerr_torus"),
    # 3D EMHD in Kerr, same torus, chi = nu = 0.01, tau_R = 1, 20 steps
    "emhd3d_kerr_192": dict(_KERR, ndim=3, n=[192, 192, 96], nvar=10, tau_R=1.0, chi=0.01, nu=0.01,
                            steps=20, ic="kerr_torus"),
})


def workload(name: str, **over) -> dict:
    """A full configuration dictionary for a named workload (copy)."""
    d = copy.deepcopy(_BASE)
    d.update(copy.deepcopy(WORKLOADS[name]))
    d["name"] = name
    d.update(over)
    return d


def small(name: str, n, **over) -> dict:
    """The named workload's physics on a smaller grid (for parity tests)."""
    return workload(name, n=list(n), **over)


def zone_centres(wl: dict):
    """Coordinates X^i of zone centres, each shaped (n3, n2, n1)."""
    n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
    xs = list(wl["x_start"]) + [0.0] * (3 - len(wl["x_start"]))
    xe = list(wl["x_end"]) + [1.0] * (3 - len(wl["x_end"]))
    ax = [xs[d] + (np.arange(n[d]) + 0.5) * (xe[d] - xs[d]) / n[d] for d in range(3)]
    X3, X2, X1 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return X1, X2, X3


def _empty(wl):
    n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
    return np.zeros((wl["nvar"], n[2], n[1], n[0]))


def alfven_1d(wl: dict, seed: int = 0, amp: float = 1e-4):
    """Right-going Alfven wave on the background rho=1, u=2, B=(0.1, 0.3, 0) at rest.

    Linear SR-MHD about a static state with k along X1 and B^3 = 0: the mode
    polarised along X3 has du^3 = A cos(phase), dB^3 = -sqrt(w) du^3 with
    w = rho + gamma u + B^2, and moves at +B^1/sqrt(w).  The phase offset is
    drawn from the seed.
    """
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * np.pi)
    P = _empty(wl)
    X1, _, _ = zone_centres(wl)
    rho0, u0, B = 1.0, 2.0, (0.1, 0.3, 0.0)
    w = rho0 + wl["gamma"] * u0 + sum(b * b for b in B)
    ph = np.cos(2.0 * np.pi * X1 + phi)
    P[0] = rho0
    P[1] = u0
    P[4] = amp * ph
    P[5] = B[0]
    P[6] = B[1]
    P[7] = B[2] - np.sqrt(w) * amp * ph
    return P


def fourier_modes_2d(wl: dict, seed: int = 0, nmodes: int = 16, amp: float = 1e-3,
                     B=(0.05, 0.05, 0.0), rho0: float = 1.0, u0: float = 1.0):
    """rho = rho0 + sum_j amp cos(2 pi (m_j x + n_j y) + phi_j), u likewise with an
    independent set; (m_j, n_j) uniform integers in [-8, 8]^2 without (0, 0)."""
    rng = np.random.default_rng(seed)
    P = _empty(wl)
    X1, X2, _ = zone_centres(wl)

    def field():
        f = np.zeros_like(X1)
        for _ in range(nmodes):
            while True:
                m, n = rng.integers(-8, 9, size=2)
                if m != 0 or n != 0:
                    break
            ph = rng.uniform(0.0, 2.0 * np.pi)
            f += amp * np.cos(2.0 * np.pi * (m * X1 + n * X2) + ph)
        return f

    P[0] = rho0 + field()
    P[1] = u0 + field()
    P[5] = B[0]
    P[6] = B[1]
    P[7] = B[2]
    return P


# Table 1 of the paper: EMHD linear mode, background and eigenvector.
TABLE1_BACKGROUND = np.array([1.0, 2.0, 0.0, 0.0, 0.0, 0.1, 0.3, 0.0, 0.0, 0.0])
TABLE1_EIGENVECTOR = np.array([
    -0.518522524082246 - 0.1792647678001878j,
    0.5516170736393813 + 0.0j,
    0.008463122479547856 + 0.011862022608466367j,
    -0.16175466371870734 - 0.034828080823603294j,
    0.0 + 0.0j,
    -0.05973794979640743 - 0.03351707506150924j,
    0.02986897489820372 + 0.016758537530754618j,
    0.0 + 0.0j,
    0.5233486841539436 + 0.04767672501939603j,
    0.2909106062057657 + 0.02159452055336572j,
])
TABLE1_OMEGA = -0.5533585207638141 - 3.6262571286888425j
TABLE1_K = (2.0 * np.pi, 4.0 * np.pi)


def table1_mode(wl: dict, t: float = 0.0, amp: float = 1e-8):
    """P = P0 + amp Re(dP exp(i (k1 x + k2 y) + omega t)) (Sec. 8.1.1, Table 1)."""
    P = _empty(wl)
    X1, X2, _ = zone_centres(wl)
    ph = np.exp(1j * (TABLE1_K[0] * X1 + TABLE1_K[1] * X2) + TABLE1_OMEGA * t)
    for v in range(10):
        P[v] = TABLE1_BACKGROUND[v] + amp * np.real(TABLE1_EIGENVECTOR[v] * ph)
    return P


def firehose_1d(wl: dict, alpha: float = 1e-4, dP: float = -0.011):
    """Firehose-unstable Alfven mode (Sec. 8.1, firehose test): rho = 1, u = 2,
    u^2 = A sin(2 pi x^1), B = (0.1, B cos(2 pi x^1), 0), DeltaP = dP, with
    A = 0.1628 alpha and B = 0.9867 alpha (the paper prints cos(2 pi x^2)
    for B^2; the mode varies along x^1)."""
    P = _empty(wl)
    X1, _, _ = zone_centres(wl)
    P[0] = 1.0
    P[1] = 2.0
    P[3] = 0.1628 * alpha * np.sin(2.0 * np.pi * X1)
    P[5] = 0.1
    P[6] = 0.9867 * alpha * np.cos(2.0 * np.pi * X1)
    P[9] = dP
    return P


# ---------------------------------------------------------------- Kerr torus
#
# Initial data only: these Boyer-Lindquist / Kerr-Schild formulas build the
# starting state of the Kerr workloads and are not used by either solver.

def _bl(r, th, a):
    sth, cth = np.sin(th), np.cos(th)
    sig = r * r + a * a * cth * cth
    dlt = r * r - 2.0 * r + a * a
    big = (r * r + a * a) ** 2 - a * a * dlt * sth * sth
    return sig, dlt, big, sth


def _keplerian_ell(r, a):
    """ell = u^t u_phi of the prograde circular equatorial orbit at r (BL, M = 1)."""
    om = 1.0 / (r ** 1.5 + a)
    gtt = -(1.0 - 2.0 / r)
    gtp = -2.0 * a / r
    gpp = r * r + a * a + 2.0 * a * a / r
    ut = 1.0 / np.sqrt(-(gtt + 2.0 * om * gtp + om * om * gpp))
    uphi_cov = ut * (gtp + om * gpp)
    return ut * uphi_cov


def _fm_state(r, th, a, ell):
    """Circular flow with constant ell = u^t u_phi (Fishbone & Moncrief): the
    zero-angular-momentum observer sees speed v with y = Gamma v solving
    y^2 (1 + y^2) = (ell alpha/varpi)^2; ln h = ln u^t - ell Omega + const."""
    sig, dlt, big, sth = _bl(r, th, a)
    with np.errstate(invalid="ignore", divide="ignore"):  # inside the horizon: masked by the caller
        return _fm_state_bl(sig, dlt, big, sth, r, a, ell)


def _fm_state_bl(sig, dlt, big, sth, r, a, ell):
    alpha2 = sig * dlt / big
    varpi2 = big * sth * sth / sig
    s2 = ell * ell * alpha2 / np.maximum(varpi2, 1e-300)
    y2 = 0.5 * (-1.0 + np.sqrt(1.0 + 4.0 * s2))
    omega = 2.0 * a * r / big
    lnh = 0.5 * np.log(1.0 + y2) - 0.5 * np.log(alpha2) - ell * omega - y2
    ut = np.sqrt(1.0 + y2) / np.sqrt(alpha2)
    uphi = omega * ut + np.sqrt(y2) / np.sqrt(np.maximum(varpi2, 1e-300))
    return lnh, ut, uphi


def _mks_r_theta(wl, X1, X2):
    h = wl["hslope"]
    return np.exp(X1), np.pi * X2 + 0.5 * (1.0 - h) * np.sin(2.0 * np.pi * X2)


def kerr_torus(wl: dict, seed: int = 0):
    """Fishbone-Moncrief torus (inner edge r_in, pressure maximum r_max) in a
    rho = rho_fl r^-3/2, u = u_fl r^-5/2 atmosphere at rest with respect to the
    normal observer, u perturbed by noise * U(-1, 1) (seeded), and one poloidal
    field loop from A_phi = max(rho/rho_max - 0.2, 0) normalised so that
    max P_gas / max(b^2/2) = beta."""
    t = wl["torus"]
    a, gam = wl["spin"], wl["gamma"]
    rng = np.random.default_rng(seed)
    P = _empty(wl)
    X1, X2, X3 = zone_centres(wl)
    r, th = _mks_r_theta(wl, X1, X2)
    ell = _keplerian_ell(t["r_max"], a)
    lnh_in, _, _ = _fm_state(np.array(t["r_in"]), np.array(np.pi / 2), a, ell)

    def torus_rho(rr, tt):
        lnh, ut, uphi = _fm_state(rr, tt, a, ell)
        lnh = lnh - lnh_in
        inside = (lnh > 0.0) & (rr >= t["r_in"])
        hh = np.exp(np.where(inside, lnh, 0.0))
        rho = np.where(inside, ((hh - 1.0) * (gam - 1.0) / (t["kappa"] * gam)) ** (1.0 / (gam - 1.0)), 0.0)
        return rho, inside, ut, uphi

    rho, inside, ut, uphi = torus_rho(r, th)
    rho_max = rho.max()
    u = t["kappa"] * rho ** gam / (gam - 1.0) / rho_max
    rho = rho / rho_max
    u = u * (1.0 + t["noise"] * rng.uniform(-1.0, 1.0, u.shape))
    rfl, ufl = wl["rho_floor"] * r ** -1.5, wl["u_floor"] * r ** -2.5
    P[0] = np.where(inside, np.maximum(rho, rfl), rfl)
    P[1] = np.where(inside, np.maximum(u, ufl), ufl)
    # velocity: circular flow has u^r = u^theta = 0, so its Kerr-Schild and
    # BL components agree; MKS: u^X1 = u^X2 = 0, u^X3 = u^phi.  Normal-observer
    # form utilde^i = u^i + alpha^2 u^0 g^{0i}, with g^{01} = 2/Sigma (MKS),
    # g^{03} = 0 and alpha^2 = 1/(1 + 2r/Sigma).
    sig = r * r + a * a * np.cos(th) ** 2
    P[2] = np.where(inside, 2.0 * ut / (sig + 2.0 * r), 0.0)
    P[4] = np.where(inside, uphi, 0.0)

    # vector potential at cell corners, field by corner differences
    n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
    xs, xe = wl["x_start"], wl["x_end"]
    d1 = (xe[0] - xs[0]) / n[0]
    d2 = (xe[1] - xs[1]) / n[1]
    c1 = xs[0] + np.arange(n[0] + 1) * d1
    c2 = xs[1] + np.arange(n[1] + 1) * d2
    C2, C1 = np.meshgrid(c2, c1, indexing="ij")
    rc, thc = _mks_r_theta(wl, C1, C2)
    rho_c, _, _, _ = torus_rho(rc, thc)
    Aphi = np.maximum(rho_c / rho_max - 0.2, 0.0)  # [n2+1][n1+1]
    h = wl["hslope"]
    dth = np.pi * (1.0 + (1.0 - h) * np.cos(2.0 * np.pi * X2[0]))
    r0, th0 = r[0], th[0]
    sig0 = r0 * r0 + a * a * np.cos(th0) ** 2
    gdet = sig0 * np.abs(np.sin(th0)) * r0 * np.abs(dth)
    B1 = (Aphi[1:, :-1] + Aphi[1:, 1:] - Aphi[:-1, :-1] - Aphi[:-1, 1:]) / (2.0 * d2) / gdet
    B2 = -(Aphi[:-1, 1:] + Aphi[1:, 1:] - Aphi[:-1, :-1] - Aphi[1:, :-1]) / (2.0 * d1) / gdet
    # b^2 = (g_ij B^i B^j + (B^i u_i)^2) / (u^0)^2 with the MKS metric
    z = 2.0 * r0 / sig0
    s2 = np.sin(th0) ** 2
    g11 = (1.0 + z) * r0 * r0
    g22 = sig0 * dth * dth
    g10 = z * r0
    g13 = -a * s2 * (1.0 + z) * r0
    ut0 = np.where(inside[0], ut[0], 1.0 / np.sqrt(1.0 / (1.0 + z)))
    up0 = np.where(inside[0], uphi[0], 0.0)
    u1 = g10 * ut0 + g13 * up0
    bsq = (g11 * B1 ** 2 + g22 * B2 ** 2 + (B1 * u1) ** 2) / ut0 ** 2
    pg_max = ((gam - 1.0) * P[1]).max()
    norm = np.sqrt(pg_max / (t["beta"] * 0.5 * bsq.max())) if bsq.max() > 0 else 0.0
    P[5] = (B1 * norm)[None, :, :]
    P[6] = (B2 * norm)[None, :, :]
    return P


def initial_state(wl: dict, seed: int = 0):
    name = wl.get("ic", wl.get("name", ""))
    if name.startswith("srmhd1d_alfven"):
        return alfven_1d(wl, seed)
    if name.startswith("emhd2d_modes"):
        return fourier_modes_2d(wl, seed)
    if name.startswith("kerr_torus"):
        return kerr_torus(wl, seed)
    raise KeyError(f"no initial data for workload {name!r}")
