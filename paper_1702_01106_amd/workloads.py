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


def initial_state(wl: dict, seed: int = 0):
    name = wl.get("ic", wl.get("name", ""))
    if name.startswith("srmhd1d_alfven"):
        return alfven_1d(wl, seed)
    if name.startswith("emhd2d_modes"):
        return fourier_modes_2d(wl, seed)
    raise KeyError(f"no initial data for workload {name!r}")
