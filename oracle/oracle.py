"""ctypes wrapper of the C oracle (``grim_oracle.c``).

TEST INFRASTRUCTURE.  Loaded only by the tests, the smoke check and the CPU
baseline of the benchmark.  Arrays are numpy float64 in the interior-only
structure-of-arrays layout [nvar][n3][n2][n1].
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "grim_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAGS = {"NOT_CONVERGED": 1, "LS_EXHAUSTED": 2, "SINGULAR": 4, "UNPHYSICAL": 8, "NONFINITE": 16}


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp",
           "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class OCfg(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int), ("ng", C.c_int),
        ("nvar", C.c_int), ("metric", C.c_int),
        ("bc1", C.c_int), ("bc2", C.c_int), ("bc3", C.c_int),
        ("x1s", C.c_double), ("x2s", C.c_double), ("x3s", C.c_double),
        ("dx1", C.c_double), ("dx2", C.c_double), ("dx3", C.c_double),
        ("spin", C.c_double), ("hslope", C.c_double),
        ("gam", C.c_double), ("tau_R", C.c_double), ("chi", C.c_double), ("nu", C.c_double),
        ("theta_plm", C.c_double),
        ("tol", C.c_double), ("eps", C.c_double), ("eps_bt", C.c_double),
        ("k_max", C.c_int), ("ls_max", C.c_int), ("ls_safeguard", C.c_int),
        ("floors", C.c_int), ("rho_fl", C.c_double), ("u_fl", C.c_double),
        ("nthreads", C.c_int),
        ("full_system", C.c_int), ("riemann", C.c_int), ("recon", C.c_int), ("closure", C.c_int),
        ("phi", C.c_double), ("psi", C.c_double), ("dp_saturation", C.c_int), ("sat_width", C.c_double),
    ]


class OStats(C.Structure):
    _fields_ = [
        ("iters_sum", C.c_double * 2), ("zones", C.c_int64), ("max_iters", C.c_int32),
        ("n_fail", C.c_int64), ("n_ls_exhausted", C.c_int64), ("n_unphysical", C.c_int64),
        ("max_resid", C.c_double), ("n_backtracks", C.c_int64),
    ]

    def as_dict(self, nsteps: int) -> dict:
        z = max(int(self.zones), 1) * max(nsteps, 1)
        return {
            "mean_iters": [self.iters_sum[0] / z, self.iters_sum[1] / z],
            "max_iters": int(self.max_iters),
            "n_fail": int(self.n_fail),
            "n_ls_exhausted": int(self.n_ls_exhausted),
            "n_unphysical": int(self.n_unphysical),
            "max_resid": float(self.max_resid),
            "n_backtracks": int(self.n_backtracks),
        }


_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)
RESID_FN = C.CFUNCTYPE(None, C.c_void_p, _D, _D)


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def cfg_from_dict(d: dict) -> OCfg:
    """Build the oracle's config struct from a plain workload dictionary."""
    c = OCfg()
    n = list(d["n"]) + [1] * (3 - len(d["n"]))
    xs = list(d["x_start"]) + [0.0] * (3 - len(d["x_start"]))
    xe = list(d["x_end"]) + [1.0] * (3 - len(d["x_end"]))
    c.ndim = d["ndim"]
    c.n1, c.n2, c.n3 = n
    c.ng = d.get("ng", 2)
    c.nvar = d["nvar"]
    c.metric = 1 if d.get("metric", "minkowski") == "mks" else 0
    bc = d.get("bc", ["periodic"] * 3)
    code = {"periodic": 0, "outflow": 1, "polar": 2}
    c.bc1, c.bc2, c.bc3 = [code[b] for b in (list(bc) + ["periodic"] * 3)[:3]]
    c.x1s, c.x2s, c.x3s = xs
    c.dx1, c.dx2, c.dx3 = [(xe[i] - xs[i]) / n[i] for i in range(3)]
    c.spin = d.get("spin", 0.0)
    c.hslope = d.get("hslope", 0.3)
    c.gam = d["gamma"]
    c.tau_R = d.get("tau_R", 1.0)
    c.chi = d.get("chi", 0.0)
    c.nu = d.get("nu", 0.0)
    c.theta_plm = d.get("plm_theta", 1.0)
    c.tol = d.get("tol", 1e-10)
    c.eps = d.get("eps_fd", 1.4901161193847656e-08)
    c.eps_bt = d.get("eps_bt", 1e-4)
    c.k_max = d.get("k_max", 20)
    c.ls_max = d.get("ls_max", 10)
    c.ls_safeguard = int(d.get("ls_safeguard", 0))
    c.floors = 1 if d.get("floors", False) else 0
    c.rho_fl = d.get("rho_floor", 1e-5)
    c.u_fl = d.get("u_floor", 1e-7)
    c.nthreads = d.get("nthreads", 0)
    c.full_system = 1 if d.get("system", "reduced") == "full" else 0
    c.riemann = {"llf": 0, "hlle": 1}[d.get("riemann", "llf")]
    c.recon = {"plm": 0, "weno5": 1, "ppm": 2}[d.get("recon", "plm")]
    c.closure = 1 if d.get("closure", False) else 0
    c.phi = d.get("phi", 1.0)
    c.psi = d.get("psi", 1.0)
    c.dp_saturation = 1 if d.get("dp_saturation", False) else 0
    c.sat_width = d.get("sat_width", 0.1)
    if c.recon != 0 and c.ng < 3:
        raise ValueError("WENO5 and PPM read three cells on each side of a face: ng >= 3")
    if c.dp_saturation and not c.closure:
        raise ValueError("DeltaP saturation scales the diffusivities through the closure: closure must be on")
    return c


class Oracle:
    """Numpy-facing calls into the C oracle for one workload configuration."""

    _lib = None

    @classmethod
    def lib(cls):
        if cls._lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            L = C.CDLL(_LIB)
            P = C.POINTER(OCfg)
            L.oracle_stage.argtypes = [P, _D, _D, C.c_double, _D, _D, _I32, _D, _U8]
            L.oracle_reconstruct.argtypes = [P, _D, _D, _D]
            L.oracle_stage_ghosted.argtypes = [P, _D, _D, C.c_double, _D, _D, _I32, _D, _U8, _I32]
            L.oracle_step.argtypes = [P, _D, C.c_double, C.POINTER(OStats)]
            L.oracle_run.argtypes = [P, _D, C.c_double, C.c_int, C.POINTER(OStats)]
            L.oracle_residual.argtypes = [P, _D, _D, C.c_double, _D, _D, _D]
            L.oracle_residual_ghosted.argtypes = [P, _D, _D, C.c_double, _D, _D, _D]
            L.oracle_system_jacobians_ghosted.argtypes = [P, _D, _D, C.c_double, _D, _D, _D]
            L.oracle_explicit.argtypes = [P, _D, _D, _D, _D]
            L.oracle_cfl_dt.argtypes = [P, _D, C.c_double]
            L.oracle_cfl_dt.restype = C.c_double
            L.oracle_geometry.argtypes = [P, _D, _D, _D, _D, _D]
            L.oracle_connection.argtypes = [P, _D, _D]
            L.oracle_prim_to_flux.argtypes = [P, _D, _D, C.c_int, _D]
            L.oracle_speeds.argtypes = [P, _D, _D, C.c_int, _D, _D]
            L.oracle_vmax2.argtypes = [P, _D, _D]
            L.oracle_vmax2.restype = C.c_double
            L.oracle_solve.argtypes = [C.c_int, _D, _D, _D]
            L.oracle_ls_lambda.argtypes = [C.c_double, C.c_double, C.c_double]
            L.oracle_ls_lambda.restype = C.c_double
            L.oracle_newton_generic.argtypes = [C.c_int, RESID_FN, C.c_void_p, _D, C.c_double, C.c_double,
                                                C.c_double, C.c_double, C.c_int, C.c_int, C.c_int, _I32, _D, _U8,
                                                _I32]
            L.oracle_divb.argtypes = [P, _D, _D]
            L.oracle_fill_ghosts.argtypes = [P, _D, _D]
            L.oracle_fd_jacobian.argtypes = [C.c_int, RESID_FN, C.c_void_p, _D, _D, C.c_double, _D]
            L.oracle_zone_jacobian.argtypes = [P, _D, _D, C.c_double, _D, C.c_long, _D, _D]
            L.oracle_sum_U.argtypes = [P, _D, _D]
            cls._lib = L
        return cls._lib

    def __init__(self, wl: dict):
        self.wl = dict(wl)
        self.cfg = cfg_from_dict(self.wl)
        self.nvar = self.cfg.nvar
        n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
        self.shape = (self.nvar, n[2], n[1], n[0])
        self.nz = n[0] * n[1] * n[2]
        self.L = self.lib()

    def _arr(self, P):
        a = np.ascontiguousarray(P, dtype=np.float64)
        assert a.size == self.nvar * self.nz, (a.shape, self.shape)
        return a

    def stage(self, Pn, PE, dtp, guess=None):
        Pn, PE = self._arr(Pn), self._arr(PE)
        g = None if guess is None else self._arr(guess)
        out = np.empty(self.shape)
        it = np.empty(self.nz, dtype=np.int32)
        rr = np.empty(self.nz)
        fl = np.empty(self.nz, dtype=np.uint8)
        rc = self.L.oracle_stage(C.byref(self.cfg), _dp(Pn), _dp(PE), dtp, _dp(g), _dp(out),
                                 it.ctypes.data_as(_I32), _dp(rr), fl.ctypes.data_as(_U8))
        assert rc == 0
        return out, it, rr, fl

    def stage_ghosted(self, Pn, PEg, dtp, guess=None):
        """One stage with P^E given on the ghosted grid [nvar][N3][N2][N1]
        (ghosts used as given).  Returns (P, iters, resid, flags, backtracks)."""
        Pn = self._arr(Pn)
        PEg = np.ascontiguousarray(PEg, dtype=np.float64)
        g = self.cfg.ng
        nd = self.cfg.ndim
        N = [self.shape[3] + 2 * g, self.shape[2] + (2 * g if nd >= 2 else 0),
             self.shape[1] + (2 * g if nd >= 3 else 0)]
        assert PEg.size == self.nvar * N[0] * N[1] * N[2], (PEg.shape, N)
        gu = None if guess is None else self._arr(guess)
        out = np.empty(self.shape)
        it = np.empty(self.nz, dtype=np.int32)
        rr = np.empty(self.nz)
        fl = np.empty(self.nz, dtype=np.uint8)
        bt = np.empty(self.nz, dtype=np.int32)
        rc = self.L.oracle_stage_ghosted(C.byref(self.cfg), _dp(Pn), _dp(PEg), dtp, _dp(gu), _dp(out),
                                         it.ctypes.data_as(_I32), _dp(rr), fl.ctypes.data_as(_U8),
                                         bt.ctypes.data_as(_I32))
        assert rc == 0
        return out, it, rr, fl, bt

    def step(self, P, dt, nsteps=1):
        P = self._arr(P).copy()
        st = OStats()
        rc = self.L.oracle_run(C.byref(self.cfg), _dp(P), dt, nsteps, C.byref(st))
        assert rc == 0
        return P, st.as_dict(nsteps)

    def residual(self, Pn, PE, dtp, P):
        Pn, PE, P = self._arr(Pn), self._arr(PE), self._arr(P)
        R = np.empty(self.shape)
        rn = np.empty(self.nz)
        self.L.oracle_residual(C.byref(self.cfg), _dp(Pn), _dp(PE), dtp, _dp(P), _dp(R), _dp(rn))
        return R, rn

    def residual_ghosted(self, Pn, PEg, dtp, P):
        """As residual, with P^E given on the ghosted grid (ghosts as given)."""
        Pn, P = self._arr(Pn), self._arr(P)
        PEg = np.ascontiguousarray(PEg, dtype=np.float64)
        assert PEg.shape == self.ghosted_shape(), (PEg.shape, self.ghosted_shape())
        R = np.empty(self.shape)
        rn = np.empty(self.nz)
        rc = self.L.oracle_residual_ghosted(C.byref(self.cfg), _dp(Pn), _dp(PEg), dtp, _dp(P), _dp(R), _dp(rn))
        assert rc == 0
        return R, rn

    def system_jacobians_ghosted(self, Pn, PEg, dtp, P):
        """Per zone, the FD Jacobian of the Newton system at P ([nz][m][m])
        and U_rho(P_n) ([nz]), for a stage with ghost-filled P^E."""
        Pn, P = self._arr(Pn), self._arr(P)
        PEg = np.ascontiguousarray(PEg, dtype=np.float64)
        assert PEg.shape == self.ghosted_shape(), (PEg.shape, self.ghosted_shape())
        m = self.nvar - 3
        J = np.empty((self.nz, m, m))
        ur = np.empty(self.nz)
        rc = self.L.oracle_system_jacobians_ghosted(C.byref(self.cfg), _dp(Pn), _dp(PEg), dtp, _dp(P), _dp(J),
                                                    _dp(ur))
        assert rc == 0
        return J, ur

    def explicit(self, PE):
        PE = self._arr(PE)
        divF = np.empty(self.shape)
        src = np.empty(self.shape)
        sp = np.empty((self.nz, 3))
        self.L.oracle_explicit(C.byref(self.cfg), _dp(PE), _dp(divF), _dp(src), _dp(sp))
        return divF, src, sp

    def zone_jacobian(self, Pn, PE, dtp, P, z):
        Pn, PE, P = self._arr(Pn), self._arr(PE), self._arr(P)
        J = np.empty((self.nvar, self.nvar))
        R = np.empty(self.nvar)
        rc = self.L.oracle_zone_jacobian(C.byref(self.cfg), _dp(Pn), _dp(PE), dtp, _dp(P), z, _dp(J), _dp(R))
        assert rc == 0
        return J, R

    def reconstruct(self, s6):
        """(left, right) states at the face between cells i-1 and i from the
        values of cells i-3..i+2."""
        a = np.ascontiguousarray(s6, dtype=np.float64)
        lo, hi = C.c_double(), C.c_double()
        self.L.oracle_reconstruct(C.byref(self.cfg), _dp(a), C.byref(lo), C.byref(hi))
        return lo.value, hi.value

    def cfl_dt(self, P, cfl):
        return float(self.L.oracle_cfl_dt(C.byref(self.cfg), _dp(self._arr(P)), cfl))

    def ghosted_shape(self):
        g, nd = self.cfg.ng, self.cfg.ndim
        return (self.nvar, self.shape[1] + (2 * g if nd >= 3 else 0), self.shape[2] + (2 * g if nd >= 2 else 0),
                self.shape[3] + 2 * g)

    def fill_ghosts(self, P):
        """Interior P -> ghosted array with the boundary conditions applied."""
        out = np.empty(self.ghosted_shape())
        self.L.oracle_fill_ghosts(C.byref(self.cfg), _dp(self._arr(P)), _dp(out))
        return out

    def divb(self, P):
        out = np.empty(self.nz)
        self.L.oracle_divb(C.byref(self.cfg), _dp(self._arr(P)), _dp(out))
        return out.reshape(self.shape[1:])

    def sum_U(self, P):
        out = np.empty(self.nvar)
        self.L.oracle_sum_U(C.byref(self.cfg), _dp(self._arr(P)), _dp(out))
        return out

    # ---- point functions -------------------------------------------------
    def geometry(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        gcov = np.empty(16)
        gcon = np.empty(16)
        gdet = C.c_double()
        alpha = C.c_double()
        self.L.oracle_geometry(C.byref(self.cfg), _dp(X), _dp(gcov), _dp(gcon), C.byref(gdet), C.byref(alpha))
        return gcov.reshape(4, 4), gcon.reshape(4, 4), gdet.value, alpha.value

    def connection(self, X):
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = np.empty(64)
        self.L.oracle_connection(C.byref(self.cfg), _dp(X), _dp(out))
        return out.reshape(4, 4, 4)

    def flux(self, P, X, d):
        P = np.ascontiguousarray(P, dtype=np.float64)
        X = np.ascontiguousarray(X, dtype=np.float64)
        out = np.empty(self.nvar)
        self.L.oracle_prim_to_flux(C.byref(self.cfg), _dp(P), _dp(X), d, _dp(out))
        return out

    def speeds(self, P, X, d):
        P = np.ascontiguousarray(P, dtype=np.float64)
        X = np.ascontiguousarray(X, dtype=np.float64)
        lp, lm = C.c_double(), C.c_double()
        self.L.oracle_speeds(C.byref(self.cfg), _dp(P), _dp(X), d, C.byref(lp), C.byref(lm))
        return lp.value, lm.value

    def vmax2(self, P, X):
        P = np.ascontiguousarray(P, dtype=np.float64)
        X = np.ascontiguousarray(X, dtype=np.float64)
        return float(self.L.oracle_vmax2(C.byref(self.cfg), _dp(P), _dp(X)))

    # ---- generic numerics ------------------------------------------------
    @classmethod
    def solve(cls, A, b):
        A = np.ascontiguousarray(A, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty(b.size)
        rc = cls.lib().oracle_solve(b.size, _dp(A), _dp(b), _dp(x))
        return x, rc

    @classmethod
    def ls_lambda(cls, f0, f1, lam):
        return float(cls.lib().oracle_ls_lambda(f0, f1, lam))

    @classmethod
    def fd_jacobian(cls, fn, x, eps=1.4901161193847656e-08):
        n = len(x)
        x = np.ascontiguousarray(x, dtype=np.float64)

        def cb(ctx, xp, rp):
            r = np.asarray(fn(np.ctypeslib.as_array(xp, shape=(n,)).copy()), dtype=np.float64)
            for i in range(n):
                rp[i] = r[i]

        cfn = RESID_FN(cb)
        R = np.ascontiguousarray(fn(x.copy()), dtype=np.float64)
        J = np.empty((n, n))
        cls.lib().oracle_fd_jacobian(n, cfn, None, _dp(x), _dp(R), eps, _dp(J))
        return J

    @classmethod
    def newton(cls, fn, x0, tol=1e-10, eps=1.4901161193847656e-08, eps_bt=1e-4, k_max=20, ls_max=10,
               nscale=1.0, ls_safeguard=0, with_backtracks=False):
        """Newton driver on a Python residual fn(x: ndarray) -> ndarray.
        Returns (x, iters, resid, flags[, backtracks])."""
        n = len(x0)
        x = np.ascontiguousarray(x0, dtype=np.float64).copy()

        def cb(ctx, xp, rp):
            xv = np.ctypeslib.as_array(xp, shape=(n,)).copy()
            r = np.asarray(fn(xv), dtype=np.float64)
            for i in range(n):
                rp[i] = r[i]

        cfn = RESID_FN(cb)
        it = C.c_int32()
        rr = C.c_double()
        fl = C.c_uint8()
        bt = C.c_int32()
        cls.lib().oracle_newton_generic(n, cfn, None, _dp(x), nscale, tol, eps, eps_bt, k_max, ls_max,
                                        int(ls_safeguard), C.byref(it), C.byref(rr), C.byref(fl), C.byref(bt))
        if with_backtracks:
            return x, it.value, rr.value, fl.value, bt.value
        return x, it.value, rr.value, fl.value
