"""ctypes binding of libgrim (include/grim.h): same names, argument marshalling only.

Every step of the method runs in the HIP kernels of ``libgrim.so``; this
module only converts Python values, numpy arrays and PyTorch device tensors
into the C call's plain pointers and sizes.  There is no fallback: if the
library has not been built, :func:`load` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgrim.so")

GRIM_OK = 0
GRIM_IDEAL_MHD, GRIM_EMHD = 8, 10
GRIM_MINKOWSKI, GRIM_MKS_KERR = 0, 1
GRIM_BC = {"periodic": 0, "outflow": 1, "polar": 2}
GRIM_JAC = {"f64": 0, "f32": 1}
GRIM_GUESS = {"pn": 0, "mlp": 1}
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 32, 128, 16, 22880
FLAGS = {"NOT_CONVERGED": 1, "LS_EXHAUSTED": 2, "SINGULAR": 4, "UNPHYSICAL": 8, "NONFINITE": 16, "F64_RETRY": 32}


class grim_config_t(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n1", C.c_int), ("n2", C.c_int), ("n3", C.c_int), ("ng", C.c_int),
        ("model", C.c_int), ("metric", C.c_int),
        ("x_start", C.c_double * 3), ("x_end", C.c_double * 3),
        ("spin_a", C.c_double), ("mks_h", C.c_double),
        ("bc", C.c_int * 3),
        ("gamma", C.c_double), ("tau_R", C.c_double), ("chi", C.c_double), ("nu", C.c_double),
        ("plm_theta", C.c_double),
        ("tol", C.c_double), ("eps_fd", C.c_double), ("eps_bt", C.c_double),
        ("k_max", C.c_int), ("ls_max", C.c_int),
        ("jac_precision", C.c_int), ("guess", C.c_int),
        ("floors", C.c_int), ("rho_floor", C.c_double), ("u_floor", C.c_double),
        ("ls_safeguard", C.c_int), ("external_workspace", C.c_int), ("stage_block", C.c_int),
        ("full_system", C.c_int), ("riemann", C.c_int), ("recon", C.c_int), ("closure", C.c_int),
        ("phi", C.c_double), ("psi", C.c_double), ("dp_saturation", C.c_int), ("sat_width", C.c_double),
    ]


class grim_stats_t(C.Structure):
    _fields_ = [
        ("mean_iters", C.c_double * 2), ("max_iters", C.c_int32), ("pad", C.c_int32),
        ("n_fail", C.c_int64), ("n_ls_exhausted", C.c_int64), ("n_unphysical", C.c_int64),
        ("max_resid", C.c_double), ("zone_stages", C.c_int64), ("n_resid_calls", C.c_int64),
        ("n_fallback", C.c_int64), ("n_f64_retry", C.c_int64), ("n_backtracks", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {
            "mean_iters": [self.mean_iters[0], self.mean_iters[1]],
            "max_iters": int(self.max_iters),
            "n_fail": int(self.n_fail),
            "n_ls_exhausted": int(self.n_ls_exhausted),
            "n_unphysical": int(self.n_unphysical),
            "max_resid": float(self.max_resid),
            "zone_stages": int(self.zone_stages),
            "n_resid_calls": int(self.n_resid_calls),
            "n_fallback": int(self.n_fallback),
            "n_f64_retry": int(self.n_f64_retry),
            "n_backtracks": int(self.n_backtracks),
        }


class grim_train_cfg_t(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("n_used", C.c_int), ("pad", C.c_int),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("seed", C.c_uint64)]


_VP = C.c_void_p
_D = C.c_double
_lib = None


class GrimError(RuntimeError):
    pass


def load():
    """Load libgrim.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GrimError(f"{LIB_PATH} is not built: run `python -m paper_1702_01106_amd.build`")
    L = C.CDLL(LIB_PATH)
    L.grim_create.argtypes = [C.POINTER(grim_config_t), _VP, C.POINTER(_VP)]
    L.grim_destroy.argtypes = [_VP]
    L.grim_last_error.argtypes = [_VP]
    L.grim_last_error.restype = C.c_char_p
    L.grim_last_global_error.restype = C.c_char_p
    L.grim_device_bytes.argtypes = [_VP]
    L.grim_device_bytes.restype = C.c_size_t
    L.grim_workspace_bytes.argtypes = [C.POINTER(grim_config_t)]
    L.grim_workspace_bytes.restype = C.c_size_t
    L.grim_bind_workspace.argtypes = [_VP, _VP, C.c_size_t]
    L.grim_set_prims.argtypes = [_VP, _VP, C.c_int]
    L.grim_get_prims.argtypes = [_VP, _VP, C.c_int]
    L.grim_cfl_dt.argtypes = [_VP, _D, C.POINTER(_D)]
    L.grim_run.argtypes = [_VP, _D, C.c_int, C.c_int, C.POINTER(grim_stats_t)]
    L.grim_residual.argtypes = [_VP, _VP, _VP, _D, _VP, _VP, _VP]
    L.grim_stage_solve.argtypes = [_VP, _VP, _VP, _D, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(grim_stats_t)]
    L.grim_explicit.argtypes = [_VP, _VP, _VP, _VP, _VP]
    L.grim_get_zone_results.argtypes = [_VP, _VP, _VP, C.c_int]
    L.grim_stream_add.argtypes = [_VP, _VP, _VP, _VP, C.c_size_t]
    L.grim_math_probe.argtypes = [_VP, _VP, _VP, C.c_size_t]
    L.grim_profile.argtypes = [_VP, C.c_int]
    L.grim_kernel_times.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]
    L.grim_mlp_set_weights.argtypes = [_VP, _VP, C.c_size_t]
    L.grim_mlp_get_weights.argtypes = [_VP, _VP, C.c_size_t]
    L.grim_mlp_forward.argtypes = [_VP, _VP, C.c_int64, _VP]
    L.grim_mlp_backward.argtypes = [_VP, _VP, _VP, C.c_int64, _VP]
    L.grim_mlp_backward_noalloc.argtypes = [_VP, _VP, _VP, C.c_int64, _VP]
    L.grim_mlp_train.argtypes = [_VP, _VP, _VP, C.c_int64, C.POINTER(grim_train_cfg_t), _VP]
    L.grim_mlp_normalisation.argtypes = [_VP, _VP, _VP, C.c_int64, C.c_int, _VP, _VP, _VP]
    L.grim_collect_pairs.argtypes = [_VP, _D, C.c_int, C.c_int, _VP, _VP, C.c_int64, C.POINTER(C.c_int64)]
    _lib = L
    return L


def exported_symbols():
    return ["grim_create", "grim_destroy", "grim_last_error", "grim_last_global_error", "grim_device_bytes",
            "grim_workspace_bytes", "grim_bind_workspace", "grim_mlp_normalisation",
            "grim_set_prims", "grim_get_prims", "grim_cfl_dt", "grim_run", "grim_residual", "grim_stage_solve",
            "grim_explicit", "grim_get_zone_results", "grim_stream_add", "grim_math_probe", "grim_profile", "grim_kernel_times",
            "grim_mlp_set_weights", "grim_mlp_get_weights", "grim_mlp_forward", "grim_mlp_backward",
            "grim_mlp_backward_noalloc",
            "grim_mlp_train", "grim_collect_pairs"]


def _ptr(x):
    """Device pointer of a torch tensor, host pointer of a numpy array, or NULL."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


def _check(ctx, rc, what):
    if rc != GRIM_OK:
        msg = load().grim_last_error(ctx) if ctx else load().grim_last_global_error()
        raise GrimError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")


def config_from_workload(wl: dict) -> grim_config_t:
    c = grim_config_t()
    n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
    xs = list(wl["x_start"]) + [0.0] * (3 - len(wl["x_start"]))
    xe = list(wl["x_end"]) + [1.0] * (3 - len(wl["x_end"]))
    c.ndim = wl["ndim"]
    c.n1, c.n2, c.n3 = n
    c.ng = wl.get("ng", 2)
    c.model = wl["nvar"]
    c.metric = GRIM_MKS_KERR if wl.get("metric", "minkowski") == "mks" else GRIM_MINKOWSKI
    for d in range(3):
        c.x_start[d] = xs[d]
        c.x_end[d] = xe[d]
    c.spin_a = wl.get("spin", 0.0)
    c.mks_h = wl.get("hslope", 0.3)
    bc = (list(wl.get("bc", ["periodic"] * 3)) + ["periodic"] * 3)[:3]
    for d in range(3):
        c.bc[d] = GRIM_BC[bc[d]]
    c.gamma = wl["gamma"]
    c.tau_R = wl.get("tau_R", 1.0)
    c.chi = wl.get("chi", 0.0)
    c.nu = wl.get("nu", 0.0)
    c.plm_theta = wl.get("plm_theta", 1.0)
    c.tol = wl.get("tol", 1e-10)
    c.eps_fd = wl.get("eps_fd", 1.4901161193847656e-08)
    c.eps_bt = wl.get("eps_bt", 1e-4)
    c.k_max = wl.get("k_max", 20)
    c.ls_max = wl.get("ls_max", 10)
    c.jac_precision = GRIM_JAC[wl.get("jac", "f64")]
    c.guess = GRIM_GUESS[wl.get("guess", "pn")]
    c.floors = 1 if wl.get("floors", False) else 0
    c.rho_floor = wl.get("rho_floor", 1e-5)
    c.u_floor = wl.get("u_floor", 1e-7)
    c.ls_safeguard = int(wl.get("ls_safeguard", 0))
    c.external_workspace = 1 if wl.get("workspace", "library") == "caller" else 0
    c.stage_block = int(wl.get("stage_block", 0))
    c.full_system = 1 if wl.get("system", "reduced") == "full" else 0
    c.riemann = {"llf": 0, "hlle": 1}[wl.get("riemann", "llf")]
    c.recon = {"plm": 0, "weno5": 1, "ppm": 2}[wl.get("recon", "plm")]
    c.closure = 1 if wl.get("closure", False) else 0
    c.phi = wl.get("phi", 1.0)
    c.psi = wl.get("psi", 1.0)
    c.dp_saturation = 1 if wl.get("dp_saturation", False) else 0
    c.sat_width = wl.get("sat_width", 0.1)
    return c


# ---------------------------------------------------------------- C names

def grim_create(cfg: grim_config_t, stream_handle=None):
    ctx = _VP()
    rc = load().grim_create(C.byref(cfg), stream_handle, C.byref(ctx))
    _check(None, rc, "grim_create")
    return ctx


def grim_destroy(ctx):
    load().grim_destroy(ctx)


def grim_set_prims(ctx, P, on_device):
    _check(ctx, load().grim_set_prims(ctx, _ptr(P), int(on_device)), "grim_set_prims")


def grim_get_prims(ctx, P, on_device):
    _check(ctx, load().grim_get_prims(ctx, _ptr(P), int(on_device)), "grim_get_prims")


def grim_cfl_dt(ctx, cfl):
    dt = _D()
    _check(ctx, load().grim_cfl_dt(ctx, cfl, C.byref(dt)), "grim_cfl_dt")
    return dt.value


def grim_run(ctx, dt, nsteps, use_graph=True, want_stats=True):
    st = grim_stats_t()
    rc = load().grim_run(ctx, dt, int(nsteps), int(use_graph), C.byref(st) if want_stats else None)
    _check(ctx, rc, "grim_run")
    return st.as_dict() if want_stats else None


def grim_residual(ctx, Pn, PE, dtp, P, R, rnorm=None):
    _check(ctx, load().grim_residual(ctx, _ptr(Pn), _ptr(PE), dtp, _ptr(P), _ptr(R), _ptr(rnorm)), "grim_residual")


def grim_stage_solve(ctx, Pn, PE, dtp, guess, P_out, iters=None, resid=None, flags=None, backtracks=None,
                     want_stats=False):
    st = grim_stats_t()
    rc = load().grim_stage_solve(ctx, _ptr(Pn), _ptr(PE), dtp, _ptr(guess), _ptr(P_out), _ptr(iters),
                                 _ptr(resid), _ptr(flags), _ptr(backtracks), C.byref(st) if want_stats else None)
    _check(ctx, rc, "grim_stage_solve")
    return st.as_dict() if want_stats else None


def grim_explicit(ctx, PE, divF, srcE, emhd_sp=None):
    _check(ctx, load().grim_explicit(ctx, _ptr(PE), _ptr(divF), _ptr(srcE), _ptr(emhd_sp)), "grim_explicit")


def grim_get_zone_results(ctx, flags, iters, on_device):
    _check(ctx, load().grim_get_zone_results(ctx, _ptr(flags), _ptr(iters), int(on_device)), "grim_get_zone_results")


def grim_math_probe(ctx, x, out, n):
    _check(ctx, load().grim_math_probe(ctx, _ptr(x), _ptr(out), int(n)), "grim_math_probe")


def grim_stream_add(ctx, a, b, c, n):
    _check(ctx, load().grim_stream_add(ctx, _ptr(a), _ptr(b), _ptr(c), int(n)), "grim_stream_add")


KERNEL_GROUPS = ["ghost_fill", "face_flux", "flux_ct_emf", "stage_rhs", "newton", "mlp_infer"]


def grim_profile(ctx, enable):
    _check(ctx, load().grim_profile(ctx, int(enable)), "grim_profile")


def grim_kernel_times(ctx):
    k = len(KERNEL_GROUPS)
    ms = (C.c_double * k)()
    n = (C.c_int64 * k)()
    _check(ctx, load().grim_kernel_times(ctx, ms, n, k), "grim_kernel_times")
    return {KERNEL_GROUPS[i]: (float(ms[i]), int(n[i])) for i in range(k)}


def grim_mlp_set_weights(ctx, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    _check(ctx, load().grim_mlp_set_weights(ctx, w.ctypes.data, w.size), "grim_mlp_set_weights")


def grim_mlp_get_weights(ctx):
    w = np.empty(MLP_PARAMS, dtype=np.float32)
    _check(ctx, load().grim_mlp_get_weights(ctx, w.ctypes.data, w.size), "grim_mlp_get_weights")
    return w


def grim_mlp_forward(ctx, X, n, Y):
    _check(ctx, load().grim_mlp_forward(ctx, _ptr(X), int(n), _ptr(Y)), "grim_mlp_forward")


def grim_mlp_backward(ctx, X, dY, n, dW):
    _check(ctx, load().grim_mlp_backward(ctx, _ptr(X), _ptr(dY), int(n), _ptr(dW)), "grim_mlp_backward")


def grim_mlp_backward_noalloc(ctx, X, dY, n, dW):
    """Asynchronous (enqueued on the context's stream); n <= 2048 rows."""
    _check(ctx, load().grim_mlp_backward_noalloc(ctx, _ptr(X), _ptr(dY), int(n), _ptr(dW)),
           "grim_mlp_backward_noalloc")


def grim_mlp_train(ctx, X, T, n, epochs, batch, n_used, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
    cfg = grim_train_cfg_t(epochs=epochs, batch=batch, n_used=n_used, pad=0, lr=lr, beta1=beta1, beta2=beta2,
                           eps=eps, seed=seed)
    hist = np.zeros(max(epochs, 1))
    _check(ctx, load().grim_mlp_train(ctx, _ptr(X), _ptr(T), int(n), C.byref(cfg), hist.ctypes.data),
           "grim_mlp_train")
    return hist[:epochs]


def grim_collect_pairs(ctx, dt, nsteps, stride, X, T, cap):
    cnt = C.c_int64()
    _check(ctx, load().grim_collect_pairs(ctx, dt, int(nsteps), int(stride), _ptr(X), _ptr(T), int(cap),
                                          C.byref(cnt)), "grim_collect_pairs")
    return int(cnt.value)


def grim_device_bytes(ctx):
    return int(load().grim_device_bytes(ctx))


def grim_workspace_bytes(cfg: grim_config_t):
    n = int(load().grim_workspace_bytes(C.byref(cfg)))
    if n == 0:
        _check(None, -1, "grim_workspace_bytes")
    return n


def grim_bind_workspace(ctx, buf, nbytes):
    _check(ctx, load().grim_bind_workspace(ctx, _ptr(buf), int(nbytes)), "grim_bind_workspace")


def grim_mlp_normalisation(ctx, X, T, n, n_used):
    xm, xs, ys = np.zeros(MLP_IN), np.zeros(MLP_IN), np.zeros(MLP_OUT)
    _check(ctx, load().grim_mlp_normalisation(ctx, _ptr(X), _ptr(T), int(n), int(n_used), xm.ctypes.data,
                                              xs.ctypes.data, ys.ctypes.data), "grim_mlp_normalisation")
    return xm, xs, ys


# ---------------------------------------------------------------- convenience

class Context:
    """One libgrim context for a workload dict; tensors are torch (cuda) float64.
    With wl["workspace"] == "caller" the device memory is a torch uint8 tensor
    (self.workspace) handed to the library with grim_bind_workspace."""

    def __init__(self, wl: dict, stream=None):
        import torch

        self.torch = torch
        self.wl = dict(wl)
        self.cfg = config_from_workload(self.wl)
        n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
        self.nvar = wl["nvar"]
        self.shape = (self.nvar, n[2], n[1], n[0])
        self.nz = n[0] * n[1] * n[2]
        self.stream = stream
        handle = None if stream is None else _VP(stream.cuda_stream)
        self.ctx = grim_create(self.cfg, handle)
        self.workspace = None
        if self.cfg.external_workspace:
            nbytes = grim_workspace_bytes(self.cfg)
            # torch's caching allocator hands out blocks on 512-byte boundaries
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            grim_bind_workspace(self.ctx, self.workspace, nbytes)

    def close(self):
        if self.ctx:
            grim_destroy(self.ctx)
            self.ctx = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x, dtype=None):
        t = self.torch
        if isinstance(x, np.ndarray):
            x = t.from_numpy(np.ascontiguousarray(x))
        x = x.to(device="cuda", dtype=dtype or t.float64).contiguous()
        return x

    def empty(self, shape=None, dtype=None):
        return self.torch.empty(shape or self.shape, dtype=dtype or self.torch.float64, device="cuda")

    def set_prims(self, P):
        if isinstance(P, np.ndarray):
            a = np.ascontiguousarray(P, dtype=np.float64)
            assert a.size == self.nvar * self.nz
            grim_set_prims(self.ctx, a, False)
        else:
            d = self._dev(P)
            assert d.numel() == self.nvar * self.nz
            grim_set_prims(self.ctx, d, True)

    def get_prims(self):
        out = np.empty(self.shape)
        grim_get_prims(self.ctx, out, False)
        return out

    def get_prims_device(self, out=None):
        out = self.empty() if out is None else out
        grim_get_prims(self.ctx, out, True)
        return out

    def cfl_dt(self, cfl):
        return grim_cfl_dt(self.ctx, cfl)

    def run(self, dt, nsteps, use_graph=True, want_stats=True):
        return grim_run(self.ctx, dt, nsteps, use_graph, want_stats)

    def residual(self, Pn, PE, dtp, P):
        Pn, PE, P = self._dev(Pn), self._dev(PE), self._dev(P)
        R = self.empty()
        rn = self.empty((self.nz,))
        grim_residual(self.ctx, Pn, PE, dtp, P, R, rn)
        return R, rn

    def stage_solve(self, Pn, PE, dtp, guess=None, extra=False):
        """(P, iters, resid, flags) of one stage; with extra=True also the
        per-zone rejected line-search trials and the stage's statistics."""
        t = self.torch
        Pn, PE = self._dev(Pn), self._dev(PE)
        g = None if guess is None else self._dev(guess)
        out = self.empty()
        it = t.empty((self.nz,), dtype=t.int32, device="cuda")
        rr = self.empty((self.nz,))
        fl = t.empty((self.nz,), dtype=t.uint8, device="cuda")
        bt = t.empty((self.nz,), dtype=t.int32, device="cuda") if extra else None
        st = grim_stage_solve(self.ctx, Pn, PE, dtp, g, out, it, rr, fl, bt, want_stats=extra)
        if extra:
            return out, it, rr, fl, bt, st
        return out, it, rr, fl

    def explicit(self, PE):
        PE = self._dev(PE)
        divF = self.empty()
        src = self.empty()
        sp = self.empty((self.nz, 3))
        grim_explicit(self.ctx, PE, divF, src, sp)
        return divF, src, sp

    def zone_results(self):
        fl = np.empty(self.nz, dtype=np.uint8)
        it = np.empty(self.nz, dtype=np.int32)
        grim_get_zone_results(self.ctx, fl, it, False)
        return fl, it

    def profile(self, enable):
        grim_profile(self.ctx, enable)

    def kernel_times(self):
        return grim_kernel_times(self.ctx)

    def device_bytes(self):
        return grim_device_bytes(self.ctx)
