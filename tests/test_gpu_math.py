"""The reciprocal, inverse square root and square root of the hot loops
(hardware estimates refined by two Newton-Raphson steps) against correctly
rounded references computed in extended precision on the host.  The parity
tests check the whole path against the oracle; this pins the arithmetic
itself over 2^-1000..2^1000: within one unit in the last place for 1/x,
two for 1/sqrt(x), and three for sqrt(x) = x * (1/sqrt(x)) (the refined
estimate's ulp plus the product's rounding, which near a power of two can
be two ulps of the result); and the special values the kernels rely on."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def probe():
    import torch

    from paper_1702_01106_amd import grim
    from paper_1702_01106_amd import workloads as W

    ctx = grim.Context(W.small("emhd2d_modes_256", [8, 8]))

    def run(x):
        xd = torch.tensor(np.asarray(x, dtype=np.float64), device="cuda")
        out = torch.empty(3 * xd.numel(), dtype=torch.float64, device="cuda")
        grim.grim_math_probe(ctx.ctx, xd, out, xd.numel())
        o = out.cpu().numpy().reshape(-1, 3)
        return o[:, 0], o[:, 1], o[:, 2]

    return run


def _ulps(got, ref):
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def test_newton_raphson_accuracy(probe):
    rng = np.random.default_rng(5)
    n = 200_000
    x = np.ldexp(rng.uniform(1.0, 2.0, n), rng.integers(-1000, 1000, n))
    x = np.concatenate([x, [1.0, 2.0, 3.0, 0.1, 1.0 - 2.0**-53, 1.0 + 2.0**-52]])
    rcp, rsq, sq = probe(x)
    xl = x.astype(np.longdouble)
    ref_rcp = (1 / xl).astype(np.float64)
    ref_rsq = (1 / np.sqrt(xl)).astype(np.float64)
    ref_sq = np.sqrt(x)
    e = (_ulps(rcp, ref_rcp).max(), _ulps(rsq, ref_rsq).max(), _ulps(sq, ref_sq).max())
    print("max ulp error: rcp %.2f  rsqrt %.2f  sqrt %.2f" % e)
    assert e[0] <= 1.0 and e[1] <= 2.0 and e[2] <= 3.0, e


def test_special_values(probe):
    inf, nan = np.inf, np.nan
    rcp, rsq, sq = probe([0.0, inf, nan, -1.0, -4.0, 4.0])
    assert rcp[0] == inf and rcp[1] == 0.0 and np.isnan(rcp[2]) and rcp[3] == -1.0 and rcp[4] == -0.25
    assert rsq[0] == inf and rsq[1] == 0.0 and np.isnan(rsq[2]) and np.isnan(rsq[3])
    assert sq[0] == 0.0 and sq[5] == 2.0
    # sqrt of a negative argument is NaN (the residual then fails the
    # line search's finiteness test, as with IEEE sqrt); of +inf non-finite
    assert np.isnan(sq[3]) and np.isnan(sq[4]) and np.isnan(sq[2]) and not np.isfinite(sq[1])
