"""CPU checks of the oracle comparison behind the benchmark's error report
and the full-size Kerr GPU tests.

One oracle step of a 32^3 box from the full grid's P_n on the box and a
2 Ng halo (stage 1 on the box grown by Ng, stage 2 on the box) must equal the
oracle's full-grid step on the box.  The box's zone centres come from its own
x_start = x_start + i0 dX, which differs from the full grid's by rounding, so
Newton may stop at a slightly different point below the tolerance.  Those
differences must lie inside the allowance of the comparison: 1e-6 of
max(|P_v|, family RMS), or twice the tolerance-implied bound
||row v of J^-1|| (||R_a|| + ||R_b||) where that is larger (for q and DP, whose
family scale is tiny early in the run: there 1e-6 of it is below what a
residual norm of 1e-10 determines).  A planted difference above the bound
must be caught."""
import numpy as np
import pytest

import bench
from paper_1702_01106_amd import workloads as W


@pytest.mark.parametrize("name", ["grmhd3d_kerr_128", "emhd3d_kerr_192"])
def test_box_step_matches_full_step(oracle_mod, name):
    wl = W.small(name, [96, 96, 40])
    P0 = W.kerr_torus(wl, seed=0)
    o = oracle_mod.Oracle(wl)
    dt = o.cfl_dt(P0, 0.5)
    P1, _ = o.step(P0, dt, 1)
    box = bench.kerr_box(wl)
    full = bench.cut(P1, box, halo=False)
    ref, info, rep = bench.oracle_step_checked(oracle_mod, wl, bench.cut(P0, box, halo=True), dt, 0, box=box,
                                               Pgpu=full)
    assert info["fail_stage1"] == 0 and info["fail_stage2"] == 0
    assert rep["within"], rep
    assert rep["max_oracle_resid_at_gpu"] < 2 * wl["tol"]
    # away from q and DP the two agree far inside 1e-6
    assert max(rep["rel"][k] for k in ("rho", "u", "u1", "u2", "u3")) < 1e-7, rep["rel"]
    # a planted error of 10x the allowance in one zone's u^1 is caught
    bad = full.copy()
    z = (5, 7, 9)
    bad[2][z] += 1e-5 * max(abs(full[2][z]), np.sqrt(np.mean(full[2:5] ** 2)))
    _, _, rep2 = bench.oracle_step_checked(oracle_mod, wl, bench.cut(P0, box, halo=True), dt, 0, box=box, Pgpu=bad)
    assert not rep2["within"] and rep2["worst_over_allowed"]["u1"] > 5
    # the box wraps in X3 (periodic): k0 = 0 takes its lower halo from the top planes
    h, i0, j0 = bench.BOX_HALO, box[0], box[1]
    top = P0[:, -h, j0 - h:j0 + bench.BOX_N + h, i0 - h:i0 + bench.BOX_N + h]
    assert box[2] == 0 and np.array_equal(bench.cut(P0, box, halo=True)[:, 0], top)


def test_full_grid_check_2d(oracle_mod):
    """The same comparison on a whole periodic 2-D grid (the 2-D variants of
    the benchmark): an oracle step against itself is within, a planted
    1e-5 error in one zone's q is not."""
    wl = W.small("emhd2d_modes_256", [48, 40])
    P0 = W.fourier_modes_2d(wl, seed=2, amp=1e-2)
    o = oracle_mod.Oracle(wl)
    dt = o.cfl_dt(P0, 0.5)
    P1, _ = o.step(P0, dt, 1)
    _, _, rep = bench.oracle_step_checked(oracle_mod, wl, P0, dt, 0, Pgpu=P1)
    assert rep["within"] and max(rep["rel"].values()) < 1e-12, rep
    bad = P1.copy()
    bad[8, 0, 3, 4] += 1e-5 * np.sqrt(np.mean(P1[8:10] ** 2))
    _, _, rep2 = bench.oracle_step_checked(oracle_mod, wl, P0, dt, 0, Pgpu=bad)
    assert not rep2["within"]
