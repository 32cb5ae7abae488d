"""CPU-side checks of the C ABI: the library loads, exports every function
include/grim.h declares, and rejects invalid configurations before touching
a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_1702_01106_amd import grim
from paper_1702_01106_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            src = open(os.path.join(ROOT, "include", f)).read()
            names |= set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(grim_\w+)\s*\(", src, re.M))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(grim.LIB_PATH):
        pytest.skip("libgrim.so not built")
    return grim.load()


def test_exports_every_declared_symbol(lib):
    decl = _declared()
    assert len(decl) >= 14
    for name in decl:
        assert hasattr(lib, name), name
    assert decl == set(grim.exported_symbols())


def test_struct_layouts_match_header(lib, tmp_path):
    """ctypes mirrors of grim_config_t / grim_stats_t have the header's field
    offsets (checked with a C program compiled against include/grim.h)."""
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "grim.h"', "int main(void){"]
    for cname, py in (("grim_config_t", grim.grim_config_t), ("grim_stats_t", grim.grim_stats_t)):
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.split("\n") if l)
    for cname, py in (("grim_config_t", grim.grim_config_t), ("grim_stats_t", grim.grim_stats_t)):
        assert int(out[cname]) == C.sizeof(py)
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("mutate,msg", [
    (dict(ndim=4), "ndim"),
    (dict(ng=1), "ng"),
    (dict(nvar=9), "model"),
    (dict(gamma=1.0), "gamma"),
    (dict(chi=0.0), "EMHD"),
    (dict(ls_max=0), "ls_max"),
    (dict(n=[256, 0]), "no zones"),
    (dict(recon="weno5"), "ng = 3"),
    (dict(recon="ppm", ng=2), "ng = 3"),
    (dict(dp_saturation=True), "closure"),
    (dict(closure=True, phi=0.0), "phi, psi"),
    (dict(closure=True, dp_saturation=True, sat_width=0.0), "sat_width"),
    (dict(system="full", riemann="hlle"), "full system"),
    (dict(ng=3, n=[256, 2]), "n >= ng"),
])
def test_invalid_config_rejected_before_device(lib, mutate, msg):
    wl = W.workload("emhd2d_modes_256")
    wl.update(mutate)
    cfg = grim.config_from_workload(wl)
    with pytest.raises(grim.GrimError) as e:
        grim.grim_create(cfg, None)
    assert msg in str(e.value)


def test_oracle_not_imported_by_product():
    """The product path never imports the oracle."""
    for f in ("grim.py", "workloads.py", "build.py", "__init__.py"):
        src = open(os.path.join(ROOT, "paper_1702_01106_amd", f)).read()
        assert "oracle" not in src.replace("oracle's", "")


def test_flag_constants_match_header():
    import re

    from paper_1702_01106_amd import grim

    hdr = open(os.path.join(ROOT, "include", "grim.h")).read()
    found = dict(re.findall(r"#define GRIM_FLAG_(\w+) (\d+)", hdr))
    assert {k: int(v) for k, v in found.items()} == grim.FLAGS


@pytest.mark.parametrize("mutate,msg", [
    (dict(k_max=101), "k_max"),
    (dict(ls_max=65), "ls_max"),
    (dict(ls_safeguard=2), "ls_safeguard"),
])
def test_solver_limits_rejected(lib, mutate, msg):
    wl = W.workload("emhd2d_modes_256")
    wl.update(mutate)
    cfg = grim.config_from_workload(wl)
    cfg.ls_safeguard = mutate.get("ls_safeguard", cfg.ls_safeguard)
    with pytest.raises(grim.GrimError) as e:
        grim.grim_create(cfg, None)
    assert msg in str(e.value)
    assert lib.grim_workspace_bytes(C.byref(cfg)) == 0


def test_workspace_bytes(lib):
    """grim_workspace_bytes (host only, no device): at least the ghosted state
    arrays (P_n/P_{n+1}, the half step, two hook copies, one face array per
    direction), the interior rhs/staging/coefficient arrays, per-zone results
    and the network's per-zone features; at most that plus 256 bytes of
    alignment per buffer and the fixed-size parts; geometry only for Kerr;
    0 for an invalid config."""
    def need(wl):
        nv = wl["nvar"]
        n = list(wl["n"]) + [1] * (3 - len(wl["n"]))
        N = [n[d] + (4 if d < wl["ndim"] else 0) for d in range(3)]
        cells, nz = N[0] * N[1] * N[2], n[0] * n[1] * n[2]
        b = 8 * nv * cells * (5 + wl["ndim"]) + 8 * nz * (2 * nv + (13 if nv == 10 else 0))
        b += nz * (4 + 8 + 1) + 4 * nz * (grim.MLP_IN + grim.MLP_OUT)
        if wl.get("metric") == "mks":
            b += 8 * N[0] * N[1] * (4 * 16 + 64)
        return b

    fixed = 256 * 128 + 32 + 8 * 258 * 48 + 4 * grim.MLP_PARAMS + 2 * (32 * 128 + 128 * 128 + 32 * 128)
    for wl in (W.workload("emhd2d_modes_256"), W.small("grmhd3d_kerr_128", [20, 16, 8]),
               W.workload("srmhd1d_alfven_128")):
        got = lib.grim_workspace_bytes(C.byref(grim.config_from_workload(wl)))
        lo = need(wl)
        assert lo <= got <= lo + fixed + 256 * 40, (wl["name"], got, lo)
        assert got % 256 == 0
    bad = grim.config_from_workload(dict(W.workload("emhd2d_modes_256"), ndim=4))
    assert lib.grim_workspace_bytes(C.byref(bad)) == 0
    assert b"ndim" in lib.grim_last_global_error()
