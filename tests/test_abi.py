"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import workloads
from paper_2109_12565_amd import _lib as tlb

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "tlb.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tlb_[a-z_]+)\s*\(", text)))


def test_header_declares_exactly_the_binding_exports():
    assert header_functions() == sorted(tlb.EXPORTS)


def test_library_loads_and_exports_every_declared_symbol():
    lib = tlb.load_library()
    for name in header_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_header(tmp_path):
    """Offsets of every field as the C compiler lays out the header's structs
    equal those of the ctypes mirrors."""
    lines = []
    for cname, cls in (("tlb_params", tlb.Params), ("tlb_obs", tlb.Obs), ("tlb_droplet", tlb.Droplet),
                        ("tlb_launch", tlb.Launch)):
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "tlb.h"\nint main(void){'
                   + "".join(lines) + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    want = {}
    for line in out:
        if line:
            cname, fname, val = line.split()
            want[(cname, fname)] = int(val)
    for cname, cls in (("tlb_params", tlb.Params), ("tlb_obs", tlb.Obs), ("tlb_droplet", tlb.Droplet),
                        ("tlb_launch", tlb.Launch)):
        assert want[(cname, "sizeof")] == ctypes.sizeof(cls)
        for fname, _ in cls._fields_:
            assert want[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def _params(**kw):
    p = tlb.Params()
    p.lx, p.ly, p.precision = kw.get("lx", 16), kw.get("ly", 8), kw.get("precision", 1)
    p.tau, p.tau_g = kw.get("tau", 1.0), kw.get("tau_g", 1.0)
    p.rho0, p.g12 = kw.get("rho0", 0.83), 0.405
    p.g_a[0], p.g_a[1] = -9.0, -8.0
    p.g_r[0], p.g_r[1] = 8.1, 7.1
    p.alpha_g, p.t_top = 0.0, 0.0
    p.rho_wall[0], p.rho_wall[1] = 0.612, 0.612
    p.dt_nominal = kw.get("dt_nominal", 1.0)
    for k in ("launch_flags", "fused", "fused_rows", "fused_strip", "rows", "fused_lanes"):
        setattr(p, k, kw.get(k, 0))
    return p


def _init(p, solid=None, null_field=False):
    lib = tlb.load_library()
    # arrays are only read after validation, so rejected sizes get small ones
    n = max(p.lx, 1) * max(p.ly, 1)
    f = np.ones(n if n <= 1 << 16 else 1)
    tb = np.ones(max(p.lx, 1))
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p(123)
    rc = lib.tlb_init(ctypes.byref(h), ctypes.byref(p), None if null_field else dp(f), dp(f), dp(f),
                      None, None,
                      None if solid is None else solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                      dp(tb), None)
    return rc, h, lib.tlb_last_error(None).decode()


@pytest.mark.parametrize("kw,msg", [
    (dict(lx=0), "lattice size"),
    (dict(ly=-3), "lattice size"),
    (dict(lx=1 << 16, ly=1 << 15), "lattice size"),
    (dict(precision=7), "precision"),
    (dict(tau=0.5), "tau"),
    (dict(tau_g=0.2), "tau"),
    (dict(rho0=0.0), "rho0"),
    (dict(dt_nominal=0.0), "dt_nominal"),
    (dict(launch_flags=4), "launch options"),
    (dict(fused=3), "launch options"),
    (dict(fused=-1), "launch options"),
    (dict(fused_rows=-2), "launch options"),
    (dict(fused_rows=5000), "launch options"),
    (dict(fused_strip=246), "launch options"),
    (dict(rows=4097), "launch options"),
    (dict(fused_lanes=64), "launch options"),
    (dict(fused_lanes=512), "launch options"),
])
def test_init_rejects_bad_params_without_device(kw, msg):
    rc, h, err = _init(_params(**kw))
    assert rc == tlb.TLB_EINVAL
    assert h.value is None
    assert msg in err


def test_init_rejects_null_arrays_and_bad_solid_flags():
    rc, h, err = _init(_params(), null_field=True)
    assert rc == tlb.TLB_EINVAL and "NULL" in err
    bad = np.zeros(16 * 8, np.uint8)
    bad[5] = 3
    rc, h, err = _init(_params(), solid=bad)
    assert rc == tlb.TLB_EINVAL and "solid flag" in err


def test_null_handle_calls():
    lib = tlb.load_library()
    assert lib.tlb_destroy(None) == tlb.TLB_OK
    assert lib.tlb_time(None) == -1
    assert lib.tlb_step(None, 1) == tlb.TLB_EINVAL
    assert lib.tlb_observables(None, None) == tlb.TLB_EINVAL
    assert lib.tlb_get_fields(None, None, None, None, None, None) == tlb.TLB_EINVAL
    assert lib.tlb_get_stress(None, None, None) == tlb.TLB_EINVAL
    assert lib.tlb_row_averages(None, None, None) == tlb.TLB_EINVAL
    assert lib.tlb_droplets(None, 0.8, None, 0, None, None) == tlb.TLB_EINVAL
    assert lib.tlb_forward_taped(None, 1, 1, None) == tlb.TLB_EINVAL
    assert lib.tlb_adjoint_step(None, 1, 1.0, None) == tlb.TLB_EINVAL
    assert lib.tlb_launch_info(None, None) == tlb.TLB_EINVAL


def test_binding_fails_loudly_without_library(tmp_path):
    saved = tlb._lib
    try:
        tlb._lib = None
        with pytest.raises(FileNotFoundError):
            tlb.load_library(str(tmp_path / "missing.so"))
    finally:
        tlb._lib = saved


def test_binding_validates_shapes_before_calling():
    w = workloads.small()
    with pytest.raises(ValueError):
        tlb.Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], launch={"fused_row": 4})
    with pytest.raises(KeyError):
        tlb.Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], launch={"fused": "yes"})
    with pytest.raises(ValueError):
        tlb.Simulation(w["params"], w["rho_a"], w["rho_b"][:, :5], w["temp"])
    with pytest.raises(ValueError):
        tlb.Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], precision="fp8")


def test_init_external_rejects_a_missing_workspace_without_device():
    lib = tlb.load_library()
    p = _params()
    f = np.ones(p.lx * p.ly)
    tb = np.ones(p.lx)
    dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p(123)
    for ws, nbytes in ((None, 1 << 20), (ctypes.c_void_p(4096), 0)):
        rc = lib.tlb_init_external(ctypes.byref(h), ctypes.byref(p), dp(f), dp(f), dp(f), None, None,
                                   None, dp(tb), None, ws, nbytes)
        assert rc == tlb.TLB_EINVAL
        assert h.value is None
        assert "workspace" in lib.tlb_last_error(None).decode()
    bad = _params(tau=0.4)
    assert lib.tlb_workspace_bytes(ctypes.byref(bad), None) == tlb.TLB_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits
    with status 2 before touching a device."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = r.stdout.strip().splitlines()[-1]
    assert "one GPU only" in line and '"n_gpus": 2' in line
