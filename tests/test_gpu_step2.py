"""The fused two-step kernel (tau = tau_g = 1; FP64, FP32 and the FP16 / BF16
deviation storages; posts; flat walls at rest or moving) against runs made of
single steps and against the oracle.

The fused kernel keeps the intermediate time level as moments per node
(density, velocity and u^2 of each field) and rebuilds its populations with the same expressions the single step
stores them with; the compiler contracts multiply-adds into fused ones
differently in the two kernels, so the results agree to rounding, not bit
for bit: after 18 steps the bar against single steps is 1e-13 relative in
FP64; in FP32 it is 2e-6 for populations, densities and temperature (a few
units in the last place) and 2e-5 of max|u| for velocities, which are small
differences of populations. Against the oracle the bars are those of the single-step parity
tests: FP64 <= 1e-12 relative, FP32 <= 1e-5 for densities, temperature and
populations (3e-5 of max|u| for velocities).

The launch option fused = "always" forces the fused kernel wherever it
applies (it is otherwise chosen only for lattices where it pays), "never"
disables it, and fused_rows sets its chunk height, so short chunks exercise
chunk edges in both marching directions. fused_lanes sets the block width:
on these small lattices the library picks 128 lanes, so 256 is forced as
the second case.
"""
import numpy as np
import pytest

import workloads
from oracle.oracle import ModelParams, Oracle
from paper_2109_12565_amd import Simulation

from test_gpu_parity import FIELDS, field_errors, pop_errors, posts_case

pytestmark = pytest.mark.gpu


def make(case, precision, fused, rows=None, strip=None, lanes=None, **extra):
    launch = {"fused": "always" if fused else "never", "fused_rows": rows or 0,
              "fused_strip": strip or 0, "fused_lanes": lanes or 0}
    p = dict(case["params"], **extra)
    sim = Simulation(p, case["rho_a"], case["rho_b"], case["temp"], solid=case.get("solid"),
                     t_bottom=case.get("t_bottom"), precision=precision, launch=launch)
    info = sim.launch_info()
    print("launch", info)
    return sim, info


def droplet_case(lx, ly, seed=11):
    """Random droplets (rho_A-rich discs of radius 6) at any lattice size."""
    rng = np.random.default_rng(seed)
    n = max(1, lx * ly // 600)
    centres = [(rng.uniform(0, lx), rng.uniform(6, max(7, ly - 6))) for _ in range(n)]
    inside = workloads.paint_discs(lx, ly, centres, 6.0)
    return dict(params=dict(workloads.BASE_PARAMS, alpha_g=1e-3),
                rho_a=np.where(inside, 1.36, 0.08) + rng.uniform(-0.01, 0.01, (ly, lx)),
                rho_b=np.where(inside, 0.08, 1.36) + rng.uniform(-0.01, 0.01, (ly, lx)),
                temp=workloads.conduction_profile(lx, ly) + rng.uniform(-1e-3, 1e-3, (ly, lx)),
                t_bottom=workloads.bottom_temperature_noise(lx, seed=seed))


def assert_close_state(a, b, tol, tol_u):
    perr = pop_errors(a.populations(), b.populations())
    ferr = field_errors(a.fields(), b.fields())
    print("fused vs single", perr, ferr)
    assert max(perr.values()) <= tol, perr
    assert max(ferr[k] for k in FIELDS) <= tol, ferr
    assert max(ferr["ux"], ferr["uy"]) <= tol_u, ferr
    oa, ob = a.observables(), b.observables()
    for k in ("mass_a", "mass_b", "sum_t", "nu", "nu_top", "ke"):
        assert oa[k] == pytest.approx(ob[k], rel=tol, abs=1e-14), (k, oa[k], ob[k])


CASES = {
    "small": workloads.small,
    "posts": posts_case,
    "ragged_two_strips": lambda: droplet_case(300, 70),
    "narrow": lambda: droplet_case(37, 20),
    "three_strips_short": lambda: droplet_case(700, 16),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("rows", [None, 1, 7])
@pytest.mark.parametrize("lanes", [None, 256])
def test_fused_matches_single_steps(precision, name, rows, lanes):
    case = CASES[name]()
    fused, info = make(case, precision, True, rows, lanes=lanes)
    assert info["fused_rows"] > 0
    assert info["fused_lanes"] == (lanes or 128)
    assert info["fused_strip"] <= info["fused_lanes"] - 10
    single, info0 = make(case, precision, False)
    assert info0["fused_rows"] == 0
    for n in (9, 1, 2, 6):   # odd and even calls; every call ends with a single step
        fused.step(n)
        single.step(n)
    assert fused.t == single.t == 18
    if precision == "fp64":
        assert_close_state(fused, single, 1e-13, 1e-13)
    else:
        assert_close_state(fused, single, 2e-6, 2e-5)


def test_fused_kernel_is_not_used_where_it_does_not_apply():
    w = workloads.small()
    _, info = make(w, "fix16dev", True)
    assert info["fused_rows"] == 0
    for precision in ("fp32", "fp16dev"):
        _, info = make(w, precision, True, tau=0.8)
        assert info["fused_rows"] == 0, precision


W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
HALF_ULP_BITS = {"fp16dev": (10, -14), "bf16dev": (7, -126)}


@pytest.mark.parametrize("precision", sorted(HALF_ULP_BITS))
@pytest.mark.parametrize("name,u_wall", [(n, (0.0, 0.0)) for n in sorted(CASES)] +
                         [("small", (-0.01, 0.02)), ("posts", (-0.01, 0.02))])
@pytest.mark.parametrize("rows", [None, 7])
@pytest.mark.parametrize("lanes", [None, 256])
def test_dev16_fused_launch_from_gpu_state(precision, name, u_wall, rows, lanes):
    """16-bit deviation storage, fused kernel forced on: from the GPU's own
    state after 4 steps (decoded exactly), tlb_step(3) runs one fused launch
    and one single step; the oracle takes 3 FP64 steps from the same state.
    The densities and temperature of t + 3 are moments of populations that
    were rounded to 16 bits once, at the end of the fused launch (its
    intermediate level stays in FP32): each node's zeroth moment at t + 3
    sums 8 rounded moving values pulled from its neighbours and loses the 8
    roundings of its own (through the exact rest remainder), so the error
    is at most 16 half ulps of the largest moving deviation, plus FP32
    arithmetic. Walls at rest, and moving Couette walls on two lattices."""
    case = CASES[name]()
    case["params"] = dict(case["params"], u_wall=u_wall)
    sim, info = make(case, precision, True, rows, lanes=lanes)
    assert info["fused_rows"] > 0 and info["fused_lanes"] == (lanes or 128)
    check_dev16_launch(sim, case, precision, f"{name} rows {rows}")


def check_dev16_launch(sim, case, precision, label, warm=4):
    """`warm` steps, then tlb_step(3) against 3 oracle steps from the decoded
    state, with the bound of 16 half ulps of the largest moving deviation
    (plus FP32 arithmetic) on each density and the temperature."""
    sim.step(warm)
    state = sim.populations()
    sim.step(3)
    ora = Oracle(ModelParams(**case["params"]), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    ora.load_post_collision(state, warm + 1).step(2)   # streams f*(warm): time warm + 1
    got, ref = sim.fields(), ora.fields()
    pr = sim.params
    solid = case.get("solid")
    fluid = np.ones(state.shape[1:], bool) if solid is None else solid == 0
    mant, emin = HALF_ULP_BITS[precision]
    post = ora.post_collision()
    for k0, key, refv in ((0, "rho_a", pr.rho_ref[0]), (9, "rho_b", pr.rho_ref[1]),
                          (18, "temp", pr.t_ref)):
        # largest moving deviation before and after the launch
        refs = (W9[1:] * refv)[:, None, None]
        big = max(np.abs(p[k0 + 1:k0 + 9] - refs)[:, fluid].max() for p in (state, post))
        hu = 0.5 * 2.0 ** (np.floor(np.log2(max(big, 2.0 ** emin))) - mant)
        err = np.abs(got[key] - ref[key])[fluid].max()
        bound = 16 * hu + 1e-5 * np.abs(ref[key]).max()
        print(precision, label, key, "err", err, "bound", bound, flush=True)
        assert err <= bound, (key, err, bound)


@pytest.mark.parametrize("precision", sorted(HALF_ULP_BITS))
def test_full_size_dev16_fused_launch_from_gpu_state(precision):
    """The 16-bit storages on 4096 x 2048 with posts in the launch
    configuration the library picks there (256-lane blocks, as the benchmark
    times them): one fused launch and a single step from the GPU's state
    after 20 steps, against the oracle, to the bound above."""
    w = workloads.large()
    sim, info = make(w, precision, True)
    assert info["fused_rows"] > 0 and info["fused_lanes"] == 256
    check_dev16_launch(sim, w, precision, "large", warm=20)
    sim.close()


def test_fp64_fused_matches_oracle():
    case = posts_case()
    sim, info = make(case, "fp64", True, rows=5)
    assert info["fused_rows"] > 0
    ora = Oracle(ModelParams(**case["params"]), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case["solid"], t_bottom=case["t_bottom"])
    sim.step(151)
    ora.step(151)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr


def test_fp32_fused_1000_steps_matches_oracle():
    case = workloads.small()
    sim, info = make(case, "fp32", True)
    assert info["fused_rows"] > 0
    ora = Oracle(ModelParams(**case["params"]), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    sim.step(1000)
    ora.step(1000)
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 fused 1000 steps", errs)
    assert max(errs[k] for k in FIELDS) <= 1e-5, errs
    assert max(errs["ux"], errs["uy"]) <= 3e-5, errs


@pytest.mark.parametrize("precision,lanes,tol", [("fp32", 256, 1e-5), ("fp64", 128, 1e-12)])
def test_full_size_fused_steps_from_gpu_state(precision, lanes, tol):
    """4096 x 2048 with posts in the launch configuration the library picks
    by default (FP32: the benchmark's 256-lane blocks; FP64: 128-lane
    blocks): from the GPU's state after 20 steps, the GPU advances 3 steps
    (one fused launch and a single step) and the oracle 3 steps from the same
    state; every field and population is compared."""
    w = workloads.large()
    p = w["params"]
    sim = Simulation(p, w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision=precision)
    info = sim.launch_info()
    print("launch", info)
    assert info["fused_rows"] > 0 and info["fused_lanes"] == lanes
    sim.step(20)
    state = sim.populations()
    sim.step(3)
    ora = Oracle(ModelParams(**p), w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                 t_bottom=w["t_bottom"])
    ora.load_post_collision(state, 21)   # streams f*(20): the state of time 21
    del state
    ora.step(2)
    errs = field_errors(sim.fields(), ora.fields())
    print("large fused fields", precision, errs)
    assert max(errs.values()) <= tol, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    print("large fused populations", precision, perr)
    assert max(perr.values()) <= tol, perr
    sim.close()


@pytest.mark.parametrize("lx,ly", [(5, 3), (64, 1), (7, 2), (250, 9), (120, 5)])
@pytest.mark.parametrize("lanes", [None, 256])
def test_fused_edge_shapes_fp64(lx, ly, lanes):
    """Lattices narrower than the kernel's halo (columns wrap several times
    across one block), a single row (both walls on it), and strips just
    above one block's stored width (246 columns of 256 lanes, 118 of 128).
    Velocities get 1e-11 of max|u|: on these lattices max|u| is small
    (about 1e-4 on the single row), while u carries the absolute rounding of
    its populations."""
    case = droplet_case(lx, ly, seed=lx + ly)
    fused, info = make(case, "fp64", True, lanes=lanes)
    assert info["fused_rows"] > 0 and info["fused_lanes"] == (lanes or 128)
    single, _ = make(case, "fp64", False)
    for n in (7, 4):
        fused.step(n)
        single.step(n)
    assert_close_state(fused, single, 1e-13, 1e-11)


def test_fused_launch_geometry():
    """At 4096 x 2048 the fused grid fits one block per resident slot, its
    strips cover the lattice with at most 246 stored columns each, and its
    chunks are at least 24 rows tall; the fused_rows and fused_strip launch
    options override the choice."""
    w = workloads.large()
    lx, ly = w["lx"], w["ly"]
    sim, info = make(w, "fp32", True)
    sim.close()
    assert info["fused_lanes"] == 256
    assert 24 <= info["fused_rows"] <= ly and info["fused_strip"] <= 246
    assert info["fused_grid_x"] * info["fused_strip"] >= lx
    assert (info["fused_grid_x"] - 1) * info["fused_strip"] < lx
    assert info["fused_grid_y"] * info["fused_rows"] >= ly
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert info["fused_grid_x"] * info["fused_grid_y"] <= 2 * cus
    sim, info2 = make(w, "fp32", True, rows=40, strip=200)
    sim.close()
    assert info2["fused_rows"] == 40 and info2["fused_strip"] <= 200


def test_fp64_runs_the_fused_kernel_in_narrow_blocks():
    """FP64: a 256-lane block needs most of a CU's LDS, so the library takes
    128-lane blocks (two per CU) at 4096 x 2048 too."""
    w = workloads.large()
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision="fp64")
    info = sim.launch_info()
    sim.close()
    assert info["fused_rows"] > 0 and info["fused_lanes"] == 128 and info["fused_strip"] <= 118
    assert info["fused_grid_x"] * info["fused_strip"] >= w["lx"]
    assert info["fused_grid_y"] * info["fused_rows"] >= w["ly"]


def test_fused_launch_geometry_narrow_blocks():
    """At 1024 x 512 blocks of 256 lanes would leave chunks of 6 rows: the
    library takes 128-lane blocks (strips of at most 118 stored columns),
    still one block per resident slot; fused_lanes = 256 overrides it."""
    w = workloads.mid()
    lx, ly = w["lx"], w["ly"]
    sim, info = make(w, "fp32", True)
    sim.close()
    assert info["fused_lanes"] == 128 and info["fused_strip"] <= 118
    assert info["fused_grid_x"] * info["fused_strip"] >= lx
    assert (info["fused_grid_x"] - 1) * info["fused_strip"] < lx
    assert info["fused_grid_y"] * info["fused_rows"] >= ly
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert info["fused_grid_x"] * info["fused_grid_y"] <= 4 * cus
    sim, info2 = make(w, "fp32", True, lanes=256)
    sim.close()
    assert info2["fused_lanes"] == 256 and info2["fused_rows"] == 6


U_WALL = (-0.01, 0.02)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["small", "posts"])
@pytest.mark.parametrize("lanes", [None, 256])
def test_fused_moving_walls_match_single_steps(precision, name, lanes):
    """Couette walls (Sec. 2.2): the second level adds the wall momentum to
    the bounced diagonal links with the node's own intermediate zeroth
    moment as rho_w, which equals the sum of its stored populations in the
    single step up to rounding."""
    case = CASES[name]()
    fused, info = make(case, precision, True, rows=7, lanes=lanes, u_wall=U_WALL)
    assert info["fused_rows"] > 0 and info["fused_lanes"] == (lanes or 128)
    single, _ = make(case, precision, False, u_wall=U_WALL)
    for n in (9, 1, 2, 6):
        fused.step(n)
        single.step(n)
    if precision == "fp64":
        assert_close_state(fused, single, 1e-13, 1e-13)
    else:
        assert_close_state(fused, single, 2e-6, 2e-5)


def test_fp64_fused_moving_walls_match_oracle():
    case = posts_case()
    sim, info = make(case, "fp64", True, rows=5, u_wall=U_WALL)
    assert info["fused_rows"] > 0
    ora = Oracle(ModelParams(**dict(case["params"], u_wall=U_WALL)), case["rho_a"], case["rho_b"],
                 case["temp"], solid=case["solid"], t_bottom=case["t_bottom"])
    sim.step(151)
    ora.step(151)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr


def test_fp32_fused_moving_walls_500_steps():
    """The single path's Couette bar (FP32 after 500 steps under shear:
    1e-5 for densities and temperature, 3e-5 of max|u| for velocities)."""
    case = workloads.small()
    sim, info = make(case, "fp32", True, u_wall=U_WALL)
    assert info["fused_rows"] > 0
    ora = Oracle(ModelParams(**dict(case["params"], u_wall=U_WALL)), case["rho_a"], case["rho_b"],
                 case["temp"], solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    sim.step(500)
    ora.step(500)
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 fused moving walls 500 steps", errs)
    assert max(errs[k] for k in FIELDS) <= 1e-5, errs
    assert max(errs["ux"], errs["uy"]) <= 3e-5, errs
