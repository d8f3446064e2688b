"""GPU (HIP, gfx950) versus the FP64 oracle, element by element.

Tolerances: FP64 storage <= 1e-12 relative after 200 steps; FP32 storage
<= 1e-5 relative after 1000 steps for densities, temperature and populations
(small-case geometry). The relative error of a field is max|gpu - oracle| /
max|oracle|; velocities are normalised by the largest oracle velocity
component, and for FP32 they get 3e-5: u is a difference of populations of
size ~0.1-0.6 stored with 24-bit mantissas, so its absolute error sits near
1e-7 at every step (measured flat from step 100 to 2000), while max|u| decays
to ~7e-3 as the droplets settle.

At full benchmark sizes the oracle cannot run many steps, so there the GPU's
own post-collision state is handed to the oracle, both advance one step, and
every element is compared; properties that hold at any size (per-component
mass, bitwise x-translation equivariance) cover the long runs.
"""
import math

import numpy as np
import pytest

import workloads
from oracle.oracle import ModelParams, Oracle
from paper_2109_12565_amd import Simulation

pytestmark = pytest.mark.gpu

FIELDS = ("rho_a", "rho_b", "temp")


def rel(a, b):
    d = np.abs(a - b).max()
    s = np.abs(b).max()
    return d / s if s > 0 else d


def field_errors(got, ref):
    errs = {k: rel(got[k], ref[k]) for k in FIELDS}
    umax = max(np.abs(ref["ux"]).max(), np.abs(ref["uy"]).max(), 1e-300)
    for k in ("ux", "uy"):
        errs[k] = np.abs(got[k] - ref[k]).max() / umax
    return errs


def pop_errors(got, ref):
    return {"f_a": rel(got[0:9], ref[0:9]), "f_b": rel(got[9:18], ref[9:18]),
            "g": rel(got[18:27], ref[18:27])}


def run_pair(case, steps, precision, **kw):
    p = dict(case["params"])
    sim = Simulation(p, case["rho_a"], case["rho_b"], case["temp"], solid=case.get("solid"),
                     t_bottom=case.get("t_bottom"), precision=precision, **kw)
    ora = Oracle(ModelParams(**p), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    sim.step(steps)
    ora.step(steps)
    return sim, ora


def posts_case(lx=96, ly=48, seed=7):
    rng = np.random.default_rng(seed)
    solid = workloads.bottom_posts(np.random.Generator(np.random.PCG64(seed)), lx, ly)
    solid[-3:, 10:18] = 2
    inside = workloads.paint_discs(lx, ly, [(30.5, 24.0), (70.0, 28.5)], 9.0)
    return dict(
        params=dict(workloads.BASE_PARAMS, alpha_g=1e-3),
        rho_a=np.where(inside, 1.36, 0.08) + rng.uniform(-0.01, 0.01, (ly, lx)),
        rho_b=np.where(inside, 0.08, 1.36) + rng.uniform(-0.01, 0.01, (ly, lx)),
        temp=workloads.conduction_profile(lx, ly) + rng.uniform(-1e-3, 1e-3, (ly, lx)),
        solid=solid, t_bottom=workloads.bottom_temperature_noise(lx, seed=5))


# ------------------------------------------------------------ FP64 parity


def test_fp64_small_200_steps_fields_populations_observables():
    w = workloads.small()
    sim, ora = run_pair(w, 200, "fp64")
    errs = field_errors(sim.fields(), ora.fields())
    print("fp64 small fields", errs)
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    print("fp64 small populations", perr)
    assert max(perr.values()) <= 1e-12, perr
    og, oo = sim.observables(), ora.observables()
    assert og["step"] == 200
    for k in ("mass_a", "mass_b", "sum_t", "ke", "nu", "nu_top"):
        assert og[k] == pytest.approx(oo[k], rel=1e-11, abs=1e-14), (k, og[k], oo[k])


def test_fp64_posts_ragged_lattice_and_varying_wall_temperature():
    """96 x 48 (row pitch padded to 128: a ragged last strip), bottom posts,
    a rough patch flagged at the top temperature, per-column T_b."""
    c = posts_case()
    sim, ora = run_pair(c, 150, "fp64")
    errs = field_errors(sim.fields(), ora.fields())
    print("fp64 posts fields", errs)
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr
    og, oo = sim.observables(), ora.observables()
    for k in ("mass_a", "mass_b", "sum_t", "ke", "nu", "nu_top"):
        assert og[k] == pytest.approx(oo[k], rel=1e-11, abs=1e-14), (k, og[k], oo[k])


def test_fp64_time_zero_and_initial_velocity():
    """t = 0 (the init variant) and a start with a velocity field."""
    w = workloads.small()
    rng = np.random.default_rng(2)
    ux = rng.uniform(-0.02, 0.02, w["rho_a"].shape)
    uy = rng.uniform(-0.02, 0.02, w["rho_a"].shape)
    p = w["params"]
    sim = Simulation(p, w["rho_a"], w["rho_b"], w["temp"], ux0=ux, uy0=uy, precision="fp64")
    ora = Oracle(ModelParams(**p), w["rho_a"], w["rho_b"], w["temp"], ux0=ux, uy0=uy)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-13, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-13, perr
    sim.step(37)
    ora.step(37)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs


@pytest.mark.parametrize("lx,ly", [(5, 3), (64, 1), (100, 45), (130, 70)])
def test_fp64_edge_shapes(lx, ly):
    """Tiny lattices (x wrap inside one strip, a single row between the
    walls), and shapes that leave ragged strips and row chunks."""
    rng = np.random.default_rng(lx * 1000 + ly)
    case = dict(params=dict(workloads.BASE_PARAMS, alpha_g=2e-3),
                rho_a=rng.uniform(0.1, 1.3, (ly, lx)), rho_b=rng.uniform(0.1, 1.3, (ly, lx)),
                temp=rng.uniform(0, 1, (ly, lx)), t_bottom=rng.uniform(0.9, 1.1, lx))
    sim, ora = run_pair(case, 25, "fp64")
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr


def test_zero_steps_is_identity():
    w = workloads.small()
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], precision="fp64")
    before = sim.populations()
    sim.step(0)
    assert sim.t == 0
    assert np.array_equal(before, sim.populations())


# ------------------------------------------------------------ FP32 parity


def test_fp32_small_1000_steps():
    w = workloads.small()
    sim, ora = run_pair(w, 1000, "fp32")
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 small 1000 fields", errs)
    assert max(errs[k] for k in FIELDS) <= 1e-5, errs
    assert max(errs["ux"], errs["uy"]) <= 3e-5, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    print("fp32 small 1000 populations", perr)
    assert max(perr.values()) <= 1e-5, perr
    og, oo = sim.observables(), ora.observables()
    for k in ("mass_a", "mass_b", "sum_t"):
        assert og[k] == pytest.approx(oo[k], rel=1e-5), (k, og[k], oo[k])


def test_fp32_posts_300_steps():
    c = posts_case(lx=128, ly=64, seed=11)
    sim, ora = run_pair(c, 300, "fp32")
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 posts fields", errs)
    assert max(errs[k] for k in FIELDS) <= 1e-5, errs
    assert max(errs["ux"], errs["uy"]) <= 3e-5, errs


@pytest.fixture(scope="module")
def mid_oracle():
    """The FP64 oracle on the 1024 x 512 emulsion (seed 2): fields and
    post-collision populations after 1000 and 2000 steps."""
    w = workloads.mid()
    ora = Oracle(ModelParams(**w["params"]), w["rho_a"], w["rho_b"], w["temp"],
                 solid=w["solid"], t_bottom=w["t_bottom"])
    out = {}
    for t in (1000, 2000):
        ora.step(t - ora.t)
        out[t] = (ora.fields(), ora.post_collision(), ora.observables())
    return w, out


def l2_rel(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


@pytest.mark.parametrize("fused", ["0", "1"])
def test_fp32_mid_1000_and_2000_steps(mid_oracle, fused):
    """The FP32 benchmark emulsion 1024 x 512 (seed 2, buoyant, noisy) against
    the FP64 oracle element by element after 1000 and 2000 steps, with single
    steps and with the fused two-step kernel: temperature <= 1e-5 of its
    largest value; densities, populations and u^H (over max|u|) at the bars
    below, set from a plain FP32 implementation of the same scheme; u^H is
    also reported as an L2 relative error."""
    w, ref = mid_oracle
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision="fp32",
                     launch={"fused": "always" if fused == "1" else "never"})
    assert (sim.launch_info()["fused_rows"] > 0) == (fused == "1")
    results = {}
    for t in (1000, 2000):
        sim.step(t - sim.t)
        f_ref, p_ref, o_ref = ref[t]
        got = sim.fields()
        errs = field_errors(got, f_ref)
        errs["u_l2"] = max(l2_rel(got["ux"], f_ref["ux"]), l2_rel(got["uy"], f_ref["uy"]))
        perr = pop_errors(sim.populations(), p_ref)
        o = sim.observables()
        errs["nu"] = abs(o["nu"] - o_ref["nu"]) / abs(o_ref["nu"])
        print(f"fp32 mid fused={fused} t={t}", errs, perr, flush=True)
        results[t] = (errs, perr, o, o_ref)
    # Bars (t: densities and populations, velocity): the 1e-5 of FP32 parity
    # holds here for T only. This buoyant emulsion (Ra ~ 5e5, 882 droplets)
    # amplifies rounding-level differences at the interfaces: a plain FP32
    # implementation of the scheme (vectorised, CPU) is at rho 1.1e-4 / 1.9e-4
    # and u 1.5e-4 / 3.0e-4 after 1000 / 2000 steps; these bars require at
    # least half that accuracy (measured here: rho 4.3e-5 / 7.3e-5, T 5.6e-7
    # / 1.2e-6, u 6.2e-5 / 1.1e-4).
    bars = {1000: (6e-5, 1e-4), 2000: (1e-4, 1.5e-4)}
    for t, (errs, perr, o, o_ref) in results.items():
        bar, bar_u = bars[t]
        assert errs["temp"] <= 1e-5, (t, errs)
        assert max(errs[k] for k in FIELDS) <= bar, (t, errs)
        assert max(perr.values()) <= bar, (t, perr)
        assert max(errs["ux"], errs["uy"]) <= bar_u, (t, errs)
        for k in ("mass_a", "mass_b", "sum_t"):
            assert o[k] == pytest.approx(o_ref[k], rel=1e-6), (t, k)


def test_observables_from_the_last_step_equal_a_reevaluated_time_level():
    """tlb_step's last launch forms the observable sums; after a new bottom
    temperature the time level is evaluated again by a separate pass. Both
    give the oracle's observables (FP64, posts, per-column T_b, fused
    launches before the last step)."""
    c = posts_case()
    sim, ora = run_pair(c, 41, "fp64")
    a = sim.observables()
    sim.set_bottom_temperature(c["t_bottom"])
    b = sim.observables()
    oo = ora.observables()
    for k in ("mass_a", "mass_b", "sum_t", "ke", "nu", "nu_top"):
        assert a[k] == pytest.approx(b[k], rel=1e-13, abs=1e-15), (k, a[k], b[k])
        assert a[k] == pytest.approx(oo[k], rel=1e-11, abs=1e-14), (k, a[k], oo[k])


@pytest.mark.parametrize("name", ["mid", "large"])
def test_fp32_full_size_one_step_from_gpu_state(name):
    """Benchmark lattices in the benchmark's launch configuration: after 20
    GPU steps, the oracle streams the GPU's post-collision state and both
    take one more step; every population and field is compared."""
    w = workloads.CONFIGS[name]()
    p = w["params"]
    sim = Simulation(p, w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision="fp32")
    sim.step(20)
    state = sim.populations()
    sim.step(1)
    got_pop = sim.populations()
    got_fields = sim.fields()
    ora = Oracle(ModelParams(**p), w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                 t_bottom=w["t_bottom"])
    ora.load_post_collision(state, 21)
    errs = field_errors(got_fields, ora.fields())
    print(name, "one-step fields", errs)
    assert max(errs.values()) <= 1e-5, errs
    ref = ora.post_collision()
    perr = pop_errors(got_pop, ref)
    print(name, "one-step populations", perr)
    assert max(perr.values()) <= 1e-5, perr


@pytest.mark.parametrize("name", ["mid"])
def test_fp32_full_size_mass_and_translation_over_1000_steps(name):
    """Per-component mass is conserved over 1000 FP32 steps (the FP64
    reduction sees only FP32 storage rounding), and shifting the start by 37
    columns shifts the result bitwise (no strip- or chunk-edge effects)."""
    w = workloads.CONFIGS[name]()
    p = w["params"]
    a = Simulation(p, w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"], t_bottom=w["t_bottom"],
                   precision="fp32")
    m0 = a.observables()
    a.step(1000)
    m1 = a.observables()
    for k in ("mass_a", "mass_b"):
        assert abs(m1[k] - m0[k]) / m0[k] < 1e-5, (k, m0[k], m1[k])
    sh = lambda z: np.roll(z, 37, axis=1)
    b = Simulation(p, sh(w["rho_a"]), sh(w["rho_b"]), sh(w["temp"]),
                   solid=None if w["solid"] is None else sh(w["solid"]),
                   t_bottom=sh(w["t_bottom"][None, :])[0], precision="fp32")
    b.step(1000)
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(sh(fa[k]), fb[k]), k


def test_wide_offsets_match_narrow_bitwise():
    """The 64-bit offset variant (used for buffers >= 4 GiB) gives bitwise the
    same state as the 32-bit one; forced on a small lattice with posts."""
    c = posts_case(lx=96, ly=48, seed=3)
    runs = []
    for wide in (False, True):
        sim = Simulation(c["params"], c["rho_a"], c["rho_b"], c["temp"], solid=c["solid"],
                         t_bottom=c["t_bottom"], precision="fp32",
                         launch={"wide_offsets": wide, "fused": "never"})
        sim.step(40)
        runs.append((sim.populations(), sim.fields()))
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in runs[0][1]:
        assert np.array_equal(runs[0][1][k], runs[1][1][k]), k


# ------------------------------------------------- 16-bit deviation storage

W9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def half_ulp(dev, mant_bits, min_exp):
    """Half a unit in the last place of |dev| in a binary format with
    `mant_bits` explicit mantissa bits and smallest normal exponent
    `min_exp` (subnormals below it)."""
    e = np.floor(np.log2(np.maximum(np.abs(dev), 2.0 ** min_exp)))
    return 0.5 * 2.0 ** (e - mant_bits)


FORMATS = {"fp16dev": (10, -14), "bf16dev": (7, -126), "fix16dev": None}
FIX_UNIT = 2.0 ** -15


@pytest.mark.parametrize("precision", sorted(FORMATS))
def test_dev16_one_step_is_the_oracle_step_rounded_once(precision):
    """From the GPU's own 16-bit state (decoded exactly), one GPU step equals
    the oracle's FP64 step up to one round-to-nearest of each stored moving
    deviation (half an ulp of the floating formats; half a unit of the
    fixed-point one) plus FP32 arithmetic; the rest population, the exact
    remainder of the zeroth moment, absorbs the eight roundings of its node
    (fixed point: 4 units; FP16 / BF16, stored in FP32: the sum of the eight
    half ulps). The fields of the streamed state agree to FP32 arithmetic."""
    w = workloads.crop(steps=0)
    p = w["params"]
    sim = Simulation(p, w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision=precision)
    sim.step(20)
    state = sim.populations()
    sim.step(1)
    got_pop, got_fields = sim.populations(), sim.fields()
    ora = Oracle(ModelParams(**p), w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                 t_bottom=w["t_bottom"]).load_post_collision(state, 21)
    errs = field_errors(got_fields, ora.fields())
    print(precision, "fields after load", errs)
    if FORMATS[precision] is None:
        # fixed point rounds the anti-bounce-back wall source onto its grid:
        # half a unit on each of the (at most 3) bounced links of a wall node
        assert errs["temp"] <= 3 * 0.5 * FIX_UNIT + 2e-6, errs
        errs.pop("temp")
    assert max(errs.values()) <= 2e-6, errs
    ref = ora.post_collision()
    pr = sim.params
    refs = np.concatenate([W9 * pr.rho_ref[0], W9 * pr.rho_ref[1], W9 * pr.t_ref])[:, None, None]
    fluid = (w["solid"] == 0)[None]
    dev = ref - refs
    if FORMATS[precision] is None:
        rounding = np.full_like(dev, 0.5 * FIX_UNIT)
        rounding[[0, 9, 18]] = 4.0 * FIX_UNIT
        # g also carries the wall-source rounding of T at wall nodes (above)
        rounding[18:27] += 3 * 0.5 * FIX_UNIT
    else:
        rounding = half_ulp(dev, *FORMATS[precision])
        for k in (0, 9, 18):
            rounding[k] = rounding[k + 1:k + 9].sum(axis=0)
    bound = rounding + 4e-6 * np.maximum(np.abs(ref), 1e-3)
    excess = np.where(fluid, np.abs(got_pop - ref) - bound, 0.0)
    print(precision, "max |gpu-ora|/bound", float(np.where(fluid, np.abs(got_pop - ref) / bound, 0).max()))
    assert excess.max() <= 0.0


@pytest.mark.parametrize("precision,fused", [("fp16dev", "0"), ("bf16dev", "0"),
                                             ("fp16dev", "1"), ("bf16dev", "1")])
def test_dev16_float_conserves_each_component_mass(precision, fused):
    """FP16 / BF16 deviations with FP32 rest populations: each component's
    mass (FP64 sum of the densities) after 1000 steps on the 512 x 256 crop
    with posts. Single steps move only stored values between nodes, and each
    collision stores the exact remainder of the rounded moving populations,
    so the mass changes only where FP32 sums of stored values round (BF16
    values much smaller than their node's sum): bar 1e-9. The fused kernel
    keeps its intermediate level in FP32 (rounded like FP32 storage, whose
    drift is ~1e-8 over 5000 steps): bar 1e-6."""
    w = workloads.crop(steps=0)
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision=precision,
                     launch={"fused": "always" if fused == "1" else "never"})
    assert (sim.launch_info()["fused_rows"] > 0) == (fused == "1")
    m0 = sim.observables()
    sim.step(1000)
    m1 = sim.observables()
    drift = {k: abs(m1[k] - m0[k]) / m0[k] for k in ("mass_a", "mass_b")}
    print(precision, "fused", fused, "mass drift over 1000 steps", drift, flush=True)
    assert max(drift.values()) <= (1e-9 if fused == "0" else 1e-6), drift


def test_fix16_conserves_each_component_mass_exactly():
    """Fixed-point storage: the integer sum of every component's stored
    deviations over the fluid nodes is the same after 1000 steps (streaming
    and bounce-back move integers, the collision's rest population takes the
    exact remainder)."""
    w = workloads.crop(steps=0)
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision="fix16dev")
    pr = sim.params
    fluid = w["solid"] == 0

    def integer_masses():
        pop = sim.populations()
        out = []
        for k, ref in ((0, pr.rho_ref[0]), (9, pr.rho_ref[1])):
            refs = (W9 * np.float64(np.float32(ref)))[:, None, None]
            q = np.rint((pop[k:k + 9] - refs) / FIX_UNIT)
            assert np.abs((pop[k:k + 9] - refs) / FIX_UNIT - q)[:, fluid].max() < 1e-6
            out.append(int(q[:, fluid].astype(np.int64).sum()))
        return out

    m0 = integer_masses()
    sim.step(1000)
    assert integer_masses() == m0


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fix16dev"])
def test_tau_one_path_matches_general_path_bitwise(precision):
    """At tau = tau_g = 1 the collision returns the equilibria; the kernels
    then keep only the moments of the pulled rows. That path must give
    bitwise the state of the general path (forced by the general_path launch
    flag)."""
    c = posts_case(lx=96, ly=48, seed=4)
    runs = []
    for general in (True, False):
        sim = Simulation(c["params"], c["rho_a"], c["rho_b"], c["temp"], solid=c["solid"],
                         t_bottom=c["t_bottom"], precision=precision,
                         launch={"general_path": general, "fused": "never"})
        sim.step(30)
        runs.append((sim.populations(), sim.fields(), sim.observables()))
        sim.close()
    assert np.array_equal(runs[0][0], runs[1][0])
    for k in runs[0][1]:
        assert np.array_equal(runs[0][1][k], runs[1][1][k]), k
    assert runs[0][2] == runs[1][2]


def test_general_path_fp32_tau_not_one():
    """tau = 0.8, tau_g = 1.3 (general path) against the oracle, FP32, 300
    steps."""
    c = posts_case(lx=128, ly=64, seed=12)
    c["params"] = dict(c["params"], tau=0.8, tau_g=1.3)
    sim, ora = run_pair(c, 300, "fp32")
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 tau 0.8/1.3 fields", errs)
    assert max(errs[k] for k in FIELDS) <= 1e-5, errs
    assert max(errs["ux"], errs["uy"]) <= 3e-5, errs
