"""GPU moving walls and stress observables (Couette walls of Sec. 2.2 and
Sec. 3.2.2) versus the FP64 oracle, element by element, and versus the
closed-form steady Couette flow.

Bars: FP64 <= 1e-12 relative (fields, populations, stress fields, row
averages); FP32 <= 1e-5 for densities and temperature after 500 steps
(velocities 3e-5 of max|u|) and <= 5e-4 of max|stress| for the stress
fields (the viscous stress is a difference of populations ~0.03 known to
FP32 rounding, against stresses of ~1e-4). Under shear the droplets keep
moving, so FP32 rounding of the interface forces integrates into a
trajectory offset that grows about as t^2 (1.4e-6 at 300 steps, 6e-6 at
600, 1.8e-5 at 1000, against 2.9e-6 at 1000 with walls at rest); FP64 runs
of the oracle do not amplify perturbations of that size (3e-8 stays below
8e-8 over 1500 steps) and the FP64 path of the same kernel code matches the
oracle to 1e-12, so the growth is the arithmetic type, not the logic.
"""
import numpy as np
import pytest

import workloads
from oracle.oracle import ModelParams, Oracle
from paper_2109_12565_amd import Simulation

from test_gpu_parity import field_errors, pop_errors, posts_case, rel

pytestmark = pytest.mark.gpu

U_WALL = (-0.01, 0.02)


def pair(case, precision, steps, **extra):
    p = dict(case["params"], **extra)
    sim = Simulation(p, case["rho_a"], case["rho_b"], case["temp"], solid=case.get("solid"),
                     t_bottom=case.get("t_bottom"), precision=precision)
    ora = Oracle(ModelParams(**p), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    sim.step(steps)
    ora.step(steps)
    return sim, ora


def oracle_row_averages(ora, solid):
    f, s = ora.fields(), ora.stress()
    fluid = np.ones(f["ux"].shape, bool) if solid is None else solid == 0
    n = fluid.sum(axis=1)
    u = np.where(fluid, f["ux"], 0.0).sum(axis=1)
    pxy = np.where(fluid, s["sxy_visc"] - s["pxy_int"], 0.0).sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(n > 0, u / n, 0.0), np.where(n > 0, pxy / n, 0.0)


def test_fp64_moving_walls_emulsion():
    sim, ora = pair(workloads.small(), "fp64", 200, u_wall=U_WALL)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr
    og, oo = sim.observables(), ora.observables()
    for k in ("mass_a", "mass_b", "sum_t", "ke", "nu", "nu_top"):
        assert og[k] == pytest.approx(oo[k], rel=1e-11, abs=1e-14), (k, og[k], oo[k])


def test_fp64_moving_walls_with_posts_and_top_patch():
    """Posts and a rough patch inside the lattice stay at rest while the flat
    walls move; per-column T_b."""
    sim, ora = pair(posts_case(), "fp64", 150, u_wall=U_WALL)
    errs = field_errors(sim.fields(), ora.fields())
    assert max(errs.values()) <= 1e-12, errs
    perr = pop_errors(sim.populations(), ora.post_collision())
    assert max(perr.values()) <= 1e-12, perr


def test_fp32_moving_walls_500_steps():
    sim, ora = pair(workloads.small(), "fp32", 500, u_wall=U_WALL)
    errs = field_errors(sim.fields(), ora.fields())
    print("fp32 moving walls", errs)
    for k in ("rho_a", "rho_b", "temp"):
        assert errs[k] <= 1e-5, errs
    for k in ("ux", "uy"):
        assert errs[k] <= 3e-5, errs


@pytest.mark.parametrize("tau", [1.0, 0.8])
@pytest.mark.parametrize("steps", [0, 150])
def test_fp64_stress_fields_and_row_averages(tau, steps):
    case = posts_case()
    sim, ora = pair(case, "fp64", steps, u_wall=U_WALL, tau=tau)
    got, ref = sim.stress(), ora.stress()
    for k in ("sxy_visc", "pxy_int"):
        assert rel(got[k], ref[k]) <= 1e-12, (k, rel(got[k], ref[k]))
    rows = sim.row_averages()
    u_ref, p_ref = oracle_row_averages(ora, case["solid"])
    assert rel(rows["u_av"], u_ref) <= 1e-12
    assert rel(rows["pxy_av"], p_ref) <= 1e-12


def test_fp32_stress_fields():
    case = workloads.small()
    sim, ora = pair(case, "fp32", 200, u_wall=U_WALL)
    got, ref = sim.stress(), ora.stress()
    for k in ("sxy_visc", "pxy_int"):
        assert rel(got[k], ref[k]) <= 5e-4, (k, rel(got[k], ref[k]))


def test_couette_steady_state_on_the_gpu():
    """Closed form: between walls moving at u_b, u_t, a fluid without
    interactions reaches u_x(y) = u_b + (u_t - u_b)(y + 1/2)/ly exactly, with
    viscous stress rho cs^2 (tau - 1/2) (u_t - u_b)/ly in every row."""
    lx, ly, tau, ub, ut = 64, 16, 0.8, -0.02, 0.03
    p = dict(workloads.BASE_PARAMS, g12=0.0, g_a=(0.0, 0.0), g_r=(0.0, 0.0), alpha_g=0.0,
             tau=tau, u_wall=(ub, ut))
    sim = Simulation(p, np.full((ly, lx), 0.6), np.full((ly, lx), 0.4), np.zeros((ly, lx)),
                     precision="fp64")
    sim.step(12000)
    y = (np.arange(ly) + 0.5) / ly
    rows = sim.row_averages()
    assert np.abs(rows["u_av"] - (ub + (ut - ub) * y)).max() < 1e-11
    eta_gamma = 1.0 / 3.0 * (tau - 0.5) * (ut - ub) / ly
    assert np.abs(rows["pxy_av"] - eta_gamma).max() < 1e-12 * eta_gamma + 1e-16


def test_adjoint_refuses_moving_walls():
    w = workloads.small()
    with Simulation(dict(w["params"], u_wall=U_WALL), w["rho_a"], w["rho_b"], w["temp"],
                    precision="fp64") as sim:
        with pytest.raises(Exception) as e:
            sim.forward_taped(5, 2)
        assert "walls at rest" in str(e.value)


@pytest.mark.parametrize("precision,fused,tol", [("fp64", "0", 1e-13), ("fp64", "1", 1e-13),
                                                 ("fp32", "0", 2e-6), ("fp32", "1", 2e-6)])
def test_uniform_translation_with_comoving_walls_is_stationary(precision, fused, tol):
    """Both moving-wall rules on the GPU (Sec. 2.2): a uniform fluid moving
    with the walls at the walls' temperature, wetting densities equal to the
    fluid's, stays at its start equilibrium (single and fused launches)."""
    lx, ly, uw, tw = 64, 24, 0.05, 0.7
    p = dict(workloads.BASE_PARAMS, alpha_g=0.0, rho_wall=(0.6, 0.4), t_top=tw, u_wall=(uw, uw))
    sim = Simulation(p, np.full((ly, lx), 0.6), np.full((ly, lx), 0.4), np.full((ly, lx), tw),
                     t_bottom=np.full(lx, tw), ux0=np.full((ly, lx), uw), uy0=np.zeros((ly, lx)),
                     precision=precision, launch={"fused": "always" if fused == "1" else "never"})
    start = sim.populations()
    sim.step(151)
    assert rel(sim.populations(), start) <= tol
    f = sim.fields()
    assert np.abs(f["ux"] - uw).max() <= tol * 10 and np.abs(f["uy"]).max() <= tol
    assert np.abs(f["temp"] - tw).max() <= tol
