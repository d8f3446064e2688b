"""Pins of the oracle's moving walls and stress observables (Couette set-up
of Sec. 3.2.2; stress of Sec. 2.1 below Eq. (14)) against closed forms.

* Steady Couette flow between half-way walls moving at u_b, u_t: the
  profile u_x(y) = u_b + (u_t - u_b)(y + 1/2)/ly is an exact steady state of
  BGK with momentum-corrected bounce-back, and the viscous stress is
  eta * gamma_dot with eta = rho cs^2 (tau - 1/2), gamma_dot = (u_t - u_b)/ly.
* Conduction between moving walls: the linear temperature profile stays
  exact when the anti-bounce-back uses the even part of the equilibrium at
  the wall velocity.
* Interaction pressure tensor on a field psi = a + b x y: at interior nodes
  P_xy = 1/2 psi(x) b sum_c G(c) c_x^2 c_y^2, with sum_c w c_x^2 c_y^2 = 1/9
  (nearest shell) and sum_c p c_x^2 c_y^2 = 4/21 (25-point weights of
  Fig. 1(b)).
* A state that depends on y only has P_xy = 0 (mirror symmetry in x) and
  a fluid at rest has no viscous stress.
"""
import numpy as np
import pytest

import workloads
from oracle.oracle import ModelParams, Oracle

CS2 = 1.0 / 3.0
FREE = dict(g12=0.0, g_a=(0.0, 0.0), g_r=(0.0, 0.0), alpha_g=0.0)


def couette(tau, ub, ut, lx=4, ly=16, steps=12000, tau_g=1.0):
    ra = np.full((ly, lx), 0.6)
    rb = np.full((ly, lx), 0.4)
    y = (np.arange(ly) + 0.5) / ly
    temp = np.repeat((1.0 - y)[:, None], lx, axis=1)
    p = ModelParams(tau=tau, tau_g=tau_g, u_wall=(ub, ut), t_top=0.0, **FREE)
    o = Oracle(p, ra, rb, temp, t_bottom=np.ones(lx), threads=1)
    o.step(steps)
    return o, y


@pytest.mark.parametrize("tau", [0.8, 1.0, 1.7])
def test_couette_profile_is_linear_and_stress_newtonian(tau):
    ub, ut = -0.02, 0.03
    o, y = couette(tau, ub, ut)
    f = o.fields()
    exact = ub + (ut - ub) * y
    assert np.abs(f["ux"] - exact[:, None]).max() < 1e-11
    assert np.abs(f["uy"]).max() < 1e-13
    rho = f["rho_a"] + f["rho_b"]
    assert np.abs(rho - 1.0).max() < 1e-12
    s = o.stress()
    eta = 1.0 * CS2 * (tau - 0.5)
    gamma = (ut - ub) / o.shape[0]
    assert np.abs(s["sxy_visc"] - eta * gamma).max() < 1e-12 * abs(eta * gamma) + 1e-15
    assert np.abs(s["pxy_int"]).max() == 0.0


def test_conduction_between_moving_walls_stays_linear():
    o, y = couette(1.0, -0.05, 0.05, tau_g=0.9, steps=6000)
    t = o.fields()["temp"]
    assert np.abs(t - (1.0 - y)[:, None]).max() < 1e-12


def test_moving_walls_conserve_each_component_mass():
    w = workloads.small()
    p = ModelParams(**dict(w["params"], u_wall=(-0.01, 0.02)))
    o = Oracle(p, w["rho_a"], w["rho_b"], w["temp"], threads=1)
    m0 = o.observables()
    o.step(150)
    m1 = o.observables()
    n = w["lx"] * w["ly"]
    for k in ("mass_a", "mass_b"):
        assert abs(m1[k] - m0[k]) <= 150 * 10 * n * 2.2e-16 * 1.4


def quadratic_state(lx, ly, a, b, rho0):
    x = np.arange(lx)[None, :]
    y = np.arange(ly)[:, None]
    psi = a + b * x * y
    return psi, -rho0 * np.log(1.0 - psi / rho0)


def test_pressure_tensor_on_a_quadratic_self_field():
    lx, ly, rho0 = 12, 10, 0.83
    ga, gr = -9.0, 8.1
    psi, rho = quadratic_state(lx, ly, 0.3, 1e-3, rho0)
    p = ModelParams(rho0=rho0, g12=0.0, g_a=(ga, 0.0), g_r=(gr, 0.0), alpha_g=0.0)
    o = Oracle(p, rho, np.full((ly, lx), 0.1), np.zeros((ly, lx)), threads=1)
    got = o.stress()["pxy_int"]
    want = 0.5 * psi * 1e-3 * (ga / 9.0 + gr * 4.0 / 21.0)
    inner = (slice(2, ly - 2), slice(2, lx - 2))
    assert np.abs(got[inner] - want[inner]).max() < 1e-14


def test_pressure_tensor_cross_term_on_a_quadratic_field():
    lx, ly, rho0, g12 = 12, 10, 0.83, 0.405
    x = np.arange(lx)[None, :]
    y = np.arange(ly)[:, None]
    rb = 0.2 + 2e-3 * x * y            # psi_x,B = rho_B / rho0 is quadratic
    ra = np.full((ly, lx), 0.7)        # psi_x,A constant
    p = ModelParams(rho0=rho0, g12=g12, g_a=(0.0, 0.0), g_r=(0.0, 0.0), alpha_g=0.0)
    o = Oracle(p, ra, rb, np.zeros((ly, lx)), threads=1)
    got = o.stress()["pxy_int"]
    want = 0.5 * g12 * (0.7 / rho0) * (2e-3 / rho0) / 9.0
    inner = (slice(2, ly - 2), slice(2, lx - 2))
    assert np.abs(got[inner] - want).max() < 1e-15


def test_layered_state_has_no_xy_stress():
    p = ModelParams(**dict(workloads.BASE_PARAMS))
    ly, lx = 12, 16
    prof_a = np.linspace(0.1, 1.3, ly)[:, None] * np.ones((1, lx))
    prof_b = np.linspace(1.2, 0.2, ly)[:, None] * np.ones((1, lx))
    o = Oracle(p, prof_a, prof_b, np.full((ly, lx), 0.5), threads=1)
    s = o.stress()
    assert np.abs(s["pxy_int"]).max() < 1e-16
    assert np.abs(s["sxy_visc"]).max() < 1e-16


@pytest.mark.parametrize("tau,tau_g", [(1.0, 1.0), (0.8, 0.7)])
def test_uniform_translation_with_comoving_walls_is_stationary(tau, tau_g):
    """Galilean check of both moving-wall rules (Sec. 2.2): a uniform fluid
    moving along x with the walls, at the walls' temperature, with wetting
    densities equal to the fluid's (so no force acts), is an exact steady
    state. Bounce-back with the momentum term returns f^eq_opp(rho, u_w), and
    anti-bounce-back against the even part 2 w_i T_w (1 + 4.5 (c_i.u_w)^2
    - 1.5 u_w^2) returns g^eq(T_w, u_w) at every wall link, for any tau;
    any other u_w^2 factor in the thermal rule moves the populations of the
    wall rows away from the equilibrium at the first step."""
    lx, ly, uw, tw = 8, 12, 0.05, 0.7
    ra, rb = np.full((ly, lx), 0.6), np.full((ly, lx), 0.4)
    p = ModelParams(**dict(workloads.BASE_PARAMS, tau=tau, tau_g=tau_g, alpha_g=0.0,
                           rho_wall=(0.6, 0.4), t_top=tw, u_wall=(uw, uw)))
    o = Oracle(p, ra, rb, np.full((ly, lx), tw), t_bottom=np.full(lx, tw),
               ux0=np.full((ly, lx), uw), uy0=np.zeros((ly, lx)), threads=1)
    start = o.populations()
    o.step(150)
    np.testing.assert_allclose(o.populations(), start, rtol=1e-13, atol=0)
    f = o.fields()
    np.testing.assert_allclose(f["ux"], uw, rtol=1e-13)
    assert np.abs(f["uy"]).max() < 1e-15
    np.testing.assert_allclose(f["temp"], tw, rtol=1e-14)
