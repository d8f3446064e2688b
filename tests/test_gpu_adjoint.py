"""GPU discrete adjoint (tlb_forward_taped / tlb_adjoint_step) versus the
oracle adjoint and finite differences.

Loss: L(T_b) = time average over the run of the top-wall Nusselt number,
2 ly / dt_nominal * mean_x (T(x, ly-1) - t_top), as a function of the bottom
wall temperature profile T_b(x).

Bars:
  * FP64 GPU gradient = oracle adjoint (reverse-mode autograd through the
    vectorised FP64 torch form of the step) to 1e-10 of max|grad|, on the
    128 x 64 case and on a strongly buoyant 64 x 16 case whose checkpoint
    segments are ragged;
  * FP32 GPU gradient = central finite differences of the FP64 GPU loss
    (h = 1e-3) to 1e-3 of max|FD| at 16 seeded columns of a 1024 x 64
    strip, N = 500, checkpoints every 25 steps; with the moments of every
    step kept, = the FP64 gradient to 1e-3 of its max;
  * at 1024 x 512 over 500 steps the top wall is outside the bottom wall's
    domain of dependence for any practical purpose (sound front c_s N ~ 289
    rows, thermal diffusion length sqrt(kappa N) ~ 9 rows): both the adjoint
    and the finite differences must vanish to round-off there.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle.torch_model import Model
from paper_2109_12565_amd import Simulation, TlbError, top_nusselt_loss

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(a, dtype=torch.float64)


def make_sim(case, precision, t_bottom=None, launch=None, **params):
    p = dict(case["params"], **params)
    tb = case["t_bottom"] if t_bottom is None else t_bottom
    return Simulation(p, case["rho_a"], case["rho_b"], case["temp"], t_bottom=tb,
                      precision=precision, launch=launch)


def gpu_loss_and_grad(case, precision, tb, nsteps, ckpt, **params):
    with make_sim(case, precision, tb, **params) as sim:
        loss = sim.forward_taped(nsteps, ckpt)
        return loss, sim.adjoint(nsteps)


def oracle_loss_and_grad(case, tb, nsteps, **params):
    p = dict(case["params"], **params)
    m = Model(p, case["lx"], case["ly"])
    st0 = m.initial_state(T(case["rho_a"]), T(case["rho_b"]), T(case["temp"]))
    t = T(tb).requires_grad_(True)
    loss = m.loss(st0, t, nsteps)
    loss.backward()
    return float(loss.detach()), t.grad.numpy().copy()


def buoyant_case():
    """64 x 16, one droplet, strong buoyancy: every term of the step's
    adjoint carries weight in dL/dT_b within a few tens of steps."""
    lx, ly = 64, 16
    rng = np.random.default_rng(11)
    inside = workloads.paint_discs(lx, ly, [(20.0, 8.0)], 5.0)
    ra = np.where(inside, 1.36, 0.08) + rng.uniform(-0.01, 0.01, (ly, lx))
    rb = np.where(inside, 0.08, 1.36) + rng.uniform(-0.01, 0.01, (ly, lx))
    temp = workloads.conduction_profile(lx, ly) + rng.uniform(-1e-3, 1e-3, (ly, lx))
    return dict(lx=lx, ly=ly, rho_a=ra, rho_b=rb, temp=temp,
                t_bottom=workloads.bottom_temperature_noise(lx, 5),
                params=dict(workloads.BASE_PARAMS, alpha_g=5e-3))


@pytest.mark.parametrize("ckpt", [25, 7, 2, 1])
def test_fp64_adjoint_matches_oracle_buoyant(ckpt):
    case = buoyant_case()
    n = 60
    loss, g = gpu_loss_and_grad(case, "fp64", case["t_bottom"], n, ckpt)
    lo, go = oracle_loss_and_grad(case, case["t_bottom"], n)
    assert abs(loss - lo) <= 1e-12 * abs(lo)
    assert np.abs(go).max() > 1e-6
    assert np.abs(g - go).max() <= 1e-10 * np.abs(go).max()


def test_fp64_adjoint_matches_oracle_small_case():
    case = workloads.small()
    tb = workloads.bottom_temperature_noise(case["lx"], 5)
    n = 100
    loss, g = gpu_loss_and_grad(case, "fp64", tb, n, 25)
    lo, go = oracle_loss_and_grad(case, tb, n)
    assert abs(loss - lo) <= 1e-12 * abs(lo)
    assert np.abs(go).max() > 0
    assert np.abs(g - go).max() <= 1e-10 * np.abs(go).max()


@pytest.mark.parametrize("ckpt", [10, 1])
def test_fp64_adjoint_matches_oracle_general_tau(ckpt):
    """tau != 1 exercises the relaxation terms of the adjoint (FP64); its
    tape holds states (checkpoints every 10 steps, or every state)."""
    case = buoyant_case()
    n = 40
    loss, g = gpu_loss_and_grad(case, "fp64", case["t_bottom"], n, ckpt, tau=0.8, tau_g=1.3)
    lo, go = oracle_loss_and_grad(case, case["t_bottom"], n, tau=0.8, tau_g=1.3)
    assert abs(loss - lo) <= 1e-12 * abs(lo)
    assert np.abs(g - go).max() <= 1e-10 * np.abs(go).max()


def fd_loss(case, tb, n):
    with make_sim(case, "fp64", tb) as sim:
        return sim.forward_taped(n, n)


def test_fp32_adjoint_matches_finite_differences_strip():
    case = workloads.adjoint_strip()
    lx, n, h = case["lx"], case["steps"], 1e-3
    tb = workloads.bottom_temperature_noise(lx, 5)
    cols = np.sort(np.random.default_rng(6).choice(lx, 16, replace=False))
    _, g32 = gpu_loss_and_grad(case, "fp32", tb, n, 25)
    _, g32_all = gpu_loss_and_grad(case, "fp32", tb, n, 1)  # moments of every step
    _, g64 = gpu_loss_and_grad(case, "fp64", tb, n, 25)
    fd = []
    for c in cols:
        tp, tm = tb.copy(), tb.copy()
        tp[c] += h
        tm[c] -= h
        fd.append((fd_loss(case, tp, n) - fd_loss(case, tm, n)) / (2 * h))
    fd = np.array(fd)
    scale = np.abs(fd).max()
    assert scale > 1e-7
    assert np.abs(g64[cols] - fd).max() <= 1e-5 * scale
    assert np.abs(g32[cols] - fd).max() <= 1e-3 * scale
    assert np.abs(g32 - g64).max() <= 1e-3 * np.abs(g64).max()
    assert np.abs(g32_all - g64).max() <= 1e-3 * np.abs(g64).max()


def test_adjoint_vanishes_outside_domain_of_dependence_mid():
    case = workloads.mid()
    lx, n, h = case["lx"], 500, 1e-3
    tb = workloads.bottom_temperature_noise(lx, 5)
    loss, g = gpu_loss_and_grad(case, "fp32", tb, n, 25)
    assert np.isfinite(loss) and np.all(np.isfinite(g))
    assert np.abs(g).max() < 1e-12
    c = 100
    tp, tm = tb.copy(), tb.copy()
    tp[c] += h
    tm[c] -= h
    fd = (fd_loss(case, tp, n) - fd_loss(case, tm, n)) / (2 * h)
    assert abs(fd) < 1e-10


def test_taped_run_matches_plain_steps_and_observables():
    """The taped forward advances exactly as tlb_step (bitwise) and its loss is
    the mean of the per-step nu_top observable (single steps on both sides)."""
    case = buoyant_case()
    n = 30
    single = {"fused": "never"}
    with make_sim(case, "fp64", launch=single) as a, make_sim(case, "fp64", launch=single) as b:
        loss = a.forward_taped(n, 8)
        nus = []
        for _ in range(n):
            b.step(1)
            nus.append(b.observables()["nu_top"])
        assert a.t == b.t == n
        assert np.array_equal(a.populations(), b.populations())
        assert loss == pytest.approx(np.mean(nus), rel=1e-13)
        # the adjoint leaves the current state alone and can run twice
        g1 = a.adjoint(n)
        g2 = a.adjoint(n, seed=2.0)
        assert np.array_equal(2.0 * g1, g2)
        assert np.array_equal(a.populations(), b.populations())


def test_fused_taped_run_matches_fused_steps_and_single_step_adjoint():
    """With the fused two-step kernel forced on, the taped run takes the same
    launches as tlb_step (fused pairs, the last steps single; checkpoints
    every 8 fall between pairs), so it advances bitwise like tlb_step; its
    loss, formed from the fused kernel's per-strip top-row sums, and the
    gradient of the reverse sweep equal those of the single-step taped run
    to rounding (FP64)."""
    case = buoyant_case()
    n = 30
    fused = {"fused": "always"}
    with make_sim(case, "fp64", launch=fused) as a, make_sim(case, "fp64", launch=fused) as b, \
            make_sim(case, "fp64", launch={"fused": "never"}) as c:
        assert a.launch_info()["fused_rows"] > 0
        loss = a.forward_taped(n, 8)
        b.step(n)
        assert np.array_equal(a.populations(), b.populations())
        ref_loss = c.forward_taped(n, 8)
        assert loss == pytest.approx(ref_loss, rel=1e-13)
        g, ref_g = a.adjoint(n), c.adjoint(n)
        scale = np.abs(ref_g).max()
        assert scale > 0
        assert np.abs(g - ref_g).max() <= 1e-11 * scale


@pytest.mark.parametrize("n", [30, 31])
def test_full_tape_fused_run_matches_steps_and_oracle(n):
    """ckpt_every = 1 at tau = 1 keeps the moments of every step's pulled
    state, written by the steps themselves (fused pairs both levels'), and no
    state; the run advances bitwise like tlb_step, the other buffer holds the
    previous state (the fields of the current time agree), and loss and
    gradient match the oracle adjoint and the checkpointed run, whose
    segments are recomputed into moments (FP64)."""
    case = buoyant_case()
    fused = {"fused": "always"}
    with make_sim(case, "fp64", launch=fused) as a, make_sim(case, "fp64", launch=fused) as b, \
            make_sim(case, "fp64", launch=fused) as c:
        assert a.launch_info()["fused_rows"] > 0
        loss = a.forward_taped(n, 1)
        b.step(n)
        assert np.array_equal(a.populations(), b.populations())
        fa, fb = a.fields(), b.fields()
        for k in fa:
            assert np.array_equal(fa[k], fb[k]), k
        ref_loss = c.forward_taped(n, 7)
        assert loss == pytest.approx(ref_loss, rel=1e-13)
        g, ref_g = a.adjoint(n), c.adjoint(n)
    lo, go = oracle_loss_and_grad(case, case["t_bottom"], n)
    assert abs(loss - lo) <= 1e-12 * abs(lo)
    scale = np.abs(go).max()
    assert scale > 1e-6
    assert np.abs(g - go).max() <= 1e-10 * scale
    assert np.abs(g - ref_g).max() <= 1e-11 * scale


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_checkpointed_sweep_is_repeatable(precision):
    """With checkpoints the segment recompute runs on a second stream beside
    the sweep; the events between them fix every dependency, so the gradient
    is bitwise the same on a fresh handle and for a second sweep of the same
    tape."""
    case = buoyant_case()
    n = 60
    grads = []
    for _ in range(2):
        with make_sim(case, precision) as sim:
            sim.forward_taped(n, 7)
            g = sim.adjoint(n)
            assert np.array_equal(g, sim.adjoint(n))
            grads.append(g)
    assert np.abs(grads[0]).max() > 0
    assert np.array_equal(grads[0], grads[1])


def test_automatic_tape_choice():
    """ckpt_every = 0 lets the library choose: on a small lattice the tape of
    every step fits, so the run and its gradient are those of ckpt_every = 1
    (bitwise, FP32)."""
    case = buoyant_case()
    n = 40
    with make_sim(case, "fp32") as a, make_sim(case, "fp32") as b:
        la, lb = a.forward_taped(n, 0), b.forward_taped(n, 1)
        assert la == lb
        assert np.array_equal(a.adjoint(n), b.adjoint(n))


def test_autograd_function_matches_adjoint():
    case = buoyant_case()
    n = 20
    tb = torch.tensor(case["t_bottom"], dtype=torch.float64, requires_grad=True)
    with make_sim(case, "fp64") as sim:
        loss = top_nusselt_loss(sim, tb, n, 5)
        (3.0 * loss).backward()
    _, g = gpu_loss_and_grad(case, "fp64", case["t_bottom"], n, 5)
    assert np.allclose(tb.grad.numpy(), 3.0 * g, rtol=1e-14, atol=0)


def test_adjoint_error_paths():
    case = buoyant_case()
    with make_sim(case, "fp64") as sim:
        with pytest.raises(TlbError) as e:
            sim.adjoint(5)
        assert e.value.code == -5
        sim.forward_taped(5, 2)
        with pytest.raises(TlbError) as e:
            sim.adjoint(6)
        assert e.value.code == -5
        sim.set_bottom_temperature(case["t_bottom"])
        with pytest.raises(TlbError) as e:
            sim.adjoint(5)
        assert e.value.code == -5
        with pytest.raises(TlbError) as e:
            sim.forward_taped(0, 1)
        assert e.value.code == -1
        with pytest.raises(TlbError) as e:
            sim.forward_taped(5, -1)
        assert e.value.code == -1
    with make_sim(case, "fix16dev") as sim:
        with pytest.raises(TlbError) as e:
            sim.forward_taped(5, 2)
        assert e.value.code == -1
    solid = np.zeros((case["ly"], case["lx"]), np.uint8)
    solid[0, 3] = 1
    p = dict(case["params"])
    with Simulation(p, case["rho_a"], case["rho_b"], case["temp"], solid=solid,
                    t_bottom=case["t_bottom"], precision="fp64") as sim:
        with pytest.raises(TlbError) as e:
            sim.forward_taped(5, 2)
        assert e.value.code == -1


def test_second_taped_window_invalidates_the_first_loss():
    """A handle holds one tape: differentiating a loss formed before a later
    taped run on the same Simulation raises instead of returning the later
    window's gradient; the latest loss still differentiates."""
    w = workloads.small()
    with make_sim(w, "fp64") as sim:
        tb = torch.tensor(w["t_bottom"], dtype=torch.float64, requires_grad=True)
        l1 = top_nusselt_loss(sim, tb, 6, 3)
        l2 = top_nusselt_loss(sim, tb, 6, 3)
        with pytest.raises(RuntimeError, match="taped again"):
            (l1 + l2).backward()
        tb.grad = None
        l3 = top_nusselt_loss(sim, tb, 6, 3)
        l3.backward()
        assert torch.isfinite(tb.grad).all()


def test_taped_run_rejects_fewer_than_three_columns():
    """The adjoint folds x offsets of two columns by one period, so a taped
    run needs lx >= 3 (checked before any adjoint kernel runs)."""
    rng = np.random.default_rng(4)
    ly, lx = 8, 2
    sim = Simulation(dict(workloads.BASE_PARAMS), rng.uniform(0.2, 1.2, (ly, lx)),
                     rng.uniform(0.2, 1.2, (ly, lx)), rng.uniform(0, 1, (ly, lx)), precision="fp64")
    with pytest.raises(TlbError) as e:
        sim.forward_taped(4, 2)
    assert e.value.code == -1 and "lx < 3" in str(e.value)
    sim.close()
