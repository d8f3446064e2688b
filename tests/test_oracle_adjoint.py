"""Pins of the oracle adjoint (vectorised FP64 PyTorch form of the step,
differentiated by autograd): its forward against the C oracle, its gradient
against central finite differences of its own forward."""
import numpy as np
import pytest
import torch

import workloads
from oracle.oracle import ModelParams, Oracle
from oracle.torch_model import Model


def T(a):
    return torch.tensor(a, dtype=torch.float64)


def emulsion(lx, ly, seed, discs, radius):
    rng = np.random.default_rng(seed)
    inside = workloads.paint_discs(lx, ly, discs, radius)
    ra = np.where(inside, 1.36, 0.08) + rng.uniform(-0.01, 0.01, (ly, lx))
    rb = np.where(inside, 0.08, 1.36) + rng.uniform(-0.01, 0.01, (ly, lx))
    temp = workloads.conduction_profile(lx, ly) + rng.uniform(-1e-3, 1e-3, (ly, lx))
    return ra, rb, temp


def test_torch_forward_matches_c_oracle():
    """Same scheme written twice (C loops in push form, whole-array torch in
    pull form): post-collision f*(0) and pre-collision f(30) agree to
    round-off, as does the top-wall Nusselt number."""
    lx, ly = 48, 24
    ra, rb, temp = emulsion(lx, ly, 0, [(15.0, 11.0), (34.0, 13.0)], 6.0)
    tb = workloads.bottom_temperature_noise(lx, 5)
    params = dict(workloads.BASE_PARAMS, alpha_g=1e-3)
    o = Oracle(ModelParams(**params), ra, rb, temp, t_bottom=tb)
    m = Model(params, lx, ly)
    st = m.initial_state(T(ra), T(rb), T(temp))
    post0 = np.concatenate([s.numpy() for s in st])
    assert np.abs(post0 - o.post_collision()).max() < 1e-14
    for _ in range(30):
        st, pre, _ = m.step(st, T(tb))
    o.step(30)
    assert np.abs(torch.cat(pre).numpy() - o.populations()).max() < 1e-14
    assert float(m.nu_top(pre[2])) == pytest.approx(o.observables()["nu_top"], rel=1e-13)


def test_torch_gradient_matches_central_differences():
    """d(mean Nu_top over 40 steps)/d T_b(x) by reverse mode equals central
    differences (h = 1e-5, FP64) to 1e-6 relative at three columns."""
    lx, ly = 24, 12
    ra, rb, temp = emulsion(lx, ly, 1, [(8.0, 6.0)], 4.0)
    m = Model(dict(workloads.BASE_PARAMS, alpha_g=5e-3), lx, ly)
    st0 = m.initial_state(T(ra), T(rb), T(temp))
    tb = T(workloads.bottom_temperature_noise(lx, 5)).requires_grad_(True)
    m.loss(st0, tb, 40).backward()
    g = tb.grad.numpy()
    h = 1e-5
    for c in (0, 5, 17):
        tp, tm = tb.detach().clone(), tb.detach().clone()
        tp[c] += h
        tm[c] -= h
        fd = (float(m.loss(st0, tp, 40)) - float(m.loss(st0, tm, 40))) / (2 * h)
        assert g[c] == pytest.approx(fd, rel=1e-6)
