"""Pins of the oracle's droplet detection (bulk rho_A > B_th, clusters,
centres of mass; Sec. 2.4) and droplet Nusselt number (Sec. 3.3.2
Eq. (25)) against closed forms and a library routine:

* a disc of radius 5 centred on a node holds the 81 lattice points of the
  Gauss circle problem for r^2 = 25, its centre of mass is its centre and
  its mass is 81 rho_in; across the periodic x boundary the same holds;
* a droplet's number is the order of its smallest node index: for a disc
  centred at (x0, y0) that node is (x0, y0 - R);
* nodes touching only diagonally are separate droplets (4-connectivity);
* away from the x boundary the partition equals scipy.ndimage.label with
  its default (4-connected) structure;
* in pure conduction at rest (no forces) every droplet has Nu = 1.
"""
import numpy as np
import pytest
from scipy import ndimage

import workloads
from oracle.oracle import ModelParams, Oracle

RHO_IN, RHO_OUT = 1.36, 0.08
FREE = dict(g12=0.0, g_a=(0.0, 0.0), g_r=(0.0, 0.0), alpha_g=0.0)


def oracle_of(inside, temp=None, **params):
    ly, lx = inside.shape
    ra = np.where(inside, RHO_IN, RHO_OUT)
    rb = np.where(inside, RHO_OUT, RHO_IN)
    if temp is None:
        temp = workloads.conduction_profile(lx, ly)
    return Oracle(ModelParams(**dict(workloads.BASE_PARAMS, **params)), ra, rb, temp, threads=1)


def disc_mask(lx, ly, x0, y0, r):
    x = np.arange(lx)[None, :]
    y = np.arange(ly)[:, None]
    dx = (x - x0 + lx / 2) % lx - lx / 2
    return dx * dx + (y - y0) ** 2 <= r * r


@pytest.mark.parametrize("x0", [20, 1])
def test_disc_size_centre_and_mass(x0):
    lx, ly = 48, 32
    d = oracle_of(disc_mask(lx, ly, x0, 15, 5)).droplets(0.8)
    assert len(d["root"]) == 1
    assert d["size"][0] == 81
    assert d["mass"][0] == pytest.approx(81 * RHO_IN, rel=1e-14)
    assert d["x"][0] == pytest.approx(x0, abs=1e-12)
    assert d["y"][0] == pytest.approx(15, abs=1e-12)
    assert (d["label"] == 0).sum() == 81 and (d["label"] == -1).sum() == lx * ly - 81


def test_numbering_is_by_smallest_node_index():
    lx, ly, r = 64, 48, 4
    centres = [(40, 30), (10, 12), (52, 8), (25, 33)]
    mask = np.zeros((ly, lx), bool)
    for c in centres:
        mask |= disc_mask(lx, ly, c[0], c[1], r)
    d = oracle_of(mask).droplets(0.8)
    want = sorted((y - r) * lx + x for x, y in centres)
    assert list(d["root"]) == want
    for i, k in enumerate(want):
        assert d["label"].flat[k] == i


def test_diagonal_contact_does_not_join():
    lx, ly = 16, 12
    mask = np.zeros((ly, lx), bool)
    mask[5, 5] = mask[6, 6] = True
    assert len(oracle_of(mask).droplets(0.8)["root"]) == 2
    mask[5, 6] = True
    d = oracle_of(mask).droplets(0.8)
    assert len(d["root"]) == 1 and d["size"][0] == 3


def test_partition_matches_scipy_label():
    lx, ly = 96, 64
    rng = np.random.default_rng(3)
    field = ndimage.gaussian_filter(rng.normal(size=(ly, lx)), 2.0)
    mask = field > 0.05
    mask[:, :2] = mask[:, -2:] = False  # no cluster touches the periodic seam
    d = oracle_of(mask).droplets(0.8)
    ref, n = ndimage.label(mask)
    assert len(d["root"]) == n
    # same partition: a bijection between labels
    pairs = {(a, b) for a, b in zip(d["label"][mask], ref[mask])}
    assert len(pairs) == n and len({a for a, _ in pairs}) == n
    assert np.all((d["label"] >= 0) == mask)
    np.testing.assert_array_equal(np.bincount(d["label"][mask]), d["size"])


def test_conduction_gives_unit_droplet_nusselt():
    lx, ly = 64, 40
    mask = disc_mask(lx, ly, 20.3, 17.6, 6) | disc_mask(lx, ly, 47, 25, 5)
    d = oracle_of(mask, **FREE).droplets(0.8)
    assert len(d["root"]) == 2
    np.testing.assert_allclose(d["nu"], 1.0, rtol=1e-12)


def test_droplet_nusselt_with_flow_on_linear_fields():
    """Eq. (25) with the flow on, at t = 0 (fields = the initial ones; no
    forces act without couplings): a 12 x 9 block droplet of uniform density
    (centre of mass (19.5, 18): between columns, on a row), u^H_y = U + s x
    and T = a + b x + c y. Bilinear interpolation reproduces the linear
    fields at the centre and the central difference gives dT/dy = c, so
    Nu_d = ((U + s X)(a + b X + c Y) - kappa c) / (kappa dt_nominal / ly).
    The product of the interpolated u_y and T differs from the interpolated
    product by s b a_x (1 - a_x), and swapped x/y weights move the centre, so
    either mistake changes Nu_d."""
    lx, ly = 48, 40
    inside = np.zeros((ly, lx), bool)
    inside[14:23, 14:26] = True
    x = np.arange(lx)[None, :] * np.ones((ly, 1))
    y = np.arange(ly)[:, None] * np.ones((1, lx))
    a, b, c, u0, s = 0.3, 0.01, 0.02, 0.01, 0.002
    tau_g, dtn = 0.8, 0.7
    kappa = (tau_g - 0.5) / 3.0
    ra = np.where(inside, RHO_IN, RHO_OUT)
    rb = np.where(inside, RHO_OUT, RHO_IN)
    o = Oracle(ModelParams(**dict(workloads.BASE_PARAMS, tau_g=tau_g, dt_nominal=dtn, **FREE)),
               ra, rb, a + b * x + c * y, ux0=np.full((ly, lx), 0.003), uy0=u0 + s * x, threads=1)
    d = o.droplets(0.8)
    assert len(d["root"]) == 1 and d["size"][0] == 12 * 9
    X, Y = 19.5, 18.0
    assert d["x"][0] == pytest.approx(X, abs=1e-12) and d["y"][0] == pytest.approx(Y, abs=1e-12)
    expect = ((u0 + s * X) * (a + b * X + c * Y) - kappa * c) / (kappa * dtn / ly)
    assert d["nu"][0] == pytest.approx(expect, rel=1e-12)
