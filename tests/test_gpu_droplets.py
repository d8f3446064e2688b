"""GPU droplet detection and droplet Nusselt number (tlb_droplets) versus
the oracle.

Bars: labels, roots, sizes and the count are integers and must be equal
(the numbering is canonical: by smallest node index). Mass and centre are
exact fixed-point sums on the GPU against FP64 sums in the oracle: <= 1e-10
relative / absolute; the droplet Nusselt number <= 1e-9 relative to the
largest |Nu| (FP64 storage). At the full 4096x2048 size: properties that
define the partition (adjacent bulk nodes share a label, every label's root
is its smallest node, sizes add up to the bulk).
"""
import numpy as np
import pytest
from scipy import ndimage

import workloads
from oracle.oracle import ModelParams, Oracle
from paper_2109_12565_amd import Simulation

from test_gpu_parity import posts_case

pytestmark = pytest.mark.gpu


def compare(got, ref):
    assert len(got["root"]) == len(ref["root"])
    np.testing.assert_array_equal(got["label"], ref["label"])
    np.testing.assert_array_equal(got["root"], ref["root"])
    np.testing.assert_array_equal(got["size"], ref["size"])
    if len(ref["root"]):
        np.testing.assert_allclose(got["mass"], ref["mass"], rtol=1e-10)
        np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-10)
        np.testing.assert_allclose(got["y"], ref["y"], rtol=0, atol=1e-10)
        scale = np.abs(ref["nu"]).max()
        assert np.abs(got["nu"] - ref["nu"]).max() <= 1e-9 * scale


def pair(case, precision, steps, **extra):
    p = dict(case["params"], **extra)
    sim = Simulation(p, case["rho_a"], case["rho_b"], case["temp"], solid=case.get("solid"),
                     t_bottom=case.get("t_bottom"), precision=precision)
    ora = Oracle(ModelParams(**p), case["rho_a"], case["rho_b"], case["temp"],
                 solid=case.get("solid"), t_bottom=case.get("t_bottom"))
    sim.step(steps)
    ora.step(steps)
    return sim, ora


@pytest.mark.parametrize("steps", [0, 120])
def test_fp64_droplets_small(steps):
    sim, ora = pair(workloads.small(), "fp64", steps)
    got, ref = sim.droplets(0.8, labels=True), ora.droplets(0.8)
    assert len(ref["root"]) == 6
    compare(got, ref)


def test_fp64_droplets_with_posts_and_moving_walls():
    sim, ora = pair(posts_case(), "fp64", 150, u_wall=(-0.01, 0.02))
    compare(sim.droplets(0.8, labels=True), ora.droplets(0.8))


def test_random_clusters_across_the_seam_and_a_spanning_cluster():
    """A random bulk mask with clusters crossing the periodic x seam, one
    cluster spanning the whole width, and single-node clusters."""
    lx, ly = 300, 120
    rng = np.random.default_rng(8)
    field = ndimage.gaussian_filter(rng.normal(size=(ly, lx)), 1.5, mode="wrap")
    mask = field > 0.0
    mask[60, :] = True                      # spans the width (wraps onto itself)
    mask[5, 7] = True
    mask[4, 7] = mask[6, 7] = mask[5, 6] = mask[5, 8] = False  # an isolated node
    ra = np.where(mask, 1.36, 0.08)
    case = dict(params=dict(workloads.BASE_PARAMS), rho_a=ra, rho_b=np.where(mask, 0.08, 1.36),
                temp=workloads.conduction_profile(lx, ly), t_bottom=np.ones(lx))
    sim, ora = pair(case, "fp64", 0)
    got, ref = sim.droplets(0.8, labels=True), ora.droplets(0.8)
    assert len(ref["root"]) > 50
    compare(got, ref)


def test_fp32_droplets_small_start():
    """FP32 storage at t = 0: densities are 1.36 / 0.08 up to FP32 rounding,
    far from the threshold, so the partition is the oracle's exactly."""
    sim, ora = pair(workloads.small(), "fp32", 0)
    got, ref = sim.droplets(0.8, labels=True), ora.droplets(0.8)
    np.testing.assert_array_equal(got["label"], ref["label"])
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-5)
    np.testing.assert_allclose(got["y"], ref["y"], atol=1e-5)


def test_full_size_partition_properties():
    w = workloads.large()
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision="fp32")
    sim.step(50)
    d = sim.droplets(0.8, labels=True)
    lab = d["label"]
    bulk = lab >= 0
    n = len(d["root"])
    assert 0.9 * w["n_droplets"] <= n <= 1.1 * w["n_droplets"]
    # adjacent bulk nodes share a label (x periodic)
    right = np.roll(lab, -1, axis=1)
    both = bulk & (right >= 0)
    assert np.all(lab[both] == right[both])
    up = lab[1:, :]
    both = bulk[:-1, :] & (up >= 0)
    assert np.all(lab[:-1, :][both] == up[both])
    # roots: the smallest node of each label, in increasing order
    flat = lab.ravel()
    idx = np.flatnonzero(flat >= 0)
    first = np.full(n, -1, np.int64)
    first[flat[idx[::-1]]] = idx[::-1]
    np.testing.assert_array_equal(first, d["root"])
    assert np.all(np.diff(d["root"]) > 0)
    np.testing.assert_array_equal(np.bincount(flat[idx], minlength=n), d["size"])
    assert np.all((d["x"] >= 0) & (d["x"] < w["lx"])) and np.all(np.isfinite(d["nu"]))


def test_more_droplets_than_the_first_buffer_and_a_tile_table():
    """8192 single-node droplets on 256 x 128: more than the per-droplet
    buffer a handle starts with (4096; the call grows it and repeats the
    sums) and, with 256 droplets in each 64 x 16 tile, more than the LDS
    table of the summing kernel holds (those groups add to global memory
    directly). A second call finds the buffer large enough."""
    lx, ly = 256, 128
    mask = np.zeros((ly, lx), bool)
    mask[::2, ::2] = True
    ra = np.where(mask, 1.36, 0.08)
    case = dict(params=dict(workloads.BASE_PARAMS), rho_a=ra, rho_b=np.where(mask, 0.08, 1.36),
                temp=workloads.conduction_profile(lx, ly), t_bottom=np.ones(lx))
    sim, ora = pair(case, "fp64", 0)
    ref = ora.droplets(0.8)
    assert len(ref["root"]) == 8192
    compare(sim.droplets(0.8, labels=True), ref)
    compare(sim.droplets(0.8, labels=True), ref)
