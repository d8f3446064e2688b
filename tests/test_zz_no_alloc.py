"""tlb_droplets_noalloc (static device workspace, no allocation) against
tlb_droplets on the same handle: two calls in a row, the second on a smaller
lattice, so the workspace holds the first call's contents when the second
starts. Both entry points run the same kernels, so every output must be
identical: labels, roots and sizes (integers), and mass, centre and droplet
Nusselt number (exact fixed-point sums and the same FP64 arithmetic)."""
import numpy as np
import pytest

import workloads
from paper_2109_12565_amd import Simulation
from paper_2109_12565_amd._lib import TLB_EINVAL, TlbError

pytestmark = pytest.mark.gpu


def run(w, precision, steps):
    sim = Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                     t_bottom=w["t_bottom"], precision=precision)
    sim.step(steps)
    return sim


def same(a, b):
    assert len(a["root"]) == len(b["root"])
    for k in ("label", "root", "size", "mass", "x", "y", "nu"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_noalloc_droplets_equal_allocating_ones_on_two_calls():
    # first call: the 1024 x 512 emulsion, the largest lattice the workspace takes
    print("noalloc: mid 1024x512 fp32, 30 steps", flush=True)
    big = run(workloads.mid(), "fp32", 30)
    want = big.droplets(0.8, labels=True)
    got = big.droplets(0.8, labels=True, noalloc=True)
    assert len(want["root"]) > 800
    same(got, want)
    big.close()
    # second call: a smaller lattice with posts, after the larger one
    print("noalloc: small 128x64 fp64 with posts, 40 steps", flush=True)
    from test_gpu_parity import posts_case
    c = posts_case()
    small = Simulation(c["params"], c["rho_a"], c["rho_b"], c["temp"], solid=c["solid"],
                       t_bottom=c["t_bottom"], precision="fp64")
    small.step(40)
    want = small.droplets(0.8, labels=True)
    got = small.droplets(0.8, labels=True, noalloc=True)
    assert len(want["root"]) > 0
    same(got, want)
    # and once more, in the other order (the workspace now holds this call)
    same(small.droplets(0.8, labels=True, noalloc=True), small.droplets(0.8, labels=True))
    small.close()


def test_noalloc_rejects_a_lattice_beyond_the_workspace():
    w = workloads.large()
    print("noalloc: large 4096x2048 fp32 rejected", flush=True)
    with Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], solid=w["solid"],
                    t_bottom=w["t_bottom"], precision="fp32") as sim:
        with pytest.raises(TlbError) as e:
            sim.droplets(0.8, noalloc=True)
        assert e.value.code == TLB_EINVAL
        assert "static workspace" in str(e.value)


def test_noalloc_reports_more_droplets_than_the_workspace():
    """131 072 single-node droplets on 1024 x 512 (the workspace holds 16 384):
    the no-allocation call numbers them all but sums only those it has room
    for, then reports TLB_EINVAL; the allocating call on the same handle grows
    its buffer and returns them all."""
    lx, ly = 1024, 512
    mask = np.zeros((ly, lx), bool)
    mask[::2, ::2] = True
    print("noalloc: 1024x512 with 131072 single-node droplets", flush=True)
    with Simulation(dict(workloads.BASE_PARAMS), np.where(mask, 1.36, 0.08),
                    np.where(mask, 0.08, 1.36), workloads.conduction_profile(lx, ly),
                    t_bottom=np.ones(lx), precision="fp32") as sim:
        with pytest.raises(TlbError) as e:
            sim.droplets(0.8, noalloc=True)
        assert e.value.code == TLB_EINVAL and "workspace" in str(e.value)
        d = sim.droplets(0.8, labels=True)
        assert len(d["root"]) == 131072
        assert np.all(d["size"] == 1)
        np.testing.assert_array_equal(d["label"][mask], np.arange(131072))
        assert np.all(d["label"][~mask] == -1)


def test_no_droplets():
    """A threshold above every density: no droplet, every label -1, on both
    entry points."""
    w = workloads.small()
    print("noalloc: small 128x64, threshold above every density", flush=True)
    with Simulation(w["params"], w["rho_a"], w["rho_b"], w["temp"], t_bottom=w["t_bottom"],
                    precision="fp32") as sim:
        for noalloc in (False, True):
            d = sim.droplets(10.0, labels=True, noalloc=noalloc)
            assert len(d["root"]) == 0
            assert np.all(d["label"] == -1)
