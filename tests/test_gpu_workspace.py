"""tlb_init_external: the state and step buffers in a device allocation
that torch's caching allocator owns (Simulation(device_memory="torch"))
against the library's own allocations. The same kernels run on the same
values, so every output must be identical."""
import numpy as np
import pytest
import torch

import workloads
from paper_2109_12565_amd import Simulation

from test_gpu_parity import posts_case

pytestmark = pytest.mark.gpu


def make(case, precision, memory):
    return Simulation(case["params"], case["rho_a"], case["rho_b"], case["temp"],
                      solid=case.get("solid"), t_bottom=case.get("t_bottom"),
                      precision=precision, device_memory=memory)


@pytest.mark.parametrize("precision", ["fp32", "fp16dev", "fp64"])
@pytest.mark.parametrize("name", ["small", "posts"])
def test_torch_owned_workspace_matches_library_owned(precision, name):
    case = workloads.small() if name == "small" else posts_case()
    print("workspace:", name, precision, flush=True)
    a, b = make(case, precision, "library"), make(case, precision, "torch")
    assert b._workspace is not None and b._workspace.is_cuda
    for n in (7, 1, 30):
        a.step(n)
        b.step(n)
    assert np.array_equal(a.populations(), b.populations())
    assert a.observables() == b.observables()
    fa, fb = a.fields(), b.fields()
    for k in fa:
        assert np.array_equal(fa[k], fb[k]), k
    da, db = a.droplets(0.8, labels=True), b.droplets(0.8, labels=True)
    for k in da:
        assert np.array_equal(da[k], db[k]), k
    a.close()
    b.close()
    assert b._workspace is None
    # the released memory is torch's again
    x = torch.ones(1 << 20, device="cuda")
    assert float(x.sum()) == float(1 << 20)


def test_torch_owned_workspace_adjoint():
    case = workloads.small()
    a, b = make(case, "fp64", "library"), make(case, "fp64", "torch")
    la, lb = a.forward_taped(40, 10), b.forward_taped(40, 10)
    assert la == lb
    assert np.array_equal(a.adjoint(40), b.adjoint(40))
    a.close()
    b.close()
