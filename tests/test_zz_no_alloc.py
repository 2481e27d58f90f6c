"""The allocation-free assembly entry point (opm_assemble_noalloc) against
opm_assemble, through the C ABI.

Both run the same kernels on the same inputs, so R, J and the 8 norms must
be bitwise equal.  Two calls in a row, the second on a smaller problem (its
partials overwrite only the first workgroups' slots of the shared scratch
array, and the final reduction must read only those), then a problem above
the array's limit, which must be refused before any device work.
"""
import ctypes

import pytest
import torch

from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    return _opm


def _both(opm, case, seed):
    g = opm.GpuModel(case)
    y = g.state(cases.random_state(case, seed=seed))
    acc0 = g.accumulation(g.state(cases.random_state(case, seed=seed + 1)))
    dt = 5 * DAY
    R, J, nrm = g.assemble(y, acc0, dt)
    R2 = torch.full_like(R, float("nan"))
    J2 = torch.full_like(J, float("nan"))
    n2 = torch.full((8,), float("nan"), dtype=torch.float64, device=R.device)
    st = g.assemble_noalloc(y, acc0, dt, R2, J2, n2)
    torch.cuda.synchronize()
    assert st == opm.OK, opm._strerror(st)
    return g, (R, J, nrm), (R2, J2, n2)


def test_no_alloc_assembly_two_calls(opm):
    # 9000 cells (36 workgroups of partials), then 120 cells (one)
    for case, seed in [(cases.config2(), 11), (cases.box_case(6, 5, 4, seed=3), 21)]:
        print(f"no-alloc assembly: {case.name} ({case.n_active} cells)", flush=True)
        g, (R, J, nrm), (R2, J2, n2) = _both(opm, case, seed)
        assert torch.equal(R, R2)
        assert torch.equal(J, J2)
        assert torch.equal(nrm, n2)
    # residual only and no norms: the other outputs stay untouched
    R3 = torch.zeros_like(R)
    y = g.state(cases.random_state(g.case, seed=21))
    acc0 = g.accumulation(g.state(cases.random_state(g.case, seed=22)))
    assert g.assemble_noalloc(y, acc0, 5 * DAY, R3, None, None) == opm.OK
    torch.cuda.synchronize()
    assert torch.equal(R3, R)


def test_no_alloc_assembly_size_limit(opm):
    g = opm.GpuModel(cases.box_case(4, 3, 2, seed=1))
    pb = type(g.pb)()
    ctypes.memmove(ctypes.byref(pb), ctypes.byref(g.pb), ctypes.sizeof(pb))
    pb.n_cells = 16777216 + 1
    y = g.initial_state()
    st = opm.lib().opm_assemble_noalloc(ctypes.byref(pb), opm._ptr(y), opm._ptr(y), DAY,
                                        opm._ptr(y), None, None, opm._stream())
    assert st == opm.EINVAL
