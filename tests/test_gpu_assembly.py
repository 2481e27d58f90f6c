"""The LDS-tiled assembly (8x8x4 lattice tiles, properties and face fluxes
staged in LDS) against the row-per-lane assembly and against the oracle.

Tolerances: the two GPU kernels sum the same terms in different orders, so
their entries agree to 1e-13 of the largest entry of the same (equation,
variable) column; against the oracle the path's bar of 1e-11 holds (as in
test_gpu_parity).  A face between two tiles is computed by both tiles from
the same staged inputs, so its two copies must be bitwise equal: checked on
two-cell systems whose face crosses a tile boundary in x, y and z, with no
pore volume and no wells, where R_0 = -R_1 and each diagonal block is minus
the other cell's off-diagonal block exactly.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1910_06059_amd import cases
from paper_1910_06059_amd.cases import DAY, PSI, STB, Well

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def opm():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    from paper_1910_06059_amd import opm as _opm
    _opm.init()
    yield _opm
    _opm.lib().opm_set_option(_opm.OPT_ASSEMBLY, 1)


def _colscale(J):
    return np.abs(J.reshape(-1, 9)).max(axis=0) + 1e-300


def _cases():
    wells = lambda nx, ny, nz: [
        Well("I", cases.WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 800 * STB / DAY),
        Well("G", cases.WELL_RATE_INJ, [(nx // 2, ny // 2, 0)], 3e3 * cases.MSCF / DAY,
             phase=cases.GAS),
        Well("P", cases.WELL_BHP_PROD, [(nx - 1, ny - 1, nz - 1)], 3000 * PSI)]
    return {
        "C1": cases.config1(),
        "C2": cases.config2(),
        "ragged_17x9x5": cases.box_case(17, 9, 5, seed=4, wells=wells(17, 9, 5)),
        "masked_19x13x6": cases.box_case(19, 13, 6, seed=6, mask=cases.masked_mask(
            np.random.default_rng(9), (6, 13, 19), 900), wells=[]),
        "line_x": cases.box_case(21, 1, 1, seed=7, wells=[]),
        "column_z": cases.box_case(1, 1, 11, seed=8, wells=[]),
    }


CASES = _cases()


def _assemble(opm, g, y, acc0, dt, kernel):
    opm.lib().opm_set_option(opm.OPT_ASSEMBLY, kernel)
    try:
        R, J, nrm = g.assemble(y, acc0, dt)
    finally:
        opm.lib().opm_set_option(opm.OPT_ASSEMBLY, 1)
    return R.cpu().numpy(), J.cpu().numpy(), nrm.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_tiled_matches_row_kernel_and_oracle(opm, name):
    case = CASES[name]
    print(f"tiled assembly: {name}", flush=True)
    g = opm.GpuModel(case)
    m = oracle.Model(case)
    for seed in (1, 5):
        y = cases.random_state(case, seed=seed)
        y0 = cases.random_state(case, seed=seed + 1)
        dt = 3 * DAY
        acc0 = g.accumulation(g.state(y0))
        Rt, Jt, nt = _assemble(opm, g, g.state(y), acc0, dt, 1)
        Rr, Jr, nr = _assemble(opm, g, g.state(y), acc0, dt, 0)
        rs = np.abs(Rr).max(axis=0) + 1e-300
        assert (np.abs(Rt - Rr) / rs).max() <= 1e-13
        assert (np.abs(Jt - Jr).reshape(-1, 9) / _colscale(Jr)).max() <= 1e-13
        np.testing.assert_allclose(nt[:3], nr[:3], rtol=1e-12, atol=0)
        st, Ro, Jo = m.assemble(y, m.accumulation(y0), dt)
        assert st == 0
        pv = m.geometry()["pore_vol"]
        scale = np.maximum(np.abs(Ro).max(axis=0),
                           (pv[:, None] / dt * np.abs(m.accumulation(y) - m.accumulation(y0))).max(axis=0))
        assert np.all(np.abs(Rt - Ro) <= 1e-11 * scale[None, :])
        assert (np.abs(Jt - Jo).reshape(-1, 9) / _colscale(Jo)).max() <= 1e-11


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_cross_tile_face_bitwise(opm, axis):
    """Cells on either side of a tile boundary (x = 7|8, y = 7|8, z = 3|4)
    alone: the face is computed by both tiles, and the two copies cancel
    exactly."""
    dims = {"x": (9, 1, 1), "y": (1, 9, 1), "z": (1, 1, 5)}[axis]
    nx, ny, nz = dims
    mask = np.zeros((nz, ny, nx), bool)
    lo = {"x": (0, 0, 7), "y": (0, 7, 0), "z": (3, 0, 0)}[axis]
    hi = {"x": (0, 0, 8), "y": (0, 8, 0), "z": (4, 0, 0)}[axis]
    mask[lo] = mask[hi] = True
    case = cases.box_case(nx, ny, nz, seed=2, mask=mask, wells=[], poro=0.0)
    g = opm.GpuModel(case)
    assert g.n == 2 and g.nf == 1
    for seed in range(4):
        y = g.state(cases.random_state(case, seed=seed, p_jitter=300 * PSI))
        R, J, _ = g.assemble(y, g.accumulation(y), DAY)
        R, J = R.cpu().numpy(), J.cpu().numpy()
        assert np.array_equal(R[0], -R[1]) and np.any(R[0] != 0.0)
        # row 0: (diag, (0,1)); row 1: ((1,0), diag)
        assert np.array_equal(J[0], -J[2]) and np.array_equal(J[3], -J[1])
