"""Seeded synthetic inputs for the three-phase TPFA Newton path.

This module only *describes* reservoir cases: grid shape, cell sizes, rock
(permeability, porosity, active-cell mask), fluid constants, wells, initial
state and report schedule, all converted to SI units.  It holds none of the
discretisation arithmetic: transmissibilities, pore volumes, depths, well
indices, properties and residuals are computed independently by the CPU
oracle (``oracle/``) and by the GPU library from these raw arrays.

Numbering convention: 3-D arrays are shaped ``(nz, ny, nx)`` in C order, so
the flat index ``c = i + nx*(j + ny*k)`` is the natural cell order.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------- units (SI)
PSI = 6894.757293168          # Pa
FT = 0.3048                   # m
MD = 9.869233e-16             # m^2 (millidarcy)
CP = 1.0e-3                   # Pa s
DAY = 86400.0                 # s
LB_FT3 = 16.01846337          # kg/m^3
STB = 0.158987294928          # m^3 (surface barrel)
MSCF = 28.316846592           # m^3 (thousand standard cubic feet)
G = 9.80665                   # m/s^2

# phase / component order used everywhere: water, oil, gas
W, O, GAS = 0, 1, 2

WELL_RATE_INJ = 0   # fixed surface-rate injector of one component
WELL_BHP_PROD = 1   # bottom-hole-pressure controlled producer


@dataclasses.dataclass
class Fluid:
    """Immiscible three-phase fluid and Corey rock-fluid constants (SI)."""
    rho_s: Tuple[float, float, float] = (62.4 * LB_FT3, 53.0 * LB_FT3, 0.06 * LB_FT3)
    c: Tuple[float, float, float] = (3e-6 / PSI, 1e-5 / PSI, 1e-3 / PSI)
    p_ref: float = 14.696 * PSI
    mu: Tuple[float, float, float] = (0.5 * CP, 2.0 * CP, 0.02 * CP)
    swc: float = 0.12
    n_corey: float = 2.0
    g: float = G
    # live oil (gas dissolved in the oil; dry gas): saturated gas-oil ratio
    # r_s(p) = rs_c p, oil swelling b_o / (1 + bo_r r) and thinning
    # mu_o / (1 + muo_r r), switching threshold eps_switch
    live: bool = False
    rs_c: float = 0.0
    bo_r: float = 0.0
    muo_r: float = 0.0
    eps_switch: float = 1e-6
    # wet gas (oil vaporised in the gas, live oil only): saturated oil-gas
    # ratio r_v(p) = rv_c p; 0 = dry gas
    rv_c: float = 0.0


@dataclasses.dataclass
class Well:
    name: str
    kind: int                       # WELL_RATE_INJ or WELL_BHP_PROD
    cells: List[Tuple[int, int, int]]   # perforated (i, j, k) box cells
    target: float                   # surface rate [m^3/s] (injector) or BHP [Pa]
    phase: int = W                  # injected component (injectors only)
    rw: float = 0.25 * FT           # wellbore radius [m]
    # standard wells: the limit of the other control, 0 = none (an injector's
    # maximum BHP [Pa]; a BHP producer's maximum oil surface rate [m^3/s])
    limit: float = 0.0


@dataclasses.dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float                       # m
    dy: float                       # m
    dz: np.ndarray                  # [nz] layer thickness, m
    perm_h: np.ndarray              # [nz,ny,nx] horizontal permeability, m^2
    poro: np.ndarray                # [nz,ny,nx]
    mask: np.ndarray                # [nz,ny,nx] bool, active cells
    kv_kh: float = 0.1
    fluid: Fluid = dataclasses.field(default_factory=Fluid)
    wells: List[Well] = dataclasses.field(default_factory=list)
    p_init: float = 4800.0 * PSI
    sw_init: float = 0.12
    sg_init: float = 0.0
    r_init: Optional[float] = None   # live oil: initial dissolved ratio (x = r_go, no free gas)
    standard_wells: bool = False     # wells with their own unknowns (Q_t, F_w, F_g, p_bhp)
    report_dt: List[float] = dataclasses.field(default_factory=list)   # s
    tol_cnv: float = 1e-8
    tol_mb: float = 1e-11
    lin_rtol: float = 1e-6
    seed: Optional[int] = None

    @property
    def n_box(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_active(self) -> int:
        return int(self.mask.sum())

    def initial_state(self) -> np.ndarray:
        """[n_active, 3] (p, s_w, s_g) in natural order of active cells."""
        n = self.n_active
        y = np.empty((n, 3), dtype=np.float64)
        y[:, 0] = self.p_init
        y[:, 1] = self.sw_init
        y[:, 2] = self.sg_init if self.r_init is None else self.r_init
        return y

    def standard_well_init(self):
        """Wellbore volumes (pi r_w^2 times the perforated thickness) and the
        initial well states [nw][4] = (Q_t, F_w, F_g, p_bhp): no flow (Q_t = 0);
        a producer's wellbore holds oil (F_w = F_g = 0) at its target BHP; an
        injector's holds its injected component at the initial pressure."""
        vol = np.array([math.pi * w.rw ** 2 * sum(float(self.dz[k]) for (_, _, k) in w.cells)
                        for w in self.wells])
        x0 = np.zeros((len(self.wells), 4))
        for n, w in enumerate(self.wells):
            if w.kind == WELL_BHP_PROD:
                x0[n] = (0.0, 0.0, 0.0, w.target)
            else:
                x0[n] = (0.0, 1.0 if w.phase == W else 0.0, 1.0 if w.phase == GAS else 0.0,
                         self.p_init)
        return vol, x0

    def standard_well_limits(self) -> np.ndarray:
        """[nw] limits of the standard wells' other controls (0 = none)."""
        return np.array([float(w.limit) for w in self.wells])

    def initial_meaning(self) -> np.ndarray:
        """[n_active] meaning of the third variable: 0 s_g, 1 r_go (the
        initial state has no free gas when r_init is given)."""
        return np.full(self.n_active, 0 if self.r_init is None else 1, dtype=np.uint8)

    def box_index(self, i: int, j: int, k: int) -> int:
        return i + self.nx * (j + self.ny * k)


# ------------------------------------------------------------ rock helpers
def lognormal_perm(rng: np.random.Generator, shape, median_md, sigma_ln: float) -> np.ndarray:
    """k_h = median * exp(sigma * xi), xi ~ N(0,1) iid per cell (m^2).

    ``median_md`` may be a scalar or an array broadcastable to ``shape``
    (per-layer medians)."""
    xi = rng.standard_normal(shape)
    return np.asarray(median_md, dtype=np.float64) * MD * np.exp(sigma_ln * xi)


def _full_mask(nz, ny, nx):
    return np.ones((nz, ny, nx), dtype=bool)


# ----------------------------------------------------------------- configs
def config1(seed: int = 1) -> Case:
    """10x10x3 gas-injection case (SPE1-shaped grid only), 300 cells."""
    nx, ny, nz = 10, 10, 3
    rng = np.random.default_rng(seed)
    perm = lognormal_perm(rng, (nz, ny, nx), 100.0, 1.0)
    poro = np.full((nz, ny, nx), 0.3)
    wells = [
        Well("INJ", WELL_RATE_INJ, [(0, 0, 0)], 1e5 * MSCF / DAY, phase=GAS),
        Well("PROD", WELL_BHP_PROD, [(9, 9, 2)], 3000.0 * PSI),
    ]
    return Case("C1_10x10x3", nx, ny, nz, 1000 * FT, 1000 * FT,
                np.array([20.0, 30.0, 50.0]) * FT, perm, poro, _full_mask(nz, ny, nx),
                wells=wells, report_dt=[30 * DAY] * 10, seed=seed)


def config2(seed: int = 2) -> Case:
    """24x25x15 waterflood (SPE9-shaped grid only), 9000 cells."""
    nx, ny, nz = 24, 25, 15
    rng = np.random.default_rng(seed)
    layer_median = np.exp(rng.uniform(np.log(10.0), np.log(500.0), size=nz))
    perm = lognormal_perm(rng, (nz, ny, nx), layer_median[:, None, None], 1.5)
    poro = np.full((nz, ny, nx), 0.3)
    wells = [Well("INJ", WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 1e4 * STB / DAY, phase=W)]
    for n, (i, j) in enumerate([(23, 0), (0, 24), (23, 24), (12, 12)]):
        wells.append(Well(f"P{n+1}", WELL_BHP_PROD, [(i, j, 0)], 2000.0 * PSI))
    return Case("C2_24x25x15", nx, ny, nz, 300 * FT, 300 * FT, np.full(nz, 20.0 * FT),
                perm, poro, _full_mask(nz, ny, nx), wells=wells,
                report_dt=[10 * DAY] * 30, seed=seed)


def _largest_component(active: np.ndarray) -> np.ndarray:
    from scipy import ndimage
    structure = ndimage.generate_binary_structure(3, 1)   # 6-connectivity
    lab, nlab = ndimage.label(active, structure=structure)
    if nlab == 0:
        return active
    sizes = np.bincount(lab.ravel())
    sizes[0] = 0
    return lab == int(np.argmax(sizes))


def masked_mask(rng: np.random.Generator, shape, target_active: int) -> np.ndarray:
    """Seeded connected mask: smoothed noise, thresholded so that the largest
    6-connected component holds about ``target_active`` cells."""
    from scipy import ndimage
    xi = rng.standard_normal(shape)
    sm = ndimage.uniform_filter(xi, size=(3, 5, 5), mode="nearest")
    vals = np.sort(sm.ravel())[::-1]
    lo, hi = target_active, min(len(vals) - 1, 3 * target_active)
    best = None
    for _ in range(40):                       # bisection on the threshold rank
        mid = (lo + hi) // 2
        comp = _largest_component(sm >= vals[mid])
        cnt = int(comp.sum())
        if best is None or abs(cnt - target_active) < abs(best[1] - target_active):
            best = (comp, cnt)
        if cnt < target_active:
            lo = mid + 1
        else:
            hi = mid - 1
        if lo > hi or abs(cnt - target_active) <= target_active // 200:
            break
    return best[0]


def config3(seed: int = 3, well_seed: int = 33, target_active: int = 45000) -> Case:
    """46x112x22 masked grid (Norne-shaped box), about 45k active cells."""
    nx, ny, nz = 46, 112, 22
    rng = np.random.default_rng(seed)
    mask = masked_mask(rng, (nz, ny, nx), target_active)
    perm = lognormal_perm(rng, (nz, ny, nx), 200.0, 2.0)
    poro = rng.uniform(0.1, 0.3, size=(nz, ny, nx))
    wr = np.random.default_rng(well_seed)
    half = nz // 2
    wells: List[Well] = []
    lower = mask[half:].any(axis=0)                 # (ny, nx) columns with lower-half cells
    cols = np.argwhere(lower)
    pick = wr.choice(len(cols), size=6, replace=False)
    for n, c in enumerate(pick):
        j, i = cols[c]
        cells = [(int(i), int(j), int(k)) for k in range(half, nz) if mask[k, j, i]]
        wells.append(Well(f"I{n+1}", WELL_RATE_INJ, cells, 5e3 * STB / DAY, phase=W))
    upper = np.argwhere(mask[:half])
    used = set()
    while len(wells) < 18:
        k, j, i = upper[wr.integers(len(upper))]
        key = (int(i), int(j), int(k))
        if key in used:
            continue
        used.add(key)
        wells.append(Well(f"P{len(wells)-5}", WELL_BHP_PROD, [key], 2000.0 * PSI))
    return Case("C3_46x112x22_masked", nx, ny, nz, 300 * FT, 300 * FT, np.full(nz, 20.0 * FT),
                perm, poro, mask, wells=wells, report_dt=[10 * DAY] * 10, seed=seed)


def config4_member(m: int, dims_seed: int = 4000) -> Case:
    """Member m of the 64-member ensemble: uneven grid, gas injection."""
    dr = np.random.default_rng(dims_seed)
    dims = np.stack([dr.integers(20, 61, size=64), dr.integers(20, 61, size=64),
                     dr.integers(20, 31, size=64)], axis=1)
    nx, ny, nz = (int(v) for v in dims[m])
    seed = 1000 + m
    rng = np.random.default_rng(seed)
    perm = lognormal_perm(rng, (nz, ny, nx), 100.0, 1.5)
    poro = np.full((nz, ny, nx), 0.3)
    dz = np.array([[20.0, 30.0, 50.0][k % 3] for k in range(nz)]) * FT
    wells = [
        Well("INJ", WELL_RATE_INJ, [(0, 0, 0)], 1e5 * MSCF / DAY, phase=GAS),
        Well("PROD", WELL_BHP_PROD, [(nx - 1, ny - 1, nz - 1)], 3000.0 * PSI),
    ]
    return Case(f"C4_m{m:02d}_{nx}x{ny}x{nz}", nx, ny, nz, 1000 * FT, 1000 * FT, dz, perm, poro,
                _full_mask(nz, ny, nx), wells=wells, report_dt=[15 * DAY] * 20, seed=seed)


def config5(seed: int = 5008, nx: int = 100, ny: int = 100, nz: int = 50) -> Case:
    """100x100x50 waterflood (500k cells); seeds 5000-5007 train, 5008-5009 test."""
    rng = np.random.default_rng(seed)
    perm = lognormal_perm(rng, (nz, ny, nx), 100.0, 2.0)
    poro = np.full((nz, ny, nx), 0.3)
    wells: List[Well] = []
    fx, fy = nx / 100.0, ny / 100.0
    for n, (i, j) in enumerate([(25, 25), (25, 75), (75, 25), (75, 75)]):
        ii, jj = int(i * fx), int(j * fy)
        wells.append(Well(f"I{n+1}", WELL_RATE_INJ, [(ii, jj, k) for k in range(nz)],
                          5e3 * STB / DAY, phase=W))
    for n, (i, j) in enumerate([(0, 0), (0, 99), (99, 0), (99, 99), (50, 50)]):
        ii, jj = min(int(i * fx), nx - 1), min(int(j * fy), ny - 1)
        wells.append(Well(f"P{n+1}", WELL_BHP_PROD, [(ii, jj, 0)], 2000.0 * PSI))
    return Case(f"C5_{nx}x{ny}x{nz}_s{seed}", nx, ny, nz, 100 * FT, 100 * FT, np.full(nz, 10.0 * FT),
                perm, poro, _full_mask(nz, ny, nx), wells=wells,
                report_dt=[10 * DAY] * 25, seed=seed)


def live_fluid(p_bubble: float = 3000.0 * PSI, r_bubble: float = 5.0) -> Fluid:
    """Live oil whose saturated gas-oil ratio reaches r_bubble (sm3/sm3) at
    the bubble point p_bubble (r_s(p) = r_bubble p / p_bubble); the oil
    swells by 10 % and thins by 25 % at r_bubble."""
    return Fluid(live=True, rs_c=r_bubble / p_bubble, bo_r=0.1 / r_bubble,
                 muo_r=0.25 / r_bubble)


def config_live(seed: int = 6, nx: int = 12, ny: int = 12, nz: int = 5) -> Case:
    """Live-oil depletion with phase appearance (SPE9-like behaviour): oil
    undersaturated at 3600 psi with a bubble point of 3000 psi (r_go = 5
    sm3/sm3 everywhere, no free gas), a water injector in one corner column
    and a producer held at 2500 psi, below the bubble point, in the opposite
    column, so that free gas appears around the producer; 20 steps of 15
    days."""
    rng = np.random.default_rng(seed)
    perm = lognormal_perm(rng, (nz, ny, nx), 100.0, 1.0)
    poro = np.full((nz, ny, nx), 0.25)
    p_b = 3000.0 * PSI
    fluid = live_fluid(p_b, 5.0)
    wells = [
        Well("INJ", WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 300 * STB / DAY, phase=W),
        Well("PROD", WELL_BHP_PROD, [(nx - 1, ny - 1, k) for k in range(nz)], 2500.0 * PSI),
    ]
    return Case(f"C6_live_{nx}x{ny}x{nz}", nx, ny, nz, 300 * FT, 300 * FT, np.full(nz, 20.0 * FT),
                perm, poro, _full_mask(nz, ny, nx), fluid=fluid, wells=wells,
                p_init=3600.0 * PSI, sw_init=0.12, r_init=fluid.rs_c * p_b,
                report_dt=[15 * DAY] * 20, seed=seed)



def config_wet(rv_bubble: float = 0.01) -> Case:
    """Wet-gas variant of the live-oil case: the corner injector puts 2
    MMscf/day of dry gas into the undersaturated oil, whose gas phase holds
    up to r_v(p) = rv_bubble p / 3000 psi of vaporised oil; twelve 30-day
    steps, over which the oil around the injector is vaporised away (cells
    switch to x = r_og)."""
    c = config_live()
    c.name = "C6_wet"
    c.fluid.rv_c = rv_bubble / (3000.0 * PSI)
    c.wells[0].phase = GAS
    c.wells[0].target = 2e6 * 0.0283168 / DAY
    c.report_dt = [30 * DAY] * 12
    return c


def box_case(nx: int, ny: int, nz: int, *, seed: int = 0, dx: float = 300 * FT,
             dy: float = 300 * FT, dz: Sequence[float] | float = 20 * FT,
             median_md: float = 100.0, sigma_ln: float = 1.0, poro: float = 0.3,
             wells: Optional[List[Well]] = None, mask: Optional[np.ndarray] = None,
             report_dt: Optional[List[float]] = None, fluid: Optional[Fluid] = None,
             p_init: float = 4800.0 * PSI, sw_init: float = 0.12, sg_init: float = 0.0,
             r_init: Optional[float] = None, name: Optional[str] = None) -> Case:
    """Small seeded box with configurable wells (tests and smoke runs)."""
    rng = np.random.default_rng(seed)
    perm = lognormal_perm(rng, (nz, ny, nx), median_md, sigma_ln)
    dzv = np.broadcast_to(np.asarray(dz, dtype=np.float64), (nz,)).copy()
    if wells is None:
        wells = [
            Well("INJ", WELL_RATE_INJ, [(0, 0, k) for k in range(nz)], 2e3 * STB / DAY, phase=W),
            Well("PROD", WELL_BHP_PROD, [(nx - 1, ny - 1, 0)], 3000.0 * PSI),
        ]
    if mask is None:
        mask = _full_mask(nz, ny, nx)
    return Case(name or f"box_{nx}x{ny}x{nz}_s{seed}", nx, ny, nz, dx, dy, dzv, perm,
                np.full((nz, ny, nx), poro), mask, fluid=fluid or Fluid(), wells=wells,
                p_init=p_init, sw_init=sw_init, sg_init=sg_init, r_init=r_init,
                report_dt=report_dt if report_dt is not None else [5 * DAY] * 3, seed=seed)


def random_state(case: Case, seed: int, p_jitter: float = 50 * PSI,
                 s_lo: float = 0.17, s_hi: float = 0.6) -> np.ndarray:
    """Seeded random state away from relperm kinks (for Jacobian checks):
    s_w in [s_lo, s_hi], s_g in [s_lo/3, s_hi/2] with s_w + s_g < 0.95."""
    rng = np.random.default_rng(seed)
    n = case.n_active
    y = np.empty((n, 3))
    y[:, 0] = case.p_init + rng.uniform(-p_jitter, p_jitter, n)
    y[:, 1] = rng.uniform(s_lo, s_hi, n)
    y[:, 2] = rng.uniform(s_lo / 3, s_hi / 2, n)
    over = y[:, 1] + y[:, 2] > 0.95
    y[over, 2] = 0.95 - y[over, 1]
    return y


CONFIGS = {"C1": config1, "C2": config2, "C3": config3, "C5": config5}


# ---------------------------------------------- learned-guess network inputs
GUESS_CH = 16
GUESS_LAYER_W = 27 * GUESS_CH * GUESS_CH
GUESS_LAYER = GUESS_LAYER_W + GUESS_CH
GUESS_PARAMS = 3 * GUESS_LAYER


def guess_init_params(seed: int = 0, last_scale: float = 0.01) -> np.ndarray:
    """Seeded starting parameters of the 3-layer 3x3x3 guess network (FP32
    [W_l[27][16 out][16 in], b_l[16]] for l = 0, 1, 2): He-normal weights
    (std sqrt(2 / fan_in), fan_in = 27 * 16), zero biases, the last layer
    scaled by last_scale so that the first corrections stay near zero."""
    rng = np.random.default_rng(seed)
    std = math.sqrt(2.0 / (27 * GUESS_CH))
    p = np.zeros(GUESS_PARAMS, dtype=np.float64)
    for l in range(3):
        w = rng.standard_normal(GUESS_LAYER_W) * std * (last_scale if l == 2 else 1.0)
        p[l * GUESS_LAYER:l * GUESS_LAYER + GUESS_LAYER_W] = w
    return p.astype(np.float32)


def guess_random_feats(shape, seed: int, active=None, channels: int = 11) -> np.ndarray:
    """Seeded BF16-representable layer inputs [nz, ny, nx, 16] (float32) for
    layer-level tests: standard normal in the first `channels` channels of
    active box cells, zero elsewhere."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    x = np.zeros((nz, ny, nx, GUESS_CH), dtype=np.float32)
    v = rng.standard_normal((nz, ny, nx, channels)).astype(np.float32)
    v = (v.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)   # exact in BF16
    x[..., :channels] = v
    if active is not None:
        x[~np.asarray(active, dtype=bool)] = 0.0
    return x
