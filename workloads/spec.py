"""Plain records describing one thermal simulation request."""
from dataclasses import dataclass, field, replace
from typing import List

FP64 = 0
MIXED = 1

DN = 0
COMPOSITE = 1
ALTERNATE = 2
CONSISTENT = 3

SURFACE = 0
VOLUME = 1


@dataclass
class Mesh:
    """Coarse box [0,lx]x[0,ly]x[0,lz] (metres, z up, laser on z = lz) with
    nx x ny x nz Q1 cells, and the fine window: win_* coarse cells refined
    `refine` times per axis, flush with the top surface."""
    lx: float
    ly: float
    lz: float
    nx: int
    ny: int
    nz: int
    refine: int
    win_nx: int
    win_ny: int
    win_nz: int


@dataclass
class Material:
    """rho [kg/m3]; c(T) and kappa(T) linear on [T_lo, T_hi], constant
    outside; latent heat [J/kg] released by a tanh sigmoid of the given
    sharpness [1/K] centred between T_sol and T_liq; temperatures in K.
    Top-surface heat loss: convection h_conv [W/m2/K] to T_amb on both
    levels, radiation of emissivity `emissivity` on the fine level only (the
    paper's boundary conditions); zero (adiabatic top) by default.
    k_fict [W/m/K] and rhoc_fict [J/m3/K]: the global problem's own constant
    coefficients inside the window in the consistent global formulation
    (coupling CONSISTENT); 0 selects kappa(T_init) and rho c(T_init)."""
    rho: float = 8000.0
    T_lo: float = 300.0
    T_hi: float = 1563.0
    c_lo: float = 450.0
    c_hi: float = 700.0
    k_lo: float = 10.0
    k_hi: float = 30.0
    latent: float = 2.7e5
    T_sol: float = 1563.0
    T_liq: float = 1623.0
    sharpness: float = 0.05
    pc_kind: int = 0
    T_init: float = 300.0
    T_bottom: float = 300.0
    h_conv: float = 0.0
    emissivity: float = 0.0
    T_amb: float = 300.0
    k_fict: float = 0.0
    rhoc_fict: float = 0.0


def default_material(**kw):
    return replace(Material(), **kw)


@dataclass
class Track:
    """Straight laser pass from (x0,y0) to (x1,y1) on the top surface at
    `speed` [m/s], beam power [W], radius [m] and absorptivity; `depth` [m]
    is the penetration depth of the volumetric source model (unused by the
    surface model)."""
    x0: float
    y0: float
    x1: float
    y1: float
    speed: float
    power: float
    radius: float
    absorptivity: float
    depth: float = 0.0


@dataclass
class ScanPath:
    tracks: List[Track]
    t_start: float = 0.0


@dataclass
class Options:
    """Defaults: Newton and two-level tolerances 1e-8 K -- the workloads use
    options_for, 1e-7 K (FP64) or 1e-5 K (mixed) -- and inner CG
    reduction 3e-2 (the Newton fixed point does not depend on it; the
    frozen-kappa Newton contracts by about 0.06 per step, so a tighter inner
    solve buys no fewer Newton steps).

    Macro step dt_coarse [s] split into m_time micro steps; arithmetic of
    the fine linear solves (FP64 or MIXED); Gauss points per face direction
    for the laser load; tolerances (kelvin for Newton and the two-level
    iteration, relative for CG); two-level relaxation theta (<= 0 selects
    refine/(refine+1)); iteration caps; how the two-level correction is
    solved: DN (0), the Dirichlet-Neumann iteration, or COMPOSITE (1, the
    default), one Newton solve on the composite grid with the fine interface
    values slaved to the coarse ones -- the same discrete solution, without
    the outer iteration -- or ALTERNATE (2), the paper's alternate global
    formulation (the global problem over the whole plate without latent
    heat, the local problem driven by it, no feedback), or CONSISTENT (3),
    the paper's consistent global formulation (the global problem over the
    whole plate with constant coefficients of its own inside the window,
    loaded there by the local solution, iterated with the local problem like
    the Dirichlet-Neumann correction); the laser model: SURFACE (0, default), a Gaussian
    flux on the top surface on both levels, or VOLUME (1), the paper's
    volumetric Gaussian on the fine level and a smeared box source on the
    coarse one (tracks along x or y only)."""
    dt_coarse: float
    m_time: int
    precision: int = FP64
    face_quad: int = 3
    newton_tol: float = 1e-8
    cg_rtol: float = 3e-2
    dn_tol: float = 1e-8
    dn_theta: float = 0.0
    newton_max: int = 60
    cg_max: int = 500
    dn_max: int = 60
    coupling: int = 1
    source: int = 0


@dataclass
class Workload:
    name: str
    mesh: Mesh
    material: Material
    scan: ScanPath
    options: Options
    n_macro: int
    meta: dict = field(default_factory=dict)


def options_for(precision, dt_coarse, m_time, **kw):
    """Options with the tolerances suited to the precision: 1e-7 K for the
    FP64 path (target 1e-9 relative, about 3e-7 K on the 300 K plate and
    2e-6 K on a 2000 K field; the frozen-kappa Newton contracts by about
    0.06 per step, so the error left after a last step of 1e-7 K is about
    6e-9 K), 1e-5 K for the mixed path (target 1e-6 relative, i.e. about
    2e-3 K on a 2000 K field: the Newton and two-level stopping errors stay
    two orders below it)."""
    tol = 1e-7 if precision == FP64 else 1e-5
    base = dict(dt_coarse=dt_coarse, m_time=m_time, precision=precision,
                newton_tol=tol, dn_tol=tol)
    base.update(kw)
    return Options(**base)
