"""Seeded, synthetic inputs for the sputtered-atom transport and the composition map.

This module only *describes* sputter systems: a vacuum chamber with its gas, one or
more magnetron cathodes, and a substrate with a tally grid (the object model of the
paper's wrapper, Methods, "The SIMTRA Python wrapper": chamber, magnetron, dummy
objects).  It holds none of the method's arithmetic: no sampling, no transport, no
normalisation.  Both the HIP path (through its Python binding) and the FP64 oracle
read these plain objects, each converting them to its own layout.

Units: mm, eV, u (atomic mass units), K, Pa.  Directions are unit vectors in the
chamber frame (cylinder axis = z).

The paper's chamber geometry is confidential (Methods, "Setup of the sputter
system"), so the workloads below are synthetic stand-ins of the same kind: planar
50.8 mm targets with a racetrack, a parallel substrate or a 10 cm wafer, four
confocal tilted cathodes (Ni, Pd, Pt, Ru) in Ar at 0.5 Pa.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

Vec3 = Tuple[float, float, float]

# Species used by the paper's quaternary Ni-Pd-Pt-Ru system (Methods, "Setup of the
# sputter system").  Surface binding energies U_s [eV], atomic masses [u], atomic
# numbers, and nominal bulk densities [g/cm^3] (handbook values; the paper converts
# arrival fractions with bulk density and atomic mass but does not print them).
SPECIES = {
    "Ni": dict(U_s=4.44, mass=58.69, Z=28, density=8.908),
    "Pd": dict(U_s=3.89, mass=106.42, Z=46, density=12.02),
    "Pt": dict(U_s=5.84, mass=195.08, Z=78, density=21.45),
    "Ru": dict(U_s=6.74, mass=101.07, Z=44, density=12.45),
}
AR_MASS = 39.95
AR_Z = 18


@dataclass
class Chamber:
    """Absorbing cylindrical chamber on the z axis filled with a homogeneous gas."""
    radius: float = 200.0
    z_lo: float = 0.0
    z_hi: float = 300.0
    pressure: float = 0.5          # Pa
    T: float = 300.0               # K
    gas_mass: float = AR_MASS      # u
    gas_Z: int = AR_Z
    gas_motion: int = 1            # 1: thermal motion of the gas partner is sampled


@dataclass
class Grid:
    """Collecting substrate (a "dummy" object) carrying the tally grid.

    ``normal`` faces the cathodes.  Bins are row-major [iv][iu] over
    [-half_u, half_u] x [-half_v, half_v] along u_axis and v = normal x u_axis.
    shape 0 = rectangle, 1 = disc of radius half_u.
    """
    center: Vec3 = (0.0, 0.0, 200.0)
    normal: Vec3 = (0.0, 0.0, -1.0)
    u_axis: Vec3 = (1.0, 0.0, 0.0)
    half_u: float = 50.0
    half_v: float = 50.0
    shape: int = 0
    nu: int = 50
    nv: int = 50


@dataclass
class Cathode:
    """Planar circular magnetron target; ``normal`` points into the gas."""
    element: str = "Ni"
    center: Vec3 = (0.0, 0.0, 100.0)
    normal: Vec3 = (0.0, 0.0, 1.0)
    u_axis: Vec3 = (1.0, 0.0, 0.0)
    radius: float = 25.4
    rt_mu: float = 15.0            # racetrack radius: normal(mu, sigma) truncated to [lo, hi]
    rt_sigma: float = 3.0
    rt_lo: float = 0.0
    rt_hi: float = 25.4
    U_s: float = 4.44
    E_i: float = 400.0             # incident ion energy, eV
    k_cut: float = 1.0             # E_max = k * Lambda * E_i - U_s
    mass: float = 58.69
    Z: int = 28
    cos_coeff: Tuple[float, ...] = (0.0, 1.0, 0.0, 0.0, 0.0, 0.0)   # emission law sum c_i cos^i
    n_particles: int = 100_000
    # measured racetrack: radial erosion-depth profile [(r mm, depth), ...] from r = 0, radii
    # increasing; None = the truncated normal above
    rt_profile: Optional[Sequence[Tuple[float, float]]] = None


@dataclass
class Absorber:
    """An absorbing "dummy" object (mask, shutter, chimney).  kind "disc" (radius half_u),
    "rect" (half sizes half_u x half_v along u_axis and normal x u_axis) or "tube" (an open
    cylinder: axis from center along normal, radius half_u, length).  Both faces absorb."""
    kind: str = "disc"
    center: Vec3 = (0.0, 0.0, 150.0)
    normal: Vec3 = (0.0, 0.0, 1.0)
    u_axis: Vec3 = (1.0, 0.0, 0.0)
    half_u: float = 10.0
    half_v: float = 10.0
    length: float = 0.0


@dataclass
class Config:
    chamber: Chamber
    grid: Grid
    cathodes: List[Cathode]
    absorbers: List[Absorber] = field(default_factory=list)
    cross_absorb: bool = False     # the other targets of the configuration absorb too


@dataclass
class Params:
    theta_min: float = 0.1         # rad; CM angle at the cross-section cut-off impact parameter
    E_th_kT: float = 3.0           # thermalisation threshold in units of k_B T
    event_cap: int = 1 << 20       # flights per particle before it is counted ESCAPED
    table_ne: int = 256            # log10(eps) nodes of the scattering table
    table_ns: int = 257            # b/b_max nodes
    log_eps_lo: float = -10.0
    log_eps_hi: float = 0.0


def species_cathode(element: str, **kw) -> Cathode:
    s = SPECIES[element]
    return Cathode(element=element, U_s=s["U_s"], mass=s["mass"], Z=s["Z"], **kw)


# ---------------------------------------------------------------------------
# Single planar Ni target facing a parallel 100 x 100 mm substrate 100 mm away.
# ---------------------------------------------------------------------------
def single_ni(pressure: float = 0.5, n_particles: int = 100_000, gas_motion: int = 1,
              nu: int = 50, nv: int = 50) -> Config:
    return Config(
        chamber=Chamber(pressure=pressure, gas_motion=gas_motion),
        grid=Grid(nu=nu, nv=nv),
        cathodes=[species_cathode("Ni", n_particles=n_particles)],
    )


def single_ni_legs(n_particles: int = 10_000_000) -> List[Config]:
    """The three chambers of the single-target batch: 0.5 Pa, 0 Pa and 2 Pa."""
    return [single_ni(0.5, n_particles), single_ni(0.0, n_particles), single_ni(2.0, n_particles)]


# ---------------------------------------------------------------------------
# Measured-racetrack and emission-law inputs.
# ---------------------------------------------------------------------------
# An emission law with an under-cosine (heart-shaped) polar distribution, sum c_i cos^i theta,
# non-negative on [0, 90 deg]: the kind of six-coefficient law the model accepts besides the
# plain cosine.
UNDER_COSINE = (0.1, 0.5, 1.0, -0.6, 0.0, 0.0)


def measured_racetrack(seed: int = 0, radius: float = 25.4, step: float = 0.5,
                       depth: float = 1.8) -> List[Tuple[float, float]]:
    """A synthetic profilometry scan of an eroded target along its diameter, folded into a
    radial erosion-depth profile (the racetrack is taken as axisymmetric).  The scan has the
    main groove at r = 15 mm (sd 3 mm), a shallow inner groove at r = 6 mm and seeded
    measurement noise; negative readings are clipped to zero.  Returns [(r, depth)] from
    r = 0 to the target radius."""
    rng = np.random.default_rng(seed)
    K = int(math.floor(radius / step + 1e-9))
    xs = np.concatenate([[-radius], step * np.arange(-K, K + 1), [radius]])
    r = np.abs(xs)
    prof = depth * (np.exp(-(r - 15.0) ** 2 / (2 * 3.0 ** 2)) + 0.12 * np.exp(-(r - 6.0) ** 2 / (2 * 2.0 ** 2)))
    scan = np.clip(prof + rng.normal(0.0, 0.02 * depth, size=xs.size), 0.0, None)
    # fold: mean of the readings at -r and +r
    nodes = np.unique(np.round(r, 9))
    out = []
    for rk in nodes:
        out.append((float(rk), float(scan[np.isclose(r, rk)].mean())))
    return out


def with_launch(cfg: Config, rt_profile=None, cos_coeff=None) -> Config:
    """Copy of cfg whose cathodes use the given racetrack profile and/or emission law."""
    cats = [replace(c, rt_profile=rt_profile if rt_profile is not None else c.rt_profile,
                    cos_coeff=tuple(cos_coeff) if cos_coeff is not None else c.cos_coeff)
            for c in cfg.cathodes]
    return replace(cfg, cathodes=cats)


def with_chimneys(cfg: Config, length: float = 30.0, gap: float = 5.0, cross_absorb: bool = True) -> Config:
    """Copy of cfg with an open chimney around each target (coaxial tube of radius
    target radius + gap from the target plane along its normal, ``length`` mm long), keeping
    the configuration's other absorbers; with cross_absorb the other targets absorb too."""
    tubes = [Absorber("tube", center=c.center, normal=c.normal, u_axis=c.u_axis, half_u=c.radius + gap,
                      half_v=c.radius + gap, length=length) for c in cfg.cathodes]
    return replace(cfg, absorbers=list(cfg.absorbers) + tubes, cross_absorb=cross_absorb)


# ---------------------------------------------------------------------------
# Four confocal cathodes (Ni, Pd, Pt, Ru) around a 100 mm wafer.
# ---------------------------------------------------------------------------
QUAT_ELEMENTS = ("Ni", "Pd", "Pt", "Ru")
QUAT_POWERS = (50.0, 10.0, 35.0, 20.0)      # W; particles per cathode = 2e5 * P
WAFER_Z = 280.0


def _confocal_cathode(element: str, k: int, tilt_deg: float, distance: float,
                      n_particles: int) -> Cathode:
    """Cathode k at azimuth 90 deg * k, tilted by ``tilt_deg`` toward the wafer
    centre, its centre ``distance`` mm from the wafer centre along its normal."""
    tau = math.radians(tilt_deg)
    phi = math.radians(90.0 * k)
    n = (-math.sin(tau) * math.cos(phi), -math.sin(tau) * math.sin(phi), math.cos(tau))
    c = (-distance * n[0], -distance * n[1], WAFER_Z - distance * n[2])
    zx = (-n[1], n[0], 0.0)                       # z_hat x n
    norm = math.hypot(zx[0], zx[1])
    u = (1.0, 0.0, 0.0) if norm < 1e-12 else (zx[0] / norm, zx[1] / norm, 0.0)
    return species_cathode(element, center=c, normal=n, u_axis=u, n_particles=n_particles)


def quaternary(pressure: float = 0.5, tilt_deg: float = 25.0, distance: float = 150.0,
               counts: Sequence[int] = None, grid_n: int = 200) -> Config:
    if counts is None:
        counts = [int(2e5 * p) for p in QUAT_POWERS]
    cats = [_confocal_cathode(el, k, tilt_deg, distance, int(n))
            for k, (el, n) in enumerate(zip(QUAT_ELEMENTS, counts))]
    grid = Grid(center=(0.0, 0.0, WAFER_Z), normal=(0.0, 0.0, -1.0), u_axis=(1.0, 0.0, 0.0),
                half_u=50.0, half_v=50.0, shape=1, nu=grid_n, nv=grid_n)
    return Config(chamber=Chamber(pressure=pressure), grid=grid, cathodes=cats)


def quaternary_sweep(n_configs: int = 64, seed: int = 0, scale: float = 1.0) -> List[Config]:
    """Batched sweep of the four-cathode design.  Per config, drawn in this order
    from numpy's default_rng(seed): pressure U(0.1, 2) Pa, tilt U(0, 40) deg,
    distance U(80, 200) mm, particle count 10**U(5, 7); the count is split over
    the cathodes in proportion to QUAT_POWERS.  ``scale`` multiplies the counts
    (test-sized sweeps keep the same geometry)."""
    rng = np.random.default_rng(seed)
    out = []
    tot = sum(QUAT_POWERS)
    for _ in range(n_configs):
        p = float(rng.uniform(0.1, 2.0))
        tau = float(rng.uniform(0.0, 40.0))
        d = float(rng.uniform(80.0, 200.0))
        n_cfg = 10.0 ** float(rng.uniform(5.0, 7.0))
        counts = [max(1, int(round(scale * n_cfg * pw / tot))) for pw in QUAT_POWERS]
        out.append(quaternary(p, tau, d, counts))
    return out


# ---------------------------------------------------------------------------
# Ternary Pd-Pt-Ru library and a sweep of the common cathode tilt (Results, the
# cathode-tilt study).  The three cathodes take positions 1-3 of the four-cathode
# ring; 200 mm keeps 50.8 mm targets clear of each other at tilts near 12 deg.
# ---------------------------------------------------------------------------
TERNARY_ELEMENTS = ("Pd", "Pt", "Ru")
TERNARY_POWERS = (40.0, 18.0, 35.0)          # W, the Pd-Pt-Ru library of Table 1 (Pd on RF)
# Sputter rate = a P + b (nm/s per W, nm/s): the lines through the two calibration samples of
# Table S1 for each element and supply (Pd RF 7 / 60 W, Pt DC 5 / 35 W, Ru DC 5 / 35 W).
TERNARY_RATE_A = (0.0013669622641509437, 0.003086333333333334, 0.0014952666666666666)
TERNARY_RATE_B = (-0.004707735849056604, -0.001321666666666701, -0.002054333333333349)
TERNARY_DISTANCE = 200.0


def ternary(pressure: float = 0.5, tilt_deg: float = 12.2, distance: float = TERNARY_DISTANCE,
            n_particles: int = 1_000_000, grid_n: int = 200) -> Config:
    """Pd, Pt, Ru on confocal cathodes 1-3 (azimuths 90, 180, 270 deg), each launching
    ``n_particles``, onto the 100 mm wafer."""
    cats = [_confocal_cathode(el, k + 1, tilt_deg, distance, int(n_particles))
            for k, el in enumerate(TERNARY_ELEMENTS)]
    grid = Grid(center=(0.0, 0.0, WAFER_Z), normal=(0.0, 0.0, -1.0), u_axis=(1.0, 0.0, 0.0),
                half_u=50.0, half_v=50.0, shape=1, nu=grid_n, nv=grid_n)
    return Config(chamber=Chamber(pressure=pressure), grid=grid, cathodes=cats)


def tilt_sweep(tilts: Sequence[float], pressure: float = 0.5, distance: float = TERNARY_DISTANCE,
               n_particles: int = 1_000_000) -> List[Config]:
    """One ternary configuration per tilt (the sweep of one launch)."""
    return [ternary(pressure, float(t), distance, n_particles) for t in tilts]


def ternary_composition_inputs():
    """(a, b, P, M, rho) of the ternary library, float64 arrays of 3."""
    M = np.array([SPECIES[e]["mass"] for e in TERNARY_ELEMENTS])
    rho = np.array([SPECIES[e]["density"] for e in TERNARY_ELEMENTS])
    return (np.array(TERNARY_RATE_A), np.array(TERNARY_RATE_B), np.array(TERNARY_POWERS), M, rho)


# ---------------------------------------------------------------------------
# Composition-map inputs: linear power-rate model and a batch of power vectors.
# ---------------------------------------------------------------------------
@dataclass
class CompositionInputs:
    a: np.ndarray          # [K] rate slope per W
    b: np.ndarray          # [K] rate offset
    P: np.ndarray          # [B, K] powers, W
    M: np.ndarray          # [K] atomic masses, u
    rho: np.ndarray        # [K] bulk densities, g/cm^3


def composition_inputs(batch: int = 1024, elements: Sequence[str] = QUAT_ELEMENTS
                       ) -> CompositionInputs:
    K = len(elements)
    r1 = np.random.default_rng(1)
    a = r1.uniform(0.5, 2.0, K)
    b = r1.uniform(0.0, 0.2, K)
    P = np.random.default_rng(2).uniform(20.0, 200.0, (batch, K))
    M = np.array([SPECIES[e]["mass"] for e in elements])
    rho = np.array([SPECIES[e]["density"] for e in elements])
    return CompositionInputs(a=a, b=b, P=P, M=M, rho=rho)


def total_particles(cfgs: Sequence[Config]) -> int:
    return sum(c.n_particles for cfg in cfgs for c in cfg.cathodes)


def with_counts(cfg: Config, n: int) -> Config:
    """Copy of ``cfg`` with every cathode launching ``n`` particles."""
    return replace(cfg, cathodes=[replace(c, n_particles=n) for c in cfg.cathodes])
