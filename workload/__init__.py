"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds workload descriptions and random draws only: mesh sizes,
subdomain cuts, physical parameters, the stimulus indicator and the initial
perturbation.  It contains none of the solver's arithmetic, so that both the
oracle and the device path can consume the same inputs without sharing any
of the method's code.

Unit system (cm, ms, mV, uA/cm^3): conductivities in mS/cm, chi*C_m in
uF/cm^3, the ionic current per unit volume is chi times the Rogers-McCulloch
current with G and eta_1 in mS/cm^2.  Parameter values follow the paper's
table of physiological coefficients (Sec. 6); the conductivities are that
table's values in mS/cm.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Physics:
    sigma_i: tuple = (3.0, 0.31525, 0.031525)      # l, t, n  (mS/cm)
    sigma_e: tuple = (2.0, 1.3514, 0.6757)         # l, t, n  (mS/cm)
    theta0: float = 0.0                             # fibre angle at z = 0 (rad)
    theta1: float = 2.0 * math.pi / 3.0             # fibre angle at z = L_z (rad)
    chi: float = 1000.0                             # 1/cm
    Cm: float = 1.0                                 # uF/cm^2
    G: float = 1.2                                  # mS/cm^2
    eta1: float = 4.4                               # mS/cm^2
    eta2: float = 0.012                             # 1/ms
    vth: float = 13.0                               # mV
    vp: float = 100.0                               # mV


@dataclasses.dataclass(frozen=True)
class Mesh:
    """nx x ny x nz box elements of size h x hy x hz (hy, hz <= 0: equal to
    h, i.e. cubes of side h) and the tensor partition's cut positions.

    A non-empty ``ellipsoid`` (a1, a2, b1, b2, c1, c2, theta_min, theta_max,
    phi_min, phi_max) maps the same logical grid onto a truncated ellipsoid
    instead (x along phi, y along theta, z along the depth r); h, hy, hz are
    then unused."""
    nx: int
    ny: int
    nz: int
    h: float
    cuts_x: tuple
    cuts_y: tuple
    cuts_z: tuple
    hy: float = 0.0
    hz: float = 0.0
    ellipsoid: tuple = ()

    @property
    def spacing(self) -> tuple:
        """Element sizes (hx, hy, hz)."""
        return (self.h, self.hy if self.hy > 0 else self.h, self.hz if self.hz > 0 else self.h)

    @property
    def nnodes(self) -> int:
        return (self.nx + 1) * (self.ny + 1) * (self.nz + 1)

    @property
    def nsub(self) -> int:
        return (len(self.cuts_x) - 1) * (len(self.cuts_y) - 1) * (len(self.cuts_z) - 1)


@dataclasses.dataclass(frozen=True)
class Solver:
    dt: float = 0.05
    newton_rtol: float = 1e-8
    newton_atol: float = 0.0
    newton_maxit: int = 20
    krylov_rtol: float = 1e-10
    krylov_maxit: int = 500
    krylov_dtol: float = 1e4


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    mesh: Mesh
    physics: Physics
    solver: Solver
    stim_amplitude: float          # uA/cm^3
    stim_block: tuple              # elements (bx, by, bz) from the origin corner
    stim_steps: int                # number of steps carrying the stimulus
    steps: int
    perturb_seed: int | None       # seed of the +/-1% initial v perturbation (None: rest)


def uniform_cuts(n: int, parts: int) -> tuple:
    if n % parts:
        raise ValueError(f"{n} elements do not split into {parts} equal parts")
    w = n // parts
    return tuple(range(0, n + 1, w))


def uneven_cuts(n: int, parts: int, widths: Sequence[int], seed: int) -> tuple:
    """Cut positions with per-part widths drawn from ``widths`` and rejection
    resampled until they sum to ``n`` (tensor partition, conforming faces)."""
    rng = np.random.default_rng(seed)
    widths = np.asarray(widths)
    for _ in range(100000):
        w = rng.choice(widths, size=parts)
        if int(w.sum()) == n:
            return tuple(int(c) for c in np.concatenate([[0], np.cumsum(w)]))
    raise RuntimeError("could not draw widths summing to n")


def box_mesh(nx, ny, nz, h, px, py, pz) -> Mesh:
    return Mesh(nx, ny, nz, h, uniform_cuts(nx, px), uniform_cuts(ny, py), uniform_cuts(nz, pz))


def stimulus_nodal(mesh: Mesh, block: tuple, amplitude: float, origin=(0, 0, 0)) -> np.ndarray:
    """Nodal stimulus I_s: ``amplitude`` on every node of the element block
    [origin, origin + block) (closed node range), zero elsewhere."""
    nx1, ny1 = mesh.nx + 1, mesh.ny + 1
    out = np.zeros(mesh.nnodes)
    ox, oy, oz = origin
    bx, by, bz = block
    for k in range(oz, oz + bz + 1):
        for j in range(oy, oy + by + 1):
            for i in range(ox, ox + bx + 1):
                out[i + nx1 * (j + ny1 * k)] = amplitude
    return out


def stimulus_sites(mesh: Mesh, n: int, seed: int, block=(2, 2, 2)) -> list:
    """``n`` element-block origins drawn uniformly (seeded) so that the block
    lies inside the mesh."""
    rng = np.random.default_rng(seed)
    hi = (mesh.nx - block[0], mesh.ny - block[1], mesh.nz - block[2])
    return [tuple(int(rng.integers(0, h + 1)) for h in hi) for _ in range(n)]


def initial_state(mesh: Mesh, physics: Physics, seed: int | None):
    """Resting state, optionally with an additive v perturbation of
    0.01 * v_p * U(-1, 1) per node (i.i.d., seeded)."""
    n = mesh.nnodes
    v = np.zeros(n)
    if seed is not None:
        rng = np.random.default_rng(seed)
        v = 0.01 * physics.vp * rng.uniform(-1.0, 1.0, size=n)
    ue = np.zeros(n)
    w = np.zeros(n)
    return v, ue, w


def random_field(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    return scale * np.random.default_rng(seed).standard_normal(n)


PAPER_STIM = 1.0e5     # 100 mA/cm^3 expressed in uA/cm^3


def workload(name: str) -> Workload:
    """Named workloads: the parity-size slab (8^3, 2x2x2), the 32^3 slab in
    4x4x4 subdomains, the 128x128x64 slab with uneven cuts, the
    256x256x128 slab in 32x32x16 subdomains (about 17.04M dofs), and the
    128x128x64 truncated ellipsoid in 8x8x4 subdomains (2,163,330 dofs)."""
    ph = Physics()
    if name == "slab8":
        m = box_mesh(8, 8, 8, 0.01, 2, 2, 2)
        return Workload(name, m, ph, Solver(), 250.0, (2, 2, 2), 20, 5, None)
    if name == "slab8_supra":
        m = box_mesh(8, 8, 8, 0.01, 2, 2, 2)
        return Workload(name, m, ph, Solver(), PAPER_STIM, (2, 2, 2), 20, 5, None)
    if name == "slab32":
        m = box_mesh(32, 32, 32, 0.01, 4, 4, 4)
        return Workload(name, m, ph, Solver(), PAPER_STIM, (2, 2, 2), 20, 40, 1)
    if name == "slab128_uneven":
        m = Mesh(128, 128, 64, 0.01,
                 uneven_cuts(128, 16, range(6, 11), 2),
                 uneven_cuts(128, 16, range(6, 11), 3),
                 uneven_cuts(64, 8, range(6, 11), 4))
        return Workload(name, m, ph, Solver(), PAPER_STIM, (2, 2, 2), 20, 20, 1)
    if name == "slab256":
        m = box_mesh(256, 256, 128, 0.01, 32, 32, 16)
        return Workload(name, m, ph, Solver(), PAPER_STIM, (2, 2, 2), 20, 50, None)
    if name == "ellipsoid128":
        return dataclasses.replace(ellipsoid_workload((8, 8, 4)), name=name)
    raise KeyError(name)


TEST3_SIDE = 0.32   # cm: 4 subdomains of H/h elements per axis, h = 0.01 cm at H/h = 8


def test3(Hh: int, steps: int = 40) -> Workload:
    """Slab of the optimality test (Sec. 6, Test 3): 4 x 4 x 4 subdomains of
    H/h elements per axis in a cube of fixed side, so h = side / (4 H/h);
    the stimulus covers a corner cube of side / 8 (H/h / 2 elements per axis)
    for the first 20 steps, and the run covers 2 ms of activation (40 steps
    of 0.05 ms) by default.  H/h must be even."""
    if Hh < 2 or Hh % 2:
        raise ValueError("H/h must be even and >= 2")
    m = box_mesh(4 * Hh, 4 * Hh, 4 * Hh, TEST3_SIDE / (4 * Hh), 4, 4, 4)
    return Workload(f"test3_Hh{Hh}", m, Physics(), Solver(), PAPER_STIM, (Hh // 2,) * 3, 20, steps, None)


TEST2_PARTS = ((12, 12, 2), (16, 16, 2), (16, 16, 4), (24, 24, 4), (32, 32, 4), (48, 48, 8))


def test2(parts, steps: int = 40) -> Workload:
    """The strong-scaling slab of Sec. 6, Test 2 (192 x 192 x 32 elements,
    2,458,434 dofs, h = 0.01 cm) cut into parts = (px, py, pz) equal boxes,
    corner stimulus as in the other slabs, 2 ms from rest by default.  The
    partitions in TEST2_PARTS range from 288 subdomains of 16 x 16 x 16
    elements to 18,432 of 4 x 4 x 4."""
    px, py, pz = parts
    if 192 % px or 192 % py or 32 % pz:
        raise ValueError("parts must divide 192 x 192 x 32")
    m = box_mesh(192, 192, 32, 0.01, px, py, pz)
    return Workload(f"test2_{px}x{py}x{pz}", m, Physics(), Solver(), PAPER_STIM, (2, 2, 2), 20, steps, None)


def test4(parts=(24, 12, 3), steps: int = 2400, paper_geometry: bool = True) -> Workload:
    """The whole-beat slab of Sec. 6, Test 4: 192 x 96 x 24 elements in equal
    box subdomains (the paper uses 8 x 8 x 2), corner stimulus of 2 x 2 x 2
    elements, 2400 steps of 0.05 ms (120 ms: activation and recovery).  With
    paper_geometry the slab is the paper's 1.92 x 1.92 x 0.48 cm, i.e. box
    elements of 0.01 x 0.02 x 0.02 cm (so the paper's 8 x 8 x 2 partition
    has subdomains that are 0.24 cm cubes of 24 x 12 x 12 elements);
    otherwise cubic elements of 0.01 cm (a 1.92 x 0.96 x 0.24 cm slab)."""
    px, py, pz = parts
    if 192 % px or 96 % py or 24 % pz:
        raise ValueError("parts must divide 192 x 96 x 24")
    m = box_mesh(192, 96, 24, 0.01, px, py, pz)
    if paper_geometry:
        m = dataclasses.replace(m, hy=0.02, hz=0.02)
    tag = "" if paper_geometry else "_cubic"
    return Workload(f"test4_{px}x{py}x{pz}{tag}", m, Physics(), Solver(), PAPER_STIM, (2, 2, 2), 20, steps, None)


# Axes (cm) and angular ranges of the truncated ellipsoid.  The paper gives
# the parametric form but not its coefficients; these describe a portion of
# an idealised left ventricle: a wall 1.2 cm thick at the equator and 0.6 cm
# at the apex end, latitudes from -67.5 to 22.5 degrees and half the
# circumference.
ELLIPSOID = (1.5, 2.7, 1.5, 2.7, 4.4, 5.0, -3.0 * math.pi / 8.0, math.pi / 8.0,
             -math.pi / 4.0, 3.0 * math.pi / 4.0)


def ellipsoid_mesh(nx, ny, nz, px, py, pz, geometry=ELLIPSOID) -> Mesh:
    """nx x ny x nz elements over (phi, theta, r) of the truncated ellipsoid,
    in px x py x pz equal subdomains."""
    return Mesh(nx, ny, nz, 1.0, uniform_cuts(nx, px), uniform_cuts(ny, py), uniform_cuts(nz, pz),
                ellipsoid=tuple(float(x) for x in geometry))


def ellipsoid_workload(parts=(8, 8, 4), mesh=(128, 128, 64), steps: int = 40) -> Workload:
    """The ellipsoid of Sec. 6, Test 2 (128 x 128 x 64 elements, 2,163,330
    dofs) or another mesh of the same geometry, in parts = (px, py, pz)
    equal subdomains; stimulus on the 2 x 2 x 2 elements at the grid origin
    (the inner surface at the apex end) for 20 steps, 2 ms from rest."""
    m = ellipsoid_mesh(*mesh, *parts)
    tag = "x".join(str(x) for x in mesh) + "_" + "x".join(str(x) for x in parts)
    return Workload(f"ellipsoid_{tag}", m, Physics(), Solver(), PAPER_STIM, (2, 2, 2), 20, steps, None)


def small_mesh(n: Sequence[int], parts: Sequence[int], h: float = 0.01) -> Mesh:
    return box_mesh(n[0], n[1], n[2], h, parts[0], parts[1], parts[2])
