"""Seeded synthetic workloads: solid masks, initial densities and run settings.

This module holds no arithmetic of the lattice Boltzmann method; it only
draws geometries and initial conditions, so both the GPU library and the CPU
oracle can be fed the same inputs.  Random draws use
``numpy.random.default_rng(seed)`` (PCG64) in the order written here.

Initial densities follow the paper's main/dissolved notion (Sec. 2.1,
Fig. 1): the dominant component at a node starts at ``RHO_MAJOR`` and the
other at ``RHO_MINOR``, mirrored between the two components.

Workloads (sizes from the run configurations):
  flat_drop       100x50 channel, droplet cap on the bottom wall      (flat contact angle)
  cylinder_drop   400x400 periodic box, droplet on a cylinder          (curved contact angle)
  porous          2048x1024 channel of random disks, displacement      (precision study)
  calibration     512 square runs, flat or cylinder walls              (batching)
  constrictions   16384x2048 channel with 64 square constrictions     (throughput)
  cocurrent       50x100 channel, two layers, Couette or Poiseuille    (Sec. 3.1)
  obstacle_drop   350x150 channel, droplet past a square obstacle      (Sec. 3.3)
"""
from __future__ import annotations

import dataclasses
import hashlib
from typing import List, Optional, Tuple

import numpy as np

PERIODIC_X = 1
PERIODIC_Y = 2
SCHEME_ORIGINAL = 4
FORCE_DENSITY = 64
INLET = 256
OUTFLOW = 512

RHO_MAJOR = 1.0
RHO_MINOR = 0.03

# Coexisting main / dissolved densities of the two components at G_c = 0.9
# with the same total 1.03: c_s^2 ln(rho_m / rho_d) = G_c (rho_m - rho_d),
# rho_m + rho_d = 1.03.  Droplets in large boxes start here; from 1.0 / 0.03
# they would have to feed the dissolved level of the whole box and dissolve.
RHO_MAJOR_EQ = 0.9319037248975761
RHO_MINOR_EQ = 0.09809627510242387

WALL_FLAT = 0
WALL_CYLINDER = 1


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    flags: int
    solid: np.ndarray            # uint8 [ny, nx], 1 = solid
    rho1: np.ndarray             # float64 [ny, nx]
    rho2: np.ndarray             # float64 [ny, nx]
    G_c: float = 0.9
    G_ads: float = 0.0
    tau: float = 1.0
    accel: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    steps: int = 1000
    wall_kind: Optional[int] = None
    wall: Optional[Tuple[float, float, float]] = None
    # sliding walls: (ubx, uby, utx, uty) of the solid rows below / above ny/2
    wall_velocity: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    # inlet velocity per row, float64 [2, ny] (with the INLET flag)
    inlet_u: Optional[np.ndarray] = None

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny

    @property
    def n_fluid(self) -> int:
        return int(self.n_nodes - int(self.solid.sum()))

    def mask_sha256(self) -> str:
        return hashlib.sha256(np.ascontiguousarray(self.solid, dtype=np.uint8).tobytes()).hexdigest()


def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64)


def _two_phase(inside: np.ndarray, solid: np.ndarray, major: float = RHO_MAJOR, minor: float = RHO_MINOR):
    """Component 1 dominant where ``inside``; mirrored for component 2."""
    rho1 = np.where(inside, major, minor).astype(np.float64)
    rho2 = np.where(inside, minor, major).astype(np.float64)
    rho1[solid != 0] = 0.0
    rho2[solid != 0] = 0.0
    return rho1, rho2


def flat_drop(nx: int = 100, ny: int = 50, radius: float = 20.0, G_ads: float = 0.2,
              G_c: float = 0.9, tau: float = 1.0, steps: int = 5000, major: float = RHO_MAJOR,
              minor: float = RHO_MINOR) -> Workload:
    """Semicircular droplet centred on a flat bottom wall.

    Solid rows y = 0 and y = ny-1, periodic in x; the droplet is
    (x - nx/2)^2 + (y - 0.5)^2 < r^2 (strict).  Flat-wall angle is read with
    the wall line at y = 0.5 (halfway bounce-back)."""
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    inside = (x - nx / 2.0) ** 2 + (y - 0.5) ** 2 < radius * radius
    rho1, rho2 = _two_phase(inside, solid, major, minor)
    return Workload("flat_drop", nx, ny, PERIODIC_X, solid, rho1, rho2, G_c=G_c, G_ads=G_ads,
                    tau=tau, steps=steps, wall_kind=WALL_FLAT, wall=(0.5, 0.0, 0.0))


def cylinder_drop(G_ads: float = 0.0, nx: int = 400, ny: int = 400, R: float = 60.0,
                  centre=(200.0, 150.0), r_drop: float = 50.0, drop_centre=(200.0, 240.0),
                  G_c: float = 0.9, tau: float = 1.0, steps: int = 20000,
                  major: float = RHO_MAJOR_EQ, minor: float = RHO_MINOR_EQ) -> Workload:
    """Droplet on a staircase-voxelised cylinder in a fully periodic box.

    Solid where (x-cx)^2 + (y-cy)^2 < R^2 (strict: with <= an integer R
    leaves a one-voxel spike at each pole, a solid feature one node thick);
    droplet (strict <) centred at ``drop_centre``.  The wall surface for the
    angle is R + 0.5.  Starts at the coexisting densities of G_c = 0.9."""
    x, y = _grid(nx, ny)
    solid = (((x - centre[0]) ** 2 + (y - centre[1]) ** 2) < R * R).astype(np.uint8)
    inside = (x - drop_centre[0]) ** 2 + (y - drop_centre[1]) ** 2 < r_drop * r_drop
    rho1, rho2 = _two_phase(inside, solid, major, minor)
    return Workload("cylinder_drop", nx, ny, PERIODIC_X | PERIODIC_Y, solid, rho1, rho2, G_c=G_c,
                    G_ads=G_ads, tau=tau, steps=steps, wall_kind=WALL_CYLINDER,
                    wall=(centre[0], centre[1], R + 0.5))


CYLINDER_SWEEP = [-0.3, -0.2, -0.1, 0.0, 0.1, 0.2, 0.3]


def porous(nx: int = 2048, ny: int = 1024, seed: int = 2505, solid_fraction: float = 0.30,
           inlet: int = 64, window_x0: int = 96, steps: int = 50000,
           max_attempts: int = 2_000_000) -> Workload:
    """Random non-overlapping disks in a walled channel (porosity ~0.7).

    Random sequential addition: per attempt draw r ~ U[8, 24), then the
    centre x ~ U[x0 + r, nx - r - 2), y ~ U[3 + r, ny - 3 - r); accept when the
    gap to every placed disk is at least 2.  Stop once the disks cover
    ``solid_fraction`` of the interior window x >= x0.  Component 1 fills the
    fluid for x < ``inlet`` and is driven by the body acceleration 1e-6."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    window_area = (nx - window_x0) * (ny - 2)
    disks: List[Tuple[float, float, float]] = []
    covered = 0
    attempts = 0
    while covered < solid_fraction * window_area and attempts < max_attempts:
        attempts += 1
        r = rng.uniform(8.0, 24.0)
        cx = rng.uniform(window_x0 + r, nx - r - 2.0)
        cy = rng.uniform(3.0 + r, ny - 3.0 - r)
        ok = True
        for (qx, qy, qr) in disks:
            if (cx - qx) ** 2 + (cy - qy) ** 2 < (r + qr + 2.0) ** 2:
                ok = False
                break
        if not ok:
            continue
        disks.append((cx, cy, r))
        x0, x1 = int(np.floor(cx - r)), int(np.ceil(cx + r)) + 1
        y0, y1 = int(np.floor(cy - r)), int(np.ceil(cy + r)) + 1
        yy, xx = np.mgrid[y0:y1, x0:x1]
        disk = ((xx - cx) ** 2 + (yy - cy) ** 2) <= r * r
        solid[y0:y1, x0:x1] |= disk.astype(np.uint8)
        covered += int(disk.sum())
    x, _ = _grid(nx, ny)
    rho1, rho2 = _two_phase(x < inlet, solid)
    wl = Workload("porous", nx, ny, PERIODIC_X, solid, rho1, rho2, G_c=0.9, G_ads=0.0, tau=1.0,
                  accel=(1e-6, 0.0, 0.0, 0.0), steps=steps)
    wl.disks = disks  # type: ignore[attr-defined]
    return wl


def calibration_runs(seed: int = 22256, nruns: int = 512, steps: int = 10000) -> List[Workload]:
    """Contact-angle calibration batch of uneven square lattices.

    Per run draw: side from {128, 192, 256, 384, 512}; wall flat or cylinder
    (Bernoulli 0.5); G_ads ~ U[-0.35, 0.35]; tau ~ U[0.7, 1.2].  Droplet radius
    0.2 side.  Flat: walls at rows 0 and side-1, droplet centre (side/2, 0.5).
    Cylinder: periodic, R = 0.15 side at (side/2, 0.375 side), droplet centre
    (side/2, 0.675 side).  Droplets start at the coexisting densities of
    G_c = 0.9."""
    rng = np.random.default_rng(seed)
    sides = [128, 192, 256, 384, 512]
    runs = []
    for _ in range(nruns):
        side = int(sides[int(rng.integers(0, len(sides)))])
        cyl = bool(rng.random() < 0.5)
        G_ads = float(rng.uniform(-0.35, 0.35))
        tau = float(rng.uniform(0.7, 1.2))
        if cyl:
            w = cylinder_drop(G_ads=G_ads, nx=side, ny=side, R=0.15 * side,
                              centre=(side / 2.0, 0.375 * side), r_drop=0.2 * side,
                              drop_centre=(side / 2.0, 0.675 * side), tau=tau, steps=steps)
        else:
            w = flat_drop(nx=side, ny=side, radius=0.2 * side, G_ads=G_ads, tau=tau, steps=steps,
                          major=RHO_MAJOR_EQ, minor=RHO_MINOR_EQ)
        w.name = "calibration"
        runs.append(w)
    return runs


def constrictions(nx: int = 16384, ny: int = 2048, seed: int = 355, n_squares: int = 64,
                  side: int = 128, steps: int = 100000, open_ends: bool = False,
                  u_inlet: float = 0.01) -> Workload:
    """Long walled microchannel with a seeded row of square constrictions.

    Square j starts at x0 = (nx / n_squares) j + U_int[32, 96] and is attached
    to the bottom wall (rows [1, 1+side)) or the top wall (rows
    [ny-1-side, ny-1)) by a fair coin, drawn in that order.  Component 1
    fills y < ny/2, component 2 the rest; both are driven along x.  Periodic
    in x, or with `open_ends` a Zou-He inlet (Poiseuille profile of peak
    `u_inlet`) at x = 0 and an outflow at x = nx-1."""
    rng = np.random.default_rng(seed)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    pitch = nx // n_squares
    for j in range(n_squares):
        x0 = pitch * j + int(rng.integers(32, 97))
        top = bool(rng.random() < 0.5)
        y0 = ny - 1 - side if top else 1
        solid[y0:y0 + side, x0:x0 + side] = 1
    _, y = _grid(nx, ny)
    rho1, rho2 = _two_phase(y < ny / 2.0, solid)
    if open_ends:
        return Workload("constrictions_open", nx, ny, INLET | OUTFLOW, solid, rho1, rho2, G_c=0.9, G_ads=0.15,
                        tau=1.0, accel=(2e-6, 0.0, 2e-6, 0.0), steps=steps,
                        inlet_u=poiseuille_profile(ny, u_inlet))
    return Workload("constrictions", nx, ny, PERIODIC_X, solid, rho1, rho2, G_c=0.9, G_ads=0.15,
                    tau=1.0, accel=(2e-6, 0.0, 2e-6, 0.0), steps=steps)


def poiseuille_profile(ny: int, u_max: float) -> np.ndarray:
    """Inlet rows of a channel walled at rows 0 and ny-1: the parabola
    u_x = 4 u_max eta (1 - eta), eta = (y - 1/2) / (ny - 2), through the
    halfway wall planes (the profile -4 U_m y (y - H) / H^2 of Sec. 3.3);
    u_y = 0.  Returns [2, ny] (wall rows 0)."""
    y = np.arange(ny, dtype=np.float64)
    eta = (y - 0.5) / (ny - 2)
    u = np.zeros((2, ny))
    u[0] = 4.0 * u_max * eta * (1.0 - eta)
    u[0, 0] = 0.0
    u[0, ny - 1] = 0.0
    return u


def cocurrent(flow: str = "couette", nx: int = 50, ny: int = 102, a: float = 25.0, G_ads: float = 0.0,
              u_wall: float = 0.005, force: float = 1e-6, tau: float = 1.01, major: float = 1.02,
              minor: float = 0.05, steps: int = 10000) -> Workload:
    """Co-current flow of two layers between walls (Sec. 3.1): 100 fluid
    rows between solid rows 0 and ny-1, periodic in x; component 1 in the
    central layer |y - yc| <= a, component 2 outside (main 1.02, dissolved
    0.05, nu = 0.17 so tau = 1.01).  Couette: the walls slide at -u_wall
    (bottom) and +u_wall (top); Poiseuille: a body force density `force`
    on both components along x."""
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    yc = (ny - 1) / 2.0
    rho1, rho2 = _two_phase(np.abs(y - yc) <= a, solid, major, minor)
    if flow == "couette":
        return Workload("couette", nx, ny, PERIODIC_X, solid, rho1, rho2, G_c=0.9, G_ads=G_ads, tau=tau,
                        steps=steps, wall_velocity=(-u_wall, 0.0, u_wall, 0.0))
    if flow == "poiseuille":
        return Workload("poiseuille", nx, ny, PERIODIC_X | FORCE_DENSITY, solid, rho1, rho2, G_c=0.9,
                        G_ads=G_ads, tau=tau, steps=steps, accel=(force, 0.0, force, 0.0))
    raise ValueError(flow)


def obstacle_drop(nx: int = 350, ny: int = 150, side: int = 25, centre=(122.0, 75.0), r_drop: float = 25.0,
                  drop_centre=(55.0, 75.0), G_ads: float = -0.2, tau: float = 1.01, reynolds: float = 7.5,
                  steps: int = 10000) -> Workload:
    """Droplet carried past a square obstacle in a microchannel (Sec. 3.3):
    walls at rows 0 and ny-1, a square of side `side` centred at `centre`,
    droplet (component 1) of radius r at `drop_centre`, component 2
    elsewhere.  Zou-He inlet at x = 0 with the Poiseuille profile, outflow
    at x = nx-1.  u_max from Re = u_max (2 r) / nu with nu = (tau - 1/2)/3;
    G_ads = -0.2 puts the static angle near the configured 30 degrees."""
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    solid[0, :] = 1
    solid[ny - 1, :] = 1
    h = side / 2.0
    sq = (np.abs(x - centre[0]) < h) & (np.abs(y - centre[1]) < h)
    solid[sq] = 1
    inside = (x - drop_centre[0]) ** 2 + (y - drop_centre[1]) ** 2 < r_drop * r_drop
    rho1, rho2 = _two_phase(inside, solid)
    nu = (tau - 0.5) / 3.0
    u_max = reynolds * nu / (2.0 * r_drop)
    return Workload("obstacle_drop", nx, ny, INLET | OUTFLOW, solid, rho1, rho2, G_c=0.9, G_ads=G_ads,
                    tau=tau, steps=steps, inlet_u=poiseuille_profile(ny, u_max))


def random_small(seed: int, nx: int = 24, ny: int = 18, flags: int = PERIODIC_X | PERIODIC_Y,
                 n_blobs: int = 3, walls: bool = False, drop: bool = True) -> Workload:
    """Small random geometry for parity cases: a few solid blobs (discs and
    rectangles at least 2 nodes thick) and a random droplet."""
    rng = np.random.default_rng(seed)
    x, y = _grid(nx, ny)
    solid = np.zeros((ny, nx), dtype=np.uint8)
    if walls:
        solid[0, :] = 1
        solid[ny - 1, :] = 1
    for _ in range(n_blobs):
        kind = int(rng.integers(0, 2))
        cx, cy = rng.uniform(0, nx), rng.uniform(0, ny)
        if kind == 0:
            r = rng.uniform(1.5, 4.0)
            dx = np.minimum(np.abs(x - cx), nx - np.abs(x - cx)) if flags & PERIODIC_X else x - cx
            dy = np.minimum(np.abs(y - cy), ny - np.abs(y - cy)) if flags & PERIODIC_Y else y - cy
            solid |= ((dx ** 2 + dy ** 2) <= r * r).astype(np.uint8)
        else:
            w, h = int(rng.integers(2, 6)), int(rng.integers(2, 6))
            x0, y0 = int(cx), int(cy)
            for j in range(h):
                for i in range(w):
                    xx, yy = x0 + i, y0 + j
                    if flags & PERIODIC_X:
                        xx %= nx
                    if flags & PERIODIC_Y:
                        yy %= ny
                    if 0 <= xx < nx and 0 <= yy < ny:
                        solid[yy, xx] = 1
    if drop:
        dcx, dcy, dr = rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(3.0, min(nx, ny) / 3.0)
        inside = (x - dcx) ** 2 + (y - dcy) ** 2 < dr * dr
    else:
        inside = np.zeros((ny, nx), dtype=bool)
    rho1, rho2 = _two_phase(inside, solid)
    # a small seeded perturbation so that no two nodes start identical
    pert = rng.uniform(-0.01, 0.01, size=(2, ny, nx))
    rho1 = np.where(solid != 0, 0.0, rho1 + pert[0] * rho1)
    rho2 = np.where(solid != 0, 0.0, rho2 + pert[1] * rho2)
    return Workload("random_small", nx, ny, flags, solid, rho1, rho2, G_c=0.9,
                    G_ads=float(rng.uniform(-0.3, 0.3)), tau=float(rng.uniform(0.7, 1.3)),
                    accel=(float(rng.uniform(-1e-4, 1e-4)), float(rng.uniform(-1e-4, 1e-4)),
                           float(rng.uniform(-1e-4, 1e-4)), float(rng.uniform(-1e-4, 1e-4))),
                    steps=100)


def random_populations(seed: int, wl: Workload, amplitude: float = 0.2) -> np.ndarray:
    """Seeded non-equilibrium population set [2, 9, ny, nx] around
    w_i-free uniform values: f_i = rho_k/9 * (1 + a U[-1, 1)).  Solid entries
    are zero.  Used to start parity runs far from equilibrium."""
    rng = np.random.default_rng(seed)
    base = np.stack([wl.rho1, wl.rho2])[:, None, :, :] / 9.0
    f = base * (1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(2, 9, wl.ny, wl.nx)))
    f[:, :, wl.solid != 0] = 0.0
    return f


# ---------------------------------------------------------------------------
# Three dimensions (Sec. 3.5): arrays are [nz, ny, nx], node id
# (z * ny + y) * nx + x.
# ---------------------------------------------------------------------------
PERIODIC_Z = 2048
WALL_SPHERE = 1


@dataclasses.dataclass
class Workload3D:
    name: str
    nx: int
    ny: int
    nz: int
    flags: int
    solid: np.ndarray            # uint8 [nz, ny, nx], 1 = solid
    rho1: np.ndarray             # float64 [nz, ny, nx]
    rho2: np.ndarray
    G_c: float = 0.9
    G_ads: float = 0.0
    tau: float = 1.0
    accel: Tuple[float, ...] = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)  # g1 (x, y, z), g2 (x, y, z)
    steps: int = 1000
    wall_kind: Optional[int] = None
    wall: Optional[Tuple[float, float, float, float]] = None

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_fluid(self) -> int:
        return int(self.n_nodes - int(self.solid.sum()))


def _grid3(nx: int, ny: int, nz: int):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx]
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def g_ads_of_lambda(lam: float, G_c: float = 0.9) -> float:
    """G_ads whose lambda = G_w1 / G_w2 = 1 + 2 G_ads / G_c is `lam`."""
    return (lam - 1.0) * G_c / 2.0


SPHERE_LAMBDAS = [0.38, 1.0, 2.1]


def sphere_drop(lam: float = 1.0, nx: int = 200, ny: int = 200, nz: int = 280, R: float = 50.0,
                centre=(100.0, 100.0, 100.0), r_drop: float = 45.0, drop_centre=(100.0, 100.0, 180.0),
                G_c: float = 0.9, tau: float = 1.0, steps: int = 20000,
                major: float = RHO_MAJOR_EQ, minor: float = RHO_MINOR_EQ) -> Workload3D:
    """Droplet on a solid sphere in a fully periodic box (Sec. 3.5: 200 x 200
    x 280, sphere R = 50 at (100, 100, 100), droplet r = 45 at (100, 100,
    180), lambda = 0.38 / 1 / 2.1).  Solid where |x - c| < R (strict);
    droplet strict too; the spheres overlap by 15 as set up in the paper.
    Starts at the coexisting densities of G_c = 0.9; the wall surface for
    the angle is R + 0.5."""
    x, y, z = _grid3(nx, ny, nz)
    solid = (((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2) < R * R).astype(np.uint8)
    inside = (x - drop_centre[0]) ** 2 + (y - drop_centre[1]) ** 2 + (z - drop_centre[2]) ** 2 < r_drop * r_drop
    rho1, rho2 = _two_phase(inside, solid, major, minor)
    return Workload3D("sphere_drop", nx, ny, nz, PERIODIC_X | PERIODIC_Y | PERIODIC_Z, solid, rho1, rho2,
                      G_c=G_c, G_ads=g_ads_of_lambda(lam, G_c), tau=tau, steps=steps, wall_kind=WALL_SPHERE,
                      wall=(centre[0], centre[1], centre[2], R + 0.5))


def flat_drop3d(nx: int = 40, ny: int = 40, nz: int = 24, radius: float = 10.0, G_ads: float = 0.0,
                G_c: float = 0.9, tau: float = 1.0, steps: int = 2000, major: float = RHO_MAJOR_EQ,
                minor: float = RHO_MINOR_EQ) -> Workload3D:
    """Hemispherical cap on the wall z = 0: solid planes z = 0 and z = nz-1,
    periodic in x and y, droplet |x - (nx/2, ny/2, 0.5)| < r (strict); the
    wall plane for the angle is z = 0.5."""
    x, y, z = _grid3(nx, ny, nz)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    solid[0] = 1
    solid[nz - 1] = 1
    inside = (x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2 + (z - 0.5) ** 2 < radius * radius
    rho1, rho2 = _two_phase(inside, solid, major, minor)
    return Workload3D("flat_drop3d", nx, ny, nz, PERIODIC_X | PERIODIC_Y, solid, rho1, rho2, G_c=G_c,
                      G_ads=G_ads, tau=tau, steps=steps, wall_kind=WALL_FLAT, wall=(0.5, 0.0, 0.0, 0.0))


def random_small3d(seed: int, nx: int = 14, ny: int = 12, nz: int = 10,
                   flags: int = PERIODIC_X | PERIODIC_Y | PERIODIC_Z, n_blobs: int = 3,
                   speckle: float = 0.0) -> Workload3D:
    """Small random 3-D geometry for parity cases: balls and boxes at least
    2 nodes thick (or, with `speckle` > 0, that fraction of single solid
    voxels), a random droplet, and a seeded perturbation of the densities."""
    rng = np.random.default_rng(seed)
    x, y, z = _grid3(nx, ny, nz)
    solid = np.zeros((nz, ny, nx), dtype=np.uint8)
    if speckle > 0.0:
        solid |= (rng.random((nz, ny, nx)) < speckle).astype(np.uint8)
    else:
        for _ in range(n_blobs):
            c = (rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz))
            r = rng.uniform(1.5, 3.0)
            d = []
            for v, cc, n, bit in ((x, c[0], nx, PERIODIC_X), (y, c[1], ny, PERIODIC_Y), (z, c[2], nz, PERIODIC_Z)):
                dv = np.abs(v - cc)
                d.append(np.minimum(dv, n - dv) if flags & bit else dv)
            if int(rng.integers(0, 2)) == 0:
                solid |= ((d[0] ** 2 + d[1] ** 2 + d[2] ** 2) <= r * r).astype(np.uint8)
            else:
                solid |= ((d[0] <= r) & (d[1] <= r) & (d[2] <= r)).astype(np.uint8)
    dc = (rng.uniform(0, nx), rng.uniform(0, ny), rng.uniform(0, nz))
    dr = rng.uniform(2.5, min(nx, ny, nz) / 3.0)
    inside = (x - dc[0]) ** 2 + (y - dc[1]) ** 2 + (z - dc[2]) ** 2 < dr * dr
    rho1, rho2 = _two_phase(inside, solid)
    pert = rng.uniform(-0.01, 0.01, size=(2, nz, ny, nx))
    rho1 = np.where(solid != 0, 0.0, rho1 + pert[0] * rho1)
    rho2 = np.where(solid != 0, 0.0, rho2 + pert[1] * rho2)
    acc = tuple(float(v) for v in rng.uniform(-1e-4, 1e-4, size=6))
    return Workload3D("random_small3d", nx, ny, nz, flags, solid, rho1, rho2, G_c=0.9,
                      G_ads=float(rng.uniform(-0.3, 0.3)), tau=float(rng.uniform(0.7, 1.3)), accel=acc, steps=100)


def random_populations3d(seed: int, wl: Workload3D, amplitude: float = 0.2) -> np.ndarray:
    """Seeded non-equilibrium population set [2, 19, nz, ny, nx]:
    f_i = rho_k / 19 * (1 + a U[-1, 1)), zero on solid nodes."""
    rng = np.random.default_rng(seed)
    base = np.stack([wl.rho1, wl.rho2])[:, None] / 19.0
    f = base * (1.0 + amplitude * rng.uniform(-1.0, 1.0, size=(2, 19, wl.nz, wl.ny, wl.nx)))
    f[:, :, wl.solid != 0] = 0.0
    return f
