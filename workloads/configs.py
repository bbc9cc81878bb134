"""The synthetic workloads: lattices of identical rigid unit cells.

Physical constants follow the sphere-array example of Section 4.1 (air,
c = 343 m/s, rho = 1.21 kg/m^3).  Every workload is a unit-cell mesh in
cell-local coordinates replicated on an M1 x M2 x M3 axis-aligned lattice; cell
(i1, i2, i3) has its centre at (i1*pitch1, i2*pitch2, i3*pitch3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .meshes import icosphere, tube_segment
from .rng import generator, unit_directions

SOUND_SPEED = 343.0
DENSITY = 1.21


@dataclass(frozen=True)
class Lattice:
    grid: tuple[int, int, int]
    pitch: tuple[float, float, float]

    @property
    def n_cells(self) -> int:
        return self.grid[0] * self.grid[1] * self.grid[2]

    def cell_index(self, i1, i2, i3):
        return i1 + self.grid[0] * (i2 + self.grid[1] * i3)

    def cell_origin(self, c: int) -> np.ndarray:
        i1 = c % self.grid[0]
        i2 = (c // self.grid[0]) % self.grid[1]
        i3 = c // (self.grid[0] * self.grid[1])
        return np.array([i1 * self.pitch[0], i2 * self.pitch[1], i3 * self.pitch[2]])


@dataclass
class Workload:
    name: str
    vertices: np.ndarray          # [nv, 3] float64, cell-local
    triangles: np.ndarray         # [nt, 3] int32
    lattice: Lattice
    frequency: float              # Hz
    order: int                    # truncation number n_t
    formulation: str = "bm"       # "bm" (Burton-Miller) or "cbie"
    plane_waves: np.ndarray | None = None     # [R, 3] unit directions
    point_sources: np.ndarray | None = None   # [R, 3] absolute positions (m)
    amplitude: float = 1.0
    near_radius: tuple[int, int, int] = (1, 1, 1)
    extra: dict = field(default_factory=dict)

    @property
    def k(self) -> float:
        return 2.0 * math.pi * self.frequency / SOUND_SPEED

    @property
    def n_dof_cell(self) -> int:
        return int(self.triangles.shape[0])

    @property
    def n_dof(self) -> int:
        return self.n_dof_cell * self.lattice.n_cells

    @property
    def n_rhs(self) -> int:
        if self.plane_waves is not None:
            return int(self.plane_waves.shape[0])
        if self.point_sources is not None:
            return int(self.point_sources.shape[0])
        return 0

    def with_(self, **kw) -> "Workload":
        d = dict(self.__dict__)
        d.update(kw)
        return Workload(**d)


def config_tiny(formulation: str = "bm") -> Workload:
    """4x1 line of icosphere-level-2 spheres (320 triangles, r = 0.1 m), pitch 0.3 m,
    500 Hz, n_t = 10, one plane wave along +x (N = 1280)."""
    v, t = icosphere(2, 0.1)
    return Workload("tiny_4x1_l2_500Hz", v, t, Lattice((4, 1, 1), (0.3, 0.3, 0.3)), 500.0, 10,
                    formulation, plane_waves=np.array([[1.0, 0.0, 0.0]]))


def config_grid16(grid=(16, 16, 1), level: int = 3, order: int = 10) -> Workload:
    """16x16 sphere lattice, icosphere level 3 (1280 triangles, r = 0.1 m), pitch 0.3 m,
    1 kHz, n_t = 10, one plane wave at 30 degrees azimuth (N = 327,680)."""
    v, t = icosphere(level, 0.1)
    a = math.radians(30.0)
    return Workload(f"grid{grid[0]}x{grid[1]}_l{level}_1kHz", v, t,
                    Lattice(tuple(grid), (0.3, 0.3, 0.3)), 1000.0, order, "bm",
                    plane_waves=np.array([[math.cos(a), math.sin(a), 0.0]]))


def config_large_cell(levels: int = 4, near_order: int = 4) -> Workload:
    """Large unit cells for the multilevel near field (Sec. 3.3): 4x4 lattice of icosphere-level-5
    spheres (20480 triangles, r = 0.1 m), pitch 0.3 m, 1 kHz, n_t = 10, one plane wave at 30
    degrees azimuth (N = 327,680, the size of the 16x16 lattice with 16 times larger cells);
    the subdivision of the cell box (levels) and n_t,near in ``extra``."""
    v, t = icosphere(5, 0.1)
    a = math.radians(30.0)
    return Workload("cells4x4_l5_1kHz", v, t, Lattice((4, 4, 1), (0.3, 0.3, 0.3)), 1000.0, 10, "bm",
                    plane_waves=np.array([[math.cos(a), math.sin(a), 0.0]]),
                    extra={"near_levels": levels, "near_order": near_order})


def config_grid16_ground(plane_z: float = -0.15, reflection: complex = 1.0) -> Workload:
    """The 16x16 sphere lattice above a plane z = plane_z (sound-hard for reflection 1), one
    plane wave at 30 degrees azimuth travelling 30 degrees downwards, toward the plane."""
    w = config_grid16()
    a, e = math.radians(30.0), math.radians(30.0)
    d = np.array([[math.cos(e) * math.cos(a), math.cos(e) * math.sin(a), -math.sin(e)]])
    return w.with_(name="grid16x16_l3_1kHz_ground", plane_waves=d,
                   extra={"plane_z": plane_z, "reflection": reflection})


BATCHED_GRIDS = ((8, 8, 1), (12, 20, 1), (32, 4, 1))
BATCHED_SEEDS = (2201120503, 2201120504, 2201120505)


def config_batched_grids(n_rhs: int = 64) -> list[Workload]:
    """Three uneven lattices of level-2 spheres at 800 Hz, n_t = 10, each with
    ``n_rhs`` seeded plane-wave directions uniform on the unit sphere."""
    v, t = icosphere(2, 0.1)
    out = []
    for g, s in zip(BATCHED_GRIDS, BATCHED_SEEDS):
        out.append(Workload(f"batched_{g[0]}x{g[1]}_l2_800Hz", v, t, Lattice(g, (0.3, 0.3, 0.3)),
                            800.0, 10, "bm", plane_waves=unit_directions(n_rhs, s)))
    return out


def barrier_frequencies(count: int = 96) -> np.ndarray:
    return 100.0 * 20.0 ** (np.arange(count) / (count - 1))


def config_barrier_r4b(freq_index: int = 95) -> Workload:
    """Sonic-crystal barrier: 40 x 2 cylinders (r = 0.08 m, 2 m tall, pitch 0.2 m), each
    cylinder split into 8 stacked open tube cells (0.25 m, 192 triangles), lattice
    40 x 2 x 8; point source 2 m in front of the front row, mid-length, mid-height."""
    v, t = tube_segment(0.08, 0.25, 32, 3)
    f = float(barrier_frequencies()[freq_index])
    lat = Lattice((40, 2, 8), (0.2, 0.2, 0.25))
    src = np.array([[39 * 0.2 / 2.0, -2.0, 7 * 0.25 / 2.0]])
    order = 10 if f <= 1000.0 else 14
    return Workload(f"barrier_40x2x8_{f:.1f}Hz", v, t, lat, f, order, "bm", point_sources=src,
                    extra={"receivers": barrier_receivers()})


def config_barrier_ground(freq_index: int = 95) -> Workload:
    """The barrier of config_barrier_r4b standing on sound-hard ground: the plane z = -0.125 m
    through the lower rim of the lowest segments (reflection 1), the point source 1 m above the
    ground, 2 m in front of the front row, mid-length."""
    w = config_barrier_r4b(freq_index)
    src = np.array([[39 * 0.2 / 2.0, -2.0, -0.125 + 1.0]])
    return w.with_(name=w.name + "_ground", point_sources=src,
                   extra={"receivers": w.extra["receivers"], "plane_z": -0.125, "reflection": 1.0})


def barrier_receivers(n_along: int = 8, n_up: int = 8) -> np.ndarray:
    """Observation points of the barrier: a vertical n_along x n_up grid 2 m behind the
    back row (y = 0.2 + 2), spanning +-2 m along the barrier about its middle (x = 3.9)
    and heights 0.25 - 1.75 m above the cylinders' base (z = -0.125); [n_along*n_up, 3]."""
    xs = 39 * 0.2 / 2.0 + np.linspace(-2.0, 2.0, n_along)
    zs = -0.125 + np.linspace(0.25, 1.75, n_up)
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    return np.stack([X.ravel(), np.full(X.size, 0.2 + 2.0), Z.ravel()], axis=1)


def serving_stream(n_requests: int, rate: float = 20.0, seed: int = 2201120505):
    """Seeded Poisson request stream: (arrival time s, grid, frequency Hz, n_rhs, direction seed)."""
    g = generator(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += g.exponential(1.0 / rate)
        n1 = int(g.integers(4, 65))
        n2 = int(g.integers(1, 17))
        f = float(g.uniform(200.0, 2000.0))
        r = int(g.integers(1, 33))
        out.append((t, (n1, n2, 1), f, r, int(seed) * 1000 + i))
    return out
