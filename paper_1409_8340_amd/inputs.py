"""Seeded synthetic inputs shared by the HIP path's tests/benchmark and the
oracle.  This module holds random draws and workload descriptions only -- none
of the method's arithmetic (no links, no stencils, no rasterising, no field
quantisation).

Every generator uses numpy's PCG64 bit generator keyed by an explicit seed, so
both sides of a comparison receive bit-identical arrays.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def psi_init(nx: int, ny: int, nz: int, seed: int, noise: float = 0.01) -> np.ndarray:
    """Initial order parameter psi = 1 + noise*(n1 + i n2), n1, n2 iid N(0,1),
    rounded to complex64.  Shape (nz, ny, nx), x fastest.  Drawn plane by
    plane (z-order) so memory stays bounded for large grids."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((nz, ny, nx), dtype=np.complex64)
    for k in range(nz):
        z = rng.standard_normal((2, ny, nx))
        out[k].real = (1.0 + noise * z[0]).astype(np.float32)
        out[k].imag = (noise * z[1]).astype(np.float32)
    return out


def random_complex(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Generic complex64 test field with iid N(0, scale^2) parts."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((2,) + tuple(shape))
    return (scale * (z[0] + 1j * z[1])).astype(np.complex64)


def random_real(shape, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=shape).astype(np.float32)


def sphere_candidates(lengths, n: int, seed: int, law: str = "fixed", d: float = 4.0,
                      d_lo: float = 2.0, d_hi: float = 6.0, median: float = 3.0,
                      sigma: float = 0.3):
    """Candidate spheres for the inclusion generator: centres uniform in
    [0, Lx) x [0, Ly) x [0, Lz) (float64) and diameters drawn from
      "fixed":     d
      "uniform":   one diameter U[d_lo, d_hi] shared by all spheres
      "lognormal": median * exp(sigma * N(0,1)) per sphere.
    Returns (centres (n,3) float64, diameters (n,) float64)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.random((n, 3)) * np.asarray(lengths, dtype=np.float64)[None, :]
    if law == "fixed":
        dia = np.full(n, float(d))
    elif law == "uniform":
        dia = np.full(n, float(rng.uniform(d_lo, d_hi)))
    elif law == "lognormal":
        dia = median * np.exp(sigma * rng.standard_normal(n))
    else:
        raise ValueError(law)
    return np.ascontiguousarray(c), np.ascontiguousarray(dia)


def ellipsoid_shape(centre, axes, rot=None) -> np.ndarray:
    """One candidate for the general inclusion generator: the ellipsoid with
    semi-axes `axes` along the columns of the rotation `rot` (default the
    identity) around `centre`, as 16 doubles (centre, Q_xx Q_yy Q_zz Q_xy
    Q_xz Q_yz, axis (unused, 0), hlen = -1, bounding half-widths)."""
    R = np.eye(3) if rot is None else np.asarray(rot, dtype=np.float64)
    a = np.asarray(axes, dtype=np.float64)
    Q = R @ np.diag(1.0 / (a * a)) @ R.T
    ext = np.sqrt((R * R) @ (a * a))
    return np.array([*centre, Q[0, 0], Q[1, 1], Q[2, 2], Q[0, 1], Q[0, 2], Q[1, 2], 0.0, 0.0, 0.0, -1.0, *ext],
                    dtype=np.float64)


def column_shape(centre, axis, radius: float, length: float) -> np.ndarray:
    """A columnar candidate: the cylinder of `radius` and `length` along the
    unit vector `axis` through `centre` (Q = (I - n n^T) / radius^2, hlen =
    length / 2), as 16 doubles."""
    n = np.asarray(axis, dtype=np.float64)
    n = n / np.sqrt(np.dot(n, n))
    Q = (np.eye(3) - np.outer(n, n)) / (radius * radius)
    hl = 0.5 * length
    ext = hl * np.abs(n) + radius * np.sqrt(np.maximum(1.0 - n * n, 0.0))
    return np.array([*centre, Q[0, 0], Q[1, 1], Q[2, 2], Q[0, 1], Q[0, 2], Q[1, 2], *n, hl, *ext],
                    dtype=np.float64)


def ellipsoid_candidates(lengths, n: int, seed: int, axes=(1.5, 1.5, 4.0), tilt_deg: float = 0.0,
                         random_azimuth: bool = False) -> np.ndarray:
    """Candidates like the paper's Fig. 2d: ellipsoids of fixed semi-axes and
    one common orientation, centres uniform in the box.  The third axis is
    tilted by tilt_deg from z towards x; with random_azimuth each candidate
    is then turned about z by its own uniform random angle.  (n, 16)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.random((n, 3)) * np.asarray(lengths, dtype=np.float64)[None, :]
    phi = rng.random(n) * 2.0 * np.pi if random_azimuth else np.zeros(n)
    t = np.deg2rad(tilt_deg)
    Ry = np.array([[np.cos(t), 0.0, np.sin(t)], [0.0, 1.0, 0.0], [-np.sin(t), 0.0, np.cos(t)]])
    out = np.empty((n, 16))
    for s in range(n):
        Rz = np.array([[np.cos(phi[s]), -np.sin(phi[s]), 0.0], [np.sin(phi[s]), np.cos(phi[s]), 0.0],
                       [0.0, 0.0, 1.0]])
        out[s] = ellipsoid_shape(c[s], axes, Rz @ Ry)
    return np.ascontiguousarray(out)


def column_candidates(lengths, n: int, seed: int, radius: float = 1.0, tilt_deg: float = 45.0) -> np.ndarray:
    """Candidates like the paper's Fig. 2e: columns of `radius` crossing the
    z extent, tilted by +tilt_deg or -tilt_deg (at random) from z in the xz
    plane, centres uniform in the box.  (n, 16)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    L = np.asarray(lengths, dtype=np.float64)
    c = rng.random((n, 3)) * L[None, :]
    sgn = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    t = np.deg2rad(tilt_deg)
    length = L[2] / np.cos(t)
    out = np.empty((n, 16))
    for s in range(n):
        out[s] = column_shape(c[s], (sgn[s] * np.sin(t), 0.0, np.cos(t)), radius, length)
    return np.ascontiguousarray(out)


def lattice_centres(kind: str, lengths, a: float, z: float = None, offset=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Centres of a regular arrangement of inclusions (Sec. 3.4): in 2D
    (kind "square", "triangular", "honeycomb"; lattice constant a, every
    centre at height z, default mid-box) or 3D ("rectangular": simple cubic
    of constant a, "hexagonal": triangular layers stacked a apart).  Sites
    fill the box [0, L) from `offset`; (n, 3)."""
    Lx, Ly, Lz = (float(v) for v in lengths)
    ox, oy, oz = offset
    zc = 0.5 * Lz if z is None else z

    def grid2(ax, ay, basis, stagger):
        pts = []
        nyr = int(np.floor(Ly / ay + 1e-9))
        nxr = int(np.floor(Lx / ax + 1e-9))
        for r in range(nyr):
            sx = stagger * (r % 2)
            for q in range(nxr):
                for bx, by in basis:
                    pts.append((ox + (q + sx) * ax + bx, oy + r * ay + by))
        return pts

    if kind == "square":
        p2 = grid2(a, a, [(0.0, 0.0)], 0.0)
    elif kind == "triangular":
        p2 = grid2(a, a * np.sqrt(3.0) / 2.0, [(0.0, 0.0)], 0.5)
    elif kind == "honeycomb":
        # two sites per cell of the triangular lattice of constant a sqrt(3)
        A = a * np.sqrt(3.0)
        p2 = grid2(A, 1.5 * a, [(0.0, 0.0), (0.5 * A, 0.5 * a)], 0.5)
    elif kind in ("rectangular", "hexagonal"):
        if kind == "rectangular":
            p2 = grid2(a, a, [(0.0, 0.0)], 0.0)
        else:
            p2 = grid2(a, a * np.sqrt(3.0) / 2.0, [(0.0, 0.0)], 0.5)
        nzl = int(np.floor(Lz / a + 1e-9))
        return np.array([(x % Lx, y % Ly, oz + l * a) for l in range(nzl) for x, y in p2], dtype=np.float64)
    else:
        raise ValueError(f"unknown lattice {kind!r}")
    return np.array([(x % Lx, y % Ly, zc) for x, y in p2], dtype=np.float64)


def voronoi_seeds(lengths, n: int, seed: int, lo: float = 0.5, hi: float = 1.0):
    """Seeds of a polycrystal (Fig. 2c): n positions uniform in the box and
    one eps per crystallite, uniform in [lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.random((n, 3)) * np.asarray(lengths, dtype=np.float64)[None, :]
    vals = lo + (hi - lo) * rng.random(n)
    return pos, vals.astype(np.float32)


def random_checkerboard(shape, cell, seed: int, values=(1.0, 0.5)) -> np.ndarray:
    """Random map of two eps values with equal probability per block of
    cell[0] x cell[1] x cell[2] nodes (z, y, x order), as in Fig. 2a; float32
    of `shape` (nz, ny, nx)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = [-(-shape[a] // cell[a]) for a in range(3)]
    pick = rng.random(nb) < 0.5
    full = np.repeat(np.repeat(np.repeat(pick, cell[0], 0), cell[1], 1), cell[2], 2)
    full = full[:shape[0], :shape[1], :shape[2]]
    return np.where(full, values[0], values[1]).astype(np.float32)


def candidate_count(lengths, target: float, mean_volume: float, safety: float = 2.5) -> int:
    """Number of candidate spheres to draw: enough for the target covered
    fraction with overlaps (coverage 1 - exp(-n v / V)), times a safety
    factor."""
    V = float(np.prod(lengths))
    if target <= 0:
        return 1
    n = -np.log(max(1e-9, 1.0 - target)) * V / max(mean_volume, 1e-12)
    return int(np.ceil(safety * n)) + 16


@dataclass
class Workload:
    """One synthetic workload of the paper's kind (free-flowing or pinned
    vortex matter, B along z, current along x)."""
    name: str
    nx: int
    ny: int
    nz: int
    h: float = 0.5
    open_: tuple = (False, False, True)
    B: float = 0.1
    J: float = 0.0
    driven: bool = False
    steps: int = 200
    window: int = 0
    eps_in: float = -1.0
    eps_out: float = 1.0
    fraction: float = 0.0
    law: str = "fixed"
    d: float = 4.0
    psi_seed: int = 0
    incl_seed: int = 0
    tol: float = 1e-8
    dt: float = 0.1
    extra: dict = field(default_factory=dict)

    def lengths(self):
        ns = (self.nx, self.ny, self.nz)
        return tuple((n - 1) * self.h if o else n * self.h for n, o in zip(ns, self.open_))


# The five workloads the solver is measured and checked on.  x periodic, y
# quasi-periodic, z open throughout; h = 0.5, dt = 0.1, u = 1, g = 1.
WORKLOADS = {
    "c1_small_undriven": Workload("c1_small_undriven", 32, 32, 16, B=0.1, J=0.0, driven=False,
                                  steps=200, psi_seed=1001, incl_seed=2001),
    "c2_256x256x64_J0.02": Workload("c2_256x256x64_J0.02", 256, 256, 64, B=0.1, J=0.02,
                                    driven=True, steps=5000, window=2000, fraction=0.10,
                                    law="fixed", d=4.0, psi_seed=1002, incl_seed=2002),
    "c4_adjoint_128x128x32": Workload("c4_adjoint_128x128x32", 128, 128, 32, B=0.1, J=0.03,
                                      driven=True, steps=500, window=500, fraction=0.08,
                                      law="fixed", d=4.0, psi_seed=1004, incl_seed=2004),
    "c5_1024x1024x128": Workload("c5_1024x1024x128", 1024, 1024, 128, B=0.2, J=0.03,
                                 driven=True, steps=2000, window=1000, fraction=0.15,
                                 law="lognormal", d=3.0, psi_seed=1005, incl_seed=2005,
                                 extra={"J_sweep": [0.005 * i for i in range(13)],
                                        "sigma": 0.3, "median": 3.0}),
}


def batch_workloads(n: int = 64, seed: int = 3003):
    """Batched workload: n instances with shapes drawn uniformly from
    {64^3, 96x96x48, 128x128x32}, B ~ U[0.05, 0.3], J ~ U[0, 0.05], one
    inclusion diameter ~ U[2, 6] and fraction ~ U[0.05, 0.20] per instance."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(64, 64, 64), (96, 96, 48), (128, 128, 32)]
    out = []
    for i in range(n):
        nx, ny, nz = shapes[int(rng.integers(0, 3))]
        B = float(rng.uniform(0.05, 0.3))
        J = float(rng.uniform(0.0, 0.05))
        d = float(rng.uniform(2.0, 6.0))
        frac = float(rng.uniform(0.05, 0.20))
        out.append(Workload(f"c3_inst{i:02d}", nx, ny, nz, B=B, J=J, driven=True, steps=1000,
                            window=1000, fraction=frac, law="fixed", d=d,
                            psi_seed=1003 * 1000 + i, incl_seed=2003 * 1000 + i))
    return out


def candidates_for(w: Workload):
    """Sphere candidates for a workload (enough for its target fraction)."""
    L = w.lengths()
    if w.law == "lognormal":
        med = w.extra.get("median", w.d)
        sig = w.extra.get("sigma", 0.3)
        mean_v = np.pi / 6.0 * med ** 3 * np.exp(4.5 * sig * sig)
    else:
        mean_v = np.pi / 6.0 * w.d ** 3
    n = candidate_count(L, w.fraction, mean_v)
    return sphere_candidates(L, n, w.incl_seed, law=w.law, d=w.d,
                             median=w.extra.get("median", 3.0),
                             sigma=w.extra.get("sigma", 0.3))
