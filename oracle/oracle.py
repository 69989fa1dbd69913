"""FP64 CPU oracle for the implicit TDGL step of Sadovskyy et al.,
"Stable large-scale solver for Ginzburg-Landau equations for superconductors"
(arXiv:1409.8340).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark may import this module.  It
shares no code with the HIP path; both sides only receive the same seeded
input arrays.

Plain stencil loops live in ``tdgl_oracle.c`` (double precision, loaded with
ctypes); this module adds what is clearer in numpy: the Landau-gauge link
variables, the exact Poisson solve (spectral, with scipy's FFT/DCT as a
library step), the time-step driver and the inclusion rasteriser.

Readings of places where the paper is silent or ambiguous are marked
"reading:" below; the same list is kept with the design notes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_SRC_PATH = os.path.join(_HERE, "tdgl_oracle.c")


def build(force: bool = False) -> str:
    """Compile the C part of the oracle (gcc, -O2, OpenMP, no FMA contraction
    beyond what plain x86-64 code generation does)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC_PATH, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _CGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("open_x", ctypes.c_int), ("open_y", ctypes.c_int), ("open_z", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("g", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        G = ctypes.POINTER(_CGrid)
        D = ctypes.c_double
        lib.orc_neighbour_sum.argtypes = [G, P, P, P, P, P]
        lib.orc_laplacian.argtypes = [G, P, P, P, P, P]
        lib.orc_assemble.argtypes = [G, P, P, P, P, P, P, D, D, P, P]
        lib.orc_apply_M.argtypes = [G, P, P, P, P, D, P, P]
        lib.orc_jacobi_sweep.argtypes = [G, P, P, P, P, P, D, P, P]
        lib.orc_jacobi_sweep.restype = D
        lib.orc_residual_max2.argtypes = [G, P, P, P, P, P, D, P]
        lib.orc_residual_max2.restype = D
        lib.orc_jav.argtypes = [G, P, P]
        lib.orc_jav.restype = D
        lib.orc_poisson_rhs.argtypes = [G, P, P, P, P, P]
        lib.orc_poisson_apply.argtypes = [G, P, P]
        lib.orc_node_weights.argtypes = [G, P]
        lib.orc_free_energy.argtypes = [G, P, P, P, P, P]
        lib.orc_free_energy.restype = D
        lib.orc_weighted_sum.argtypes = [G, P]
        lib.orc_weighted_sum.restype = D
        lib.orc_cut_neighbour_sum.argtypes = [G, P, P, P, P, P, P, P]
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def set_threads(n: int) -> int:
    """Sets the OpenMP thread count of the C loops; returns the previous one."""
    lib = _load()
    prev = lib.orc_max_threads()
    lib.orc_set_threads(int(n))
    return prev


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# Grid, field, links
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    """Cuboid mesh of Sec. 3: nodes x = i hx, y = j hy, z = k hz.

    ``open_`` holds, per axis, True for open (Neumann, Sec. 3.3.2) and False
    for periodic / quasi-periodic (Sec. 3.3.1).
    """
    nx: int
    ny: int
    nz: int
    hx: float = 0.5
    hy: float = 0.5
    hz: float = 0.5
    open_: tuple = (False, False, True)
    g: float = 1.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def length(self, axis: int) -> float:
        """System size: L = N h for periodic axes, (N-1) h for open axes
        (Sec. 3, mesh spacing definitions)."""
        n = (self.nx, self.ny, self.nz)[axis]
        h = (self.hx, self.hy, self.hz)[axis]
        return (n - 1) * h if self.open_[axis] else n * h

    def c(self) -> _CGrid:
        return _CGrid(self.nx, self.ny, self.nz, int(self.open_[0]), int(self.open_[1]),
                      int(self.open_[2]), self.hx, self.hy, self.hz, self.g)


def quantize_field(grid: Grid, Bx: float, Bz: float):
    """Round the field of the xz-plane gauge to whole flux quanta through the
    periodic cross sections (Sec. 3.3.1, "Implications for the magnetic
    field"): Bz = 2 pi n_z / (Lx Ly) when x and y are both periodic,
    Bx = 2 pi n_x / (Ly Lz) when y and z are both periodic.  Components that
    are not constrained are returned unchanged."""
    Lx, Ly, Lz = grid.length(0), grid.length(1), grid.length(2)
    if not grid.open_[0] and not grid.open_[1]:
        Bz = 2 * np.pi * np.round(Bz * Lx * Ly / (2 * np.pi)) / (Lx * Ly)
    if not grid.open_[1] and not grid.open_[2]:
        Bx = 2 * np.pi * np.round(Bx * Ly * Lz / (2 * np.pi)) / (Ly * Lz)
    return float(Bx), float(Bz)


def landau_links(grid: Grid, Bx: float, Bz: float, K: float):
    """Per-edge link variables U = exp(-i h_a A~_a) (Eq. link_variables) for
    the xz-plane field in the Landau gauge A = ybar [-Bz, 0, Bx]
    (Eq. A_xz), with the current phase K folded into A~ = A - [K, 0, 0]
    (Sec. 2.2):

      x links: exp(+i hx (K + Bz ybar_j))
      z links: exp(-i hz Bx ybar_j)
      y links: 1, except the wrap edge j = ny-1 -> 0 of a periodic y axis,
               which carries conj(P_{i,k}),
               P_{i,k} = exp(i (i hx Ly Bz - k hz Ly Bx))  (Sec. 3.3.1),
               so that psi_{i,-1,k} = P_{i,k} psi_{i,ny-1,k}.

    reading: ybar_j = j hy - Ly/2 with Ly the system size of Sec. 3.
    """
    nz, ny, nx = grid.shape
    Ly = grid.length(1)
    j = np.arange(ny, dtype=np.float64)
    ybar = j * grid.hy - Ly / 2.0
    phx = grid.hx * (K + Bz * ybar)
    phz = -grid.hz * Bx * ybar
    lx = np.broadcast_to(np.exp(1j * phx)[None, :, None], grid.shape).astype(np.complex128)
    lz = np.broadcast_to(np.exp(1j * phz)[None, :, None], grid.shape).astype(np.complex128)
    ly = np.ones(grid.shape, dtype=np.complex128)
    if not grid.open_[1]:
        i = np.arange(nx, dtype=np.float64)[None, :]
        k = np.arange(nz, dtype=np.float64)[:, None]
        P = np.exp(1j * (i * grid.hx * Ly * Bz - k * grid.hz * Ly * Bx))
        ly[:, ny - 1, :] = np.conj(P)
    return (np.ascontiguousarray(lx), np.ascontiguousarray(ly), np.ascontiguousarray(lz))


def quantize_field_yz(grid: Grid, By: float, Bz: float):
    """Rounding for the yz-plane field (Sec. 3.3.1, "Implications for the
    magnetic field", applied to the x seam of the yz gauge): the phase jump
    P_{j,k} must be periodic in j and k, so Bz = 2 pi n_z / (Lx Ly) when x
    and y are both periodic and By = 2 pi n_y / (Lx Lz) when x and z are."""
    Lx, Ly, Lz = grid.length(0), grid.length(1), grid.length(2)
    if not grid.open_[0] and not grid.open_[1]:
        Bz = 2 * np.pi * np.round(Bz * Lx * Ly / (2 * np.pi)) / (Lx * Ly)
    if not grid.open_[0] and not grid.open_[2]:
        By = 2 * np.pi * np.round(By * Lx * Lz / (2 * np.pi)) / (Lx * Lz)
    return float(By), float(Bz)


def landau_links_yz(grid: Grid, By: float, Bz: float, K: float):
    """Link variables for the yz-plane field (Eq. B_yz) in the gauge of
    Eq. A_yz, A = xbar [0, Bz, -By], with the current phase K on the x
    links (Eq. link_variables with the index i, Eq. LaplUV_yz):

      x links: exp(+i hx K), except the wrap edge i = nx-1 -> 0 of a
               periodic x axis, which also carries conj(P_{j,k}),
               P_{j,k} = exp(i (-j hy Lx Bz + k hz Lx By))  (Sec. 3.3.1,
               "Magnetic field in yz plane"), so that
               psi_{-1,j,k} = P_{j,k} psi_{nx-1,j,k};
      y links: exp(-i hy Bz xbar_i);
      z links: exp(+i hz By xbar_i);

    reading: xbar_i = i hx - Lx/2 with Lx the system size of Sec. 3; the
    index typos of the printed x-boundary formulas are read as corrected.
    """
    nz, ny, nx = grid.shape
    Lx = grid.length(0)
    i = np.arange(nx, dtype=np.float64)
    xbar = i * grid.hx - Lx / 2.0
    lx = np.full(grid.shape, np.exp(1j * grid.hx * K), dtype=np.complex128)
    if not grid.open_[0]:
        j = np.arange(ny, dtype=np.float64)[None, :]
        k = np.arange(nz, dtype=np.float64)[:, None]
        P = np.exp(1j * (-j * grid.hy * Lx * Bz + k * grid.hz * Lx * By))
        lx[:, :, nx - 1] = lx[:, :, nx - 1] * np.conj(P)
    ly = np.broadcast_to(np.exp(-1j * grid.hy * Bz * xbar)[None, None, :], grid.shape).astype(np.complex128)
    lz = np.broadcast_to(np.exp(1j * grid.hz * By * xbar)[None, None, :], grid.shape).astype(np.complex128)
    return (np.ascontiguousarray(lx), np.ascontiguousarray(ly), np.ascontiguousarray(lz))


def base_links_of(grid: Grid, p) -> tuple:
    """Links at K = 0 of the field in p: the xz-plane gauge (Eq. A_xz) or,
    for p.plane == "yz", the yz-plane gauge (Eq. A_yz)."""
    if getattr(p, "plane", "xz") == "yz":
        return landau_links_yz(grid, p.By, p.Bz, 0.0)
    return landau_links(grid, p.Bx, p.Bz, 0.0)


def rewind_K(K: float, hx: float) -> float:
    """Phase rewind K -> K - (2 pi / hx) floor(K hx / 2 pi) (Sec. 2.2).

    reading: applied after every K update; it maps K into [0, 2 pi / hx) and
    leaves every link variable unchanged."""
    return K - (2 * np.pi / hx) * np.floor(K * hx / (2 * np.pi))


# ---------------------------------------------------------------------------
# Operators (thin wrappers over the C loops)
# ---------------------------------------------------------------------------
def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def neighbour_sum(grid, links, psi):
    psi = _c128(psi)
    out = np.empty(grid.shape, np.complex128)
    G = grid.c()
    _load().orc_neighbour_sum(ctypes.byref(G), *map(_p, links), _p(psi), _p(out))
    return out


def laplacian(grid, links, psi):
    """Covariant 7-point Laplacian (Eq. LaplUV_xz, Sec. 3.3 boundary forms)."""
    psi = _c128(psi)
    out = np.empty(grid.shape, np.complex128)
    G = grid.c()
    _load().orc_laplacian(ctypes.byref(G), *map(_p, links), _p(psi), _p(out))
    return out


def assemble(grid, links, psi_prev, eps, mu, u, ht):
    """b and diag(M) of Eq. GL_linearized / Eq. b."""
    psi_prev = _c128(psi_prev)
    eps = _f64(eps)
    mu_arr = _f64(mu) if mu is not None else None  # keep a reference for the call
    mu_p = _p(mu_arr) if mu_arr is not None else None
    b = np.empty(grid.shape, np.complex128)
    d = np.empty(grid.shape, np.complex128)
    G = grid.c()
    _load().orc_assemble(ctypes.byref(G), *map(_p, links), _p(psi_prev), _p(eps), mu_p,
                         float(u), float(ht), _p(b), _p(d))
    return b, d


def apply_M(grid, links, diag, ht, psi):
    psi = _c128(psi)
    out = np.empty(grid.shape, np.complex128)
    G = grid.c()
    _load().orc_apply_M(ctypes.byref(G), *map(_p, links), _p(_c128(diag)), float(ht), _p(psi),
                        _p(out))
    return out


def jacobi_sweep(grid, links, b, diag, ht, psi_in):
    """One iteration of Eq. final; returns (psi_out, max |r(psi_in)|^2)."""
    psi_in = _c128(psi_in)
    out = np.empty(grid.shape, np.complex128)
    G = grid.c()
    r2 = _load().orc_jacobi_sweep(ctypes.byref(G), *map(_p, links), _p(_c128(b)),
                                  _p(_c128(diag)), float(ht), _p(psi_in), _p(out))
    return out, r2


def residual_max2(grid, links, b, diag, ht, psi):
    G = grid.c()
    return _load().orc_residual_max2(ctypes.byref(G), *map(_p, links), _p(_c128(b)),
                                     _p(_c128(diag)), float(ht), _p(_c128(psi)))


def jav(grid, links, psi):
    """Average supercurrent J_av (Sec. 3.1.1)."""
    G = grid.c()
    return _load().orc_jav(ctypes.byref(G), _p(links[0]), _p(_c128(psi)))


def poisson_rhs(grid, links, psi):
    """Right side of the discrete Poisson equation (Sec. 3.2)."""
    out = np.empty(grid.shape, np.float64)
    G = grid.c()
    _load().orc_poisson_rhs(ctypes.byref(G), *map(_p, links), _p(_c128(psi)), _p(out))
    return out


def poisson_apply(grid, mu):
    """Discrete Laplacian of the scalar potential (Sec. 3.2, left side)."""
    out = np.empty(grid.shape, np.float64)
    G = grid.c()
    _load().orc_poisson_apply(ctypes.byref(G), _p(_f64(mu)), _p(out))
    return out


def node_weights(grid):
    out = np.empty(grid.shape, np.float64)
    G = grid.c()
    _load().orc_node_weights(ctypes.byref(G), _p(out))
    return out


def weighted_sum(grid, x):
    G = grid.c()
    return _load().orc_weighted_sum(ctypes.byref(G), _p(_f64(x)))


def free_energy(grid, links, eps, psi):
    """Discrete GL free energy (dimensionless functional whose psi* derivative
    is the right side of Eq. GL_dimensionless; B uniform so the field energy
    is a constant and omitted)."""
    G = grid.c()
    return _load().orc_free_energy(ctypes.byref(G), *map(_p, links), _p(_f64(eps)),
                                   _p(_c128(psi)))


# ---------------------------------------------------------------------------
# Exact solves
# ---------------------------------------------------------------------------
def _axis_eigs(n, h, open_, cfac=1.0):
    """Eigenvalues of minus the 1D second difference (Sec. 3.2 stencil) with
    periodic wrap (Fourier modes) or Neumann reflection (cosine modes)."""
    c = cfac / (h * h)
    if n == 1:
        return np.zeros(1)
    k = np.arange(n, dtype=np.float64)
    if open_:
        return c * (2.0 - 2.0 * np.cos(np.pi * k / (n - 1)))
    return c * (2.0 - 2.0 * np.cos(2.0 * np.pi * k / n))


def poisson_exact(grid: Grid, f: np.ndarray) -> np.ndarray:
    """Exact solution of  Delta_h mu = f  (Sec. 3.2 discretisation) with the
    weighted mean  sum_m w_m mu_m = 0  (w = 1/2 per open face).

    Delta_h is diagonalised exactly by a DFT along periodic axes and a DCT-I
    along open axes (Neumann reflection); the solve divides by the
    eigenvalues and drops the zero mode.  The zero mode of the DCT-I is
    proportional to the weighted sum, so dropping it both projects f onto the
    range of Delta_h and fixes the weighted mean of mu to zero.

    reading: the paper's pseudo-time relaxation (Sec. 3.2) is an iterative
    route to this same solution; the oracle solves it exactly.
    """
    f = np.asarray(f, dtype=np.float64).reshape(grid.shape)
    axes_np = {0: 2, 1: 1, 2: 0}  # physical axis -> numpy axis
    ns = (grid.nx, grid.ny, grid.nz)
    hs = (grid.hx, grid.hy, grid.hz)
    cf = (1.0, 1.0, 1.0 / (grid.g * grid.g))
    x = f.astype(np.float64)
    for a in range(3):
        if grid.open_[a] and ns[a] > 1:
            x = sfft.dct(x, type=1, axis=axes_np[a])
    x = x.astype(np.complex128)
    for a in range(3):
        if not grid.open_[a]:
            x = sfft.fft(x, axis=axes_np[a])
    lam = np.zeros(grid.shape)
    lam += _axis_eigs(grid.nx, grid.hx, grid.open_[0], cf[0])[None, None, :]
    lam += _axis_eigs(grid.ny, grid.hy, grid.open_[1], cf[1])[None, :, None]
    lam += _axis_eigs(grid.nz, grid.hz, grid.open_[2], cf[2])[:, None, None]
    lam[0, 0, 0] = 1.0
    x = -x / lam
    x[0, 0, 0] = 0.0
    for a in range(3):
        if not grid.open_[a]:
            x = sfft.ifft(x, axis=axes_np[a])
    x = x.real
    for a in range(3):
        if grid.open_[a] and ns[a] > 1:
            x = sfft.idct(x, type=1, axis=axes_np[a])
    return np.ascontiguousarray(x)


# ---------------------------------------------------------------------------
# Langevin noise (Sec. 3.1.2, "Noise terms"; Eq. b)
# ---------------------------------------------------------------------------
def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of Salmon, Moraes, Dror and Shaw (SC'11), elementwise over
    numpy arrays: ten rounds; in each, the first and third counter words are
    multiplied by 0xD2511F53 and 0xCD9E8D57 into 64 bits, the new words are
    (hi(c2 M1) ^ c1 ^ k0, lo(c2 M1), hi(c0 M0) ^ c3 ^ k1, lo(c0 M0)), and the
    key is advanced by (0x9E3779B9, 0xBB67AE85) before every round but the
    first.  Returns the four output words as uint64 arrays below 2^32."""
    mask = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & mask for x in (c0, c1, c2, c3)]
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(0x9E3779B9)) & mask
            k1 = (k1 + np.uint64(0xBB67AE85)) & mask
        p0 = c[0] * np.uint64(0xD2511F53)
        p1 = c[2] * np.uint64(0xCD9E8D57)
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c[3] ^ k1, p0 & mask]
    return c


def zeta_max(T: float, u: float, dt: float, hx: float, hy: float, hz: float) -> float:
    """Amplitude of the uniform Langevin draws: zeta_max^2 = 3 T u /
    (2 dt hx hy hz) (Sec. 3.1.2; dt is the reduced time step h_tbar)."""
    return float(np.sqrt(3.0 * T * u / (2.0 * dt * hx * hy * hz)))


def langevin_zeta(grid, T: float, u: float, dt: float, seed: int, n: int) -> np.ndarray:
    """zeta_m(n) = zeta_1 + i zeta_2 at every node for step n: independent
    uniform draws on [-zeta_max, zeta_max] (Sec. 3.1.2).

    reading (generator): the paper names no generator; the draws come from
    Philox4x32-10 with counter (m, n mod 2^32, n div 2^32, 0), m = i + nx (j +
    ny k), key (seed mod 2^32, seed div 2^32), and output words r0, r1 mapped
    to (2 (r >> 8) - (2^24 - 1)) 2^-24, an exact value in (-1, 1)."""
    m = np.arange(grid.N, dtype=np.uint64)
    n = int(n)
    w = philox4x32_10(m, np.full_like(m, n & 0xFFFFFFFF), np.full_like(m, n >> 32), np.zeros_like(m),
                      int(seed) & 0xFFFFFFFF, int(seed) >> 32)

    def uni(r):
        return (2.0 * (r >> np.uint64(8)).astype(np.float64) - (2.0 ** 24 - 1.0)) * 2.0 ** -24

    zm = zeta_max(T, u, dt, grid.hx, grid.hy, grid.hz)
    return (zm * (uni(w[0]) + 1j * uni(w[1]))).reshape(grid.shape)


# ---------------------------------------------------------------------------
# Time step
# ---------------------------------------------------------------------------
@dataclass
class Params:
    """Physical and solver parameters (reduced units of Sec. 2.1).

    tol: threshold on max_m |r_m|^2 (Eq. convergence; squared max norm).
    mode: "mirror" -- the paper's Jacobi iteration with its stop rule
          (psi^(0) = psi^-, stop after the first sweep whose input residual
          meets tol, return that sweep's output);
          "exact" -- Jacobi iterated to max|r| <= 1e-13 max(1, max|b|).
    driven: solve mu~ and K (Sec. 2.2); without a current both stay zero.
    """
    Bx: float = 0.0
    Bz: float = 0.0
    By: float = 0.0          # yz-plane field (plane == "yz")
    plane: str = "xz"        # "xz": Eq. B_xz / A_xz; "yz": Eq. B_yz / A_yz
    J_ext: float = 0.0
    u: float = 1.0
    dt: float = 0.1
    tol: float = 1e-8
    max_iter: int = 100
    mode: str = "mirror"
    driven: bool = False
    noise_T: float = 0.0     # Langevin term (Sec. 3.1.2): reduced temperature, 0 = off
    noise_seed: int = 0
    insulators: np.ndarray = None  # Sec. 3.4 (ii): nonzero = insulating node (cut edges)


@dataclass
class State:
    psi: np.ndarray
    mu: np.ndarray
    K: float = 0.0
    n: int = 0
    V_sum: float = 0.0
    n_avg: int = 0
    last_sweeps: int = 0
    last_res2: float = 0.0
    last_E: float = 0.0
    last_Jav: float = 0.0
    sweeps_hist: list = field(default_factory=list)


def new_state(grid: Grid, psi0) -> State:
    return State(psi=_c128(np.asarray(psi0).reshape(grid.shape)).copy(),
                 mu=np.zeros(grid.shape))


def gl_solve(grid, links, b, diag, ht, psi_prev, tol, max_iter, mode, sweep=None):
    """Jacobi solution of M psi = b (Sec. 3.1, Eq. final / Eq. convergence).

    reading: the initial iterate is psi^-; the residual tested after sweep l
    is that of the sweep's input, r^(l) = b - M psi^(l) = M_mm (psi^(l+1) -
    psi^(l)); the output of the first sweep whose r^(l) passes is returned.
    Returns (psi, sweeps, last max|r|^2).  sweep: the iteration to use
    (default: the uncut Eq. final, jacobi_sweep)."""
    if sweep is None:
        sweep = lambda b_, d_, p_: jacobi_sweep(grid, links, b_, d_, ht, p_)  # noqa: E731
    psi = psi_prev
    if mode == "exact":
        bmax = float(np.max(np.abs(b)))
        thr = (1e-13 * max(1.0, bmax)) ** 2
        for l in range(100000):
            psi_new, r2 = sweep(b, diag, psi)
            psi = psi_new
            if r2 <= thr:
                return psi, l + 1, r2
        raise RuntimeError("exact GL solve did not converge")
    r2 = np.inf
    for l in range(max_iter):
        psi_new, r2 = sweep(b, diag, psi)
        psi = psi_new
        if r2 < tol:
            return psi, l + 1, r2
    return psi, max_iter, r2


def with_K(base_links, hx: float, K: float):
    """Links of A~ = A - [K, 0, 0]: every x link gains the factor exp(i hx K)
    (Eq. link_variables with Eq. psi_transformation)."""
    lx, ly, lz = base_links
    return (np.ascontiguousarray(lx * np.exp(1j * hx * K)), ly, lz)


def step(grid: Grid, p: Params, eps: np.ndarray, st: State, in_window: bool = True,
         base_links=None):
    """One implicit time step in the order of Sec. 4.1: solve psi, then the
    electric field and K, then mu~.

    reading (step order): the paper's Sec. 3 introduction lists psi -> mu~ ->
    K, its implementation section psi -> E/K -> mu~; the implementation order
    is used.  Step n assembles with mu~_{n-1} and K_{n-1}; J_av uses
    (psi_n, K_{n-1}); the Poisson right side uses (psi_n, K_n).
    reading (K integrator): explicit Euler, K_n = K_{n-1} + dt (J_ext - J_av),
    from Eq. K_ODE with dA/dt = 0 (large-lambda limit, Sec. 2.3) and
    Eq. fig:KttoE; the voltage is accumulated from E_n, never from K.
    reading (u): ht = dt/u (the footnote of Eq. GL_numCN), the i u mu~ term
    keeps u, and K advances in real time dt.
    """
    ht = p.dt / p.u
    base = base_links if base_links is not None else base_links_of(grid, p)
    links = with_K(base, grid.hx, st.K)
    mu = st.mu if p.driven else None
    ins = None if p.insulators is None else (np.asarray(p.insulators).reshape(grid.shape) != 0)
    if ins is None:
        b, d = assemble(grid, links, st.psi, eps, mu, p.u, ht)
        sweep = None
    else:
        # Sec. 3.4 (ii): psi is 0 on insulating nodes, which are not solved for
        st.psi = np.where(ins, 0.0, _c128(st.psi))
        b, d = cut_assemble(grid, links, ins, st.psi, eps, mu, p.u, ht)
        sweep = lambda b_, d_, p_: cut_jacobi_sweep(grid, links, ins, b_, d_, ht, p_)  # noqa: E731
    if p.noise_T > 0:
        # Eq. b: (ht/2) 2 zeta_m(t), drawn for the step counter before the step
        b = b + ht * langevin_zeta(grid, p.noise_T, p.u, p.dt, p.noise_seed, st.n)
        if ins is not None:
            b[ins] = 0.0
    psi, sweeps, r2 = gl_solve(grid, links, b, d, ht, st.psi, p.tol, p.max_iter, p.mode,
                               sweep=sweep)
    st.psi = psi
    st.last_sweeps, st.last_res2 = sweeps, r2
    st.sweeps_hist.append(sweeps)
    if p.driven:
        Jav = jav(grid, links, psi) if ins is None else cut_jav(grid, links, ins, psi)
        E = p.J_ext - Jav
        st.K = st.K + p.dt * E
        if in_window:
            st.V_sum += E
            st.n_avg += 1
        st.K = rewind_K(st.K, grid.hx)
        st.last_E, st.last_Jav = E, Jav
        links = with_K(base, grid.hx, st.K)
        f = poisson_rhs(grid, links, psi) if ins is None else cut_poisson_rhs(grid, links, ins, psi)
        st.mu = poisson_exact(grid, f)
    st.n += 1
    return st


def run(grid, p, eps, st, nsteps, window_begin=0, base_links=None):
    """Advance nsteps; the voltage window holds the steps with index >=
    window_begin (counted from the state's step counter at entry).
    base_links: links at K = 0 (default: Landau gauge of the field in p)."""
    n0 = st.n
    if base_links is None:
        base_links = base_links_of(grid, p)
    for s in range(nsteps):
        step(grid, p, eps, st, in_window=(st.n - n0) >= window_begin, base_links=base_links)
    return st


def mean_E(st: State) -> float:
    """Time-averaged electric field <E_x> over the voltage window; the
    voltage across the sample is Lx <E_x>."""
    return st.V_sum / max(st.n_avg, 1)


# ---------------------------------------------------------------------------
# Inclusion generator (Sec. 3.4)
# ---------------------------------------------------------------------------
def gen_voronoi(grid: Grid, seeds: np.ndarray, values: np.ndarray, metric: int = 0, axes: int = 7,
                eps: np.ndarray = None):
    """Tessellation pattern (Sec. 3.4, the Voronoi polycrystal of Fig. 2c):
    each node takes the value of its nearest seed.

    reading: the distance is the standard Euclidean one (metric 0) or one of
    the extensions the paper names, absolute (1) and maximum (2).  Per axis
    the separation of x = i h from the seed coordinate c is |x - c| on an
    open axis and the smallest of |d|, |d - L|, |d + L| (d = x - c, L = n h)
    on a periodic one; axes outside the bit mask `axes` contribute 0.
    Metric 0 compares (dx^2 + dy^2) + dz^2, metric 1 (dx + dy) + dz,
    metric 2 max(max(dx, dy), dz), in double precision without fused
    multiply-add.  Seeds are visited in index order and only a strictly
    smaller distance replaces the nearest so far (ties go to the lowest
    index).  Seeds with a non-finite coordinate are skipped; nodes with no
    finite distance keep `eps` (default all ones).  Returns (eps, owner),
    owner = -1 where no seed was taken.
    """
    nz, ny, nx = grid.shape
    seeds = np.asarray(seeds, dtype=np.float64).reshape(-1, 3)
    values = np.asarray(values, dtype=np.float64).reshape(-1)
    out = np.ones(grid.shape) if eps is None else np.array(eps, dtype=np.float64)
    best = np.full(grid.shape, np.inf)
    owner = np.full(grid.shape, -1, dtype=np.int64)
    ns = (nx, ny, nz)
    hs = (grid.hx, grid.hy, grid.hz)
    coord = [np.arange(ns[a], dtype=np.float64) * hs[a] for a in range(3)]
    shape_of = [(1, 1, nx), (1, ny, 1), (nz, 1, 1)]
    for s in range(seeds.shape[0]):
        if not np.all(np.isfinite(seeds[s])):
            continue
        sep = []
        for a in range(3):
            if not (axes >> a) & 1:
                sep.append(np.zeros(shape_of[a]))
                continue
            d = coord[a] - seeds[s, a]
            sa = np.abs(d)
            if not grid.open_[a]:
                L = ns[a] * hs[a]
                sa = np.minimum(sa, np.minimum(np.abs(d - L), np.abs(d + L)))
            sep.append(sa.reshape(shape_of[a]))
        dx, dy, dz = sep
        if metric == 0:
            dist = (dx * dx + dy * dy) + dz * dz
        elif metric == 1:
            dist = (dx + dy) + dz
        else:
            dist = np.maximum(np.maximum(dx, dy), dz)
        closer = dist < best
        best = np.where(closer, dist, best)
        owner = np.where(closer, s, owner)
    taken = owner >= 0
    out[taken] = values[owner[taken]]
    return out, owner


def cut_neighbour_sum(grid: Grid, links, mask, psi):
    """Insulating inclusions (Sec. 3.4, item (ii): no-current boundary
    conditions across the internal edges that bound them).

    reading: every edge with an insulating end (mask != 0) is removed from
    the covariant Laplacian, psi is 0 on insulating nodes and their rows are
    not part of the system (the scalar potential's equation is left on the
    full grid: only the supercurrent is cut).  Returns (NS, D): the sum over
    each superconducting node's remaining edges of w_e c_a U_e psi_n and of
    w_e c_a (w_e = 2 for the inner edge of an open outer face node), so that
    L_cut psi = NS - D psi; both are 0 on insulating nodes."""
    m8 = np.ascontiguousarray(np.asarray(mask).reshape(grid.shape) != 0, dtype=np.uint8)
    out = np.empty(grid.shape, np.complex128)
    dsum = np.empty(grid.shape, np.float64)
    G = grid.c()
    _load().orc_cut_neighbour_sum(ctypes.byref(G), *map(_p, links), _p(m8), _p(_c128(psi)),
                                  _p(out), _p(dsum))
    return out, dsum


def cut_laplacian(grid: Grid, links, mask, psi):
    """Covariant Laplacian with the insulator-bounding edges cut out."""
    ns, d = cut_neighbour_sum(grid, links, mask, psi)
    return ns - d * _c128(psi)


def cut_assemble(grid: Grid, links, mask, psi_prev, eps, mu, u, ht):
    """b and diag(M) of Eq. GL_linearized / Eq. b for the cut operator: on a
    superconducting node the 2S of the uncut diagonal becomes the node's own
    sum D_m of remaining edge coefficients; insulating rows hold the trivial
    equation psi = 0 (b = 0, M_mm = 1, no neighbours)."""
    psi_prev = _c128(psi_prev)
    ns, d = cut_neighbour_sum(grid, links, mask, psi_prev)
    lap = ns - d * psi_prev
    eps = _f64(eps)
    mu_ = np.zeros(grid.shape) if mu is None else _f64(mu)
    a2 = psi_prev.real ** 2 + psi_prev.imag ** 2
    b = psi_prev + 0.5 * ht * ((eps - 1j * u * mu_) * psi_prev - a2 * psi_prev + lap)
    diag = 1.0 + 0.5 * ht * (a2 + d + 1j * u * mu_ - eps)
    ins = np.asarray(mask).reshape(grid.shape) != 0
    b[ins] = 0.0
    diag[ins] = 1.0
    return b, diag


def cut_jacobi_sweep(grid: Grid, links, mask, b, diag, ht, psi_in):
    """One iteration of Eq. final for the cut system; returns (psi_out, max
    |r(psi_in)|^2) with r = M_mm (psi_out - psi_in) as for the uncut sweep."""
    ns, _ = cut_neighbour_sum(grid, links, mask, psi_in)
    out = (b + 0.5 * ht * ns) / diag
    r = diag * (out - psi_in)
    return out, float(np.max(r.real ** 2 + r.imag ** 2))


def cut_jav(grid: Grid, links, mask, psi):
    """J_av of Sec. 3.1.1 over the x edges that remain: (1 / (N hx)) times
    the sum of Im[psi*_m U_x psi_{m+x}] over edges with two superconducting
    ends (periodic x, the one-sided form of the same sum)."""
    if grid.open_[0]:
        raise ValueError("a current along x needs a periodic x axis")
    ins = np.asarray(mask).reshape(grid.shape) != 0
    keep = ~ins & ~np.roll(ins, -1, axis=2)
    psi = _c128(psi)
    t = np.imag(np.conj(psi) * links[0] * np.roll(psi, -1, axis=2))
    return float(np.sum(np.where(keep, t, 0.0))) / (grid.N * grid.hx)


def cut_poisson_rhs(grid: Grid, links, mask, psi):
    """Right side of the Poisson equation of Sec. 3.2 with the cut operator:
    f_m = Im[psi*_m (L_cut psi)_m] = Im[psi*_m NS_m] (the D_m |psi_m|^2 part
    is real)."""
    ns, _ = cut_neighbour_sum(grid, links, mask, psi)
    return np.imag(np.conj(_c128(psi)) * ns)


# A candidate whose box reaches farther than 2^50 node spacings from the
# origin (or holds a non-finite number) covers nothing.
INCL_REACH = 2.0 ** 50


def gen_shapes(grid: Grid, shapes: np.ndarray, target: float, eps_in: float = -1.0, eps_out: float = 1.0):
    """Inclusions of general convex shape (Sec. 3.4; the ellipsoids and
    tilted columns of Fig. 2d/e), added in order until the covered node
    count reaches target * N, as for spheres.

    reading: candidate s is (c, Q, n, hlen, ext) (16 doubles); a node image
    u is inside iff, with d = u h - c,
        q = (((Qxx dx) dx + (Qyy dy) dy) + (Qzz dz) dz)
            + 2 (((Qxy dx) dy + (Qxz dx) dz) + (Qyz dy) dz) <= 1
    and, when hlen >= 0, |(nx dx + ny dy) + nz dz| <= hlen, in double
    precision without fused multiply-add.  The images tested are those of
    the box c +- ext with a one-node margin, clipped on open axes and kept
    within one period of the centre on periodic axes.  Returns (eps,
    shapes_used, covered_fraction).
    """
    nz, ny, nx = grid.shape
    N = grid.N
    covered = np.zeros(grid.shape, dtype=bool)
    count = 0
    used = 0
    ns = (nx, ny, nz)
    hs = (grid.hx, grid.hy, grid.hz)
    need = target * float(N)
    shapes = np.asarray(shapes, dtype=np.float64).reshape(-1, 16)
    if need > 0:
        for s in range(shapes.shape[0]):
            sh = shapes[s]
            used = s + 1
            if not (np.all(np.abs(sh) < 1e30) and np.all(sh[13:16] >= 0)
                    and np.all(np.abs(sh[0:3]) + sh[13:16] <= INCL_REACH * np.asarray(hs))):
                continue
            idx, off = [], []
            for a in range(3):
                c, e = sh[a], sh[13 + a]
                lo = int(np.floor((c - e) / hs[a])) - 1
                hi = int(np.ceil((c + e) / hs[a])) + 1
                if grid.open_[a]:
                    lo, hi = max(lo, 0), min(hi, ns[a] - 1)
                else:
                    cc = int(np.floor(c / hs[a]))
                    lo, hi = max(lo, cc - ns[a] - 1), min(hi, cc + ns[a] + 1)
                uu = np.arange(lo, hi + 1, dtype=np.int64)
                idx.append(np.mod(uu, ns[a]))
                off.append(uu.astype(np.float64) * hs[a] - c)
            if all(len(x) for x in idx):
                dx = off[0][None, None, :]
                dy = off[1][None, :, None]
                dz = off[2][:, None, None]
                qxx, qyy, qzz, qxy, qxz, qyz = sh[3:9]
                q = (((qxx * dx) * dx + (qyy * dy) * dy) + (qzz * dz) * dz) + \
                    2.0 * (((qxy * dx) * dy + (qxz * dx) * dz) + (qyz * dy) * dz)
                inside = q <= 1.0
                if sh[12] >= 0:
                    inside &= np.abs((sh[9] * dx + sh[10] * dy) + sh[11] * dz) <= sh[12]
                kk, jj, ii = np.nonzero(inside)
                K_, J_, I_ = idx[2][kk], idx[1][jj], idx[0][ii]
                newly = ~covered[K_, J_, I_]
                sel = np.unique(np.stack([K_[newly], J_[newly], I_[newly]]), axis=1)
                covered[sel[0], sel[1], sel[2]] = True
                count += sel.shape[1]
            if count >= need:
                break
    eps = np.where(covered, eps_in, eps_out).astype(np.float64)
    return eps, used, count / N


def gen_inclusions(grid: Grid, centers: np.ndarray, diameters: np.ndarray,
                   target: float, eps_in: float = -1.0, eps_out: float = 1.0):
    """Random spherical inclusions modulating eps (Sec. 3.4, item (i); random
    arrangement of spheres, Sec. 3.4 second paragraph).

    reading: candidate spheres (centre, diameter) are taken in the given
    order; sphere s is added and the covered-node count updated until
    count >= target * N.  A node is inside a sphere iff, for some periodic
    image of the node, ((dx*dx + dy*dy) + dz*dz) <= (d/2)*(d/2) in double
    precision without fused multiply-add, where dx = u*hx - cx with u the
    node's (unwrapped) integer coordinate.  Open axes are clipped, not
    wrapped.  Returns (eps, spheres_used, covered_fraction).
    """
    nz, ny, nx = grid.shape
    N = grid.N
    covered = np.zeros(grid.shape, dtype=bool)
    count = 0
    used = 0
    ns = (nx, ny, nz)
    hs = (grid.hx, grid.hy, grid.hz)
    need = target * float(N)
    if need > 0:
        for s in range(len(diameters)):
            c = centers[s]
            r = 0.5 * float(diameters[s])
            r2 = r * r
            used = s + 1
            if not (r >= 0.0 and r < 1e30):
                continue
            rng_idx = []
            rng_off = []
            ok = True
            for a in range(3):
                if not abs(c[a]) + r <= INCL_REACH * hs[a]:
                    ok = False
                    break
                lo = int(np.floor((c[a] - r) / hs[a])) - 1
                hi = int(np.ceil((c[a] + r) / hs[a])) + 1
                uu = np.arange(lo, hi + 1, dtype=np.int64)
                if grid.open_[a]:
                    uu = uu[(uu >= 0) & (uu < ns[a])]
                d = uu.astype(np.float64) * hs[a] - c[a]
                rng_idx.append(np.mod(uu, ns[a]))
                rng_off.append(d)
                if len(uu) == 0:
                    ok = False
            used = s + 1
            if ok:
                dx2 = rng_off[0] * rng_off[0]
                dy2 = rng_off[1] * rng_off[1]
                dz2 = rng_off[2] * rng_off[2]
                d2 = (dx2[None, None, :] + dy2[None, :, None]) + dz2[:, None, None]
                inside = d2 <= r2
                kk, jj, ii = np.nonzero(inside)
                K_ = rng_idx[2][kk]
                J_ = rng_idx[1][jj]
                I_ = rng_idx[0][ii]
                newly = ~covered[K_, J_, I_]
                # duplicates within one sphere (images mapping to one node)
                sel = np.unique(np.stack([K_[newly], J_[newly], I_[newly]]), axis=1)
                covered[sel[0], sel[1], sel[2]] = True
                count += sel.shape[1]
            if count >= need:
                break
    eps = np.where(covered, eps_in, eps_out).astype(np.float64)
    return eps, used, count / N
