"""Dense brute-force matrices for tiny grids, written independently of the
stencil loops in ``tdgl_oracle.c``.  TEST INFRASTRUCTURE ONLY.

Every matrix element is written out from the paper's element formulas:
  * M and b of the linearised Crank-Nicolson system (Sec. 3.1,
    Eq. GL_linearized, Eq. b) for the xz-plane field, with the link variables
    of Eq. link_variables, the quasi-periodic y wrap of Sec. 3.3.1 and the
    open-face rows of Sec. 3.3.2;
  * the Poisson operator and right side of Sec. 3.2.
The oracle's loops are checked against these with dense LAPACK solves.
"""
from __future__ import annotations

import numpy as np


def _axes(grid):
    return ((grid.nx, grid.hx, grid.open_[0], 1.0),
            (grid.ny, grid.hy, grid.open_[1], 1.0),
            (grid.nz, grid.hz, grid.open_[2], 1.0 / (grid.g * grid.g)))


def _m(grid, i, j, k):
    return i + grid.nx * (j + grid.ny * k)


def link(grid, axis, i, j, k, Bx, Bz, K):
    """Link on the edge from node (i,j,k) to its +axis neighbour, written
    from Eq. link_variables for A~ = ybar [-Bz, 0, Bx] - [K, 0, 0]:
    U_x = exp(-i hx A~_x), U_z = exp(-i hz A~_z), U_y = 1, and on the y wrap
    edge the conjugate phase jump conj(P_{i,k})."""
    Ly = grid.ny * grid.hy if not grid.open_[1] else (grid.ny - 1) * grid.hy
    ybar = j * grid.hy - Ly / 2.0
    if axis == 0:
        A = -ybar * Bz - K
        return np.exp(-1j * grid.hx * A)
    if axis == 2:
        A = ybar * Bx
        return np.exp(-1j * grid.hz * A)
    if j == grid.ny - 1 and not grid.open_[1]:
        P = np.exp(1j * (i * grid.hx * Ly * Bz - k * grid.hz * Ly * Bx))
        return np.conj(P)
    return 1.0 + 0j


def link_yz(grid, axis, i, j, k, By, Bz, K):
    """Link on the edge from node (i,j,k) to its +axis neighbour for the
    yz-plane field, written from Eq. link_variables for
    A~ = xbar [0, Bz, -By] - [K, 0, 0] (Eq. A_yz): U_x = exp(-i hx A~_x),
    U_y = exp(-i hy A~_y), U_z = exp(-i hz A~_z), and on the x wrap edge the
    conjugate phase jump conj(P_{j,k}) of the yz case of Sec. 3.3.1."""
    Lx = grid.nx * grid.hx if not grid.open_[0] else (grid.nx - 1) * grid.hx
    xbar = i * grid.hx - Lx / 2.0
    if axis == 0:
        U = np.exp(-1j * grid.hx * (-K))
        if i == grid.nx - 1 and not grid.open_[0]:
            P = np.exp(1j * (-j * grid.hy * Lx * Bz + k * grid.hz * Lx * By))
            U = U * np.conj(P)
        return U
    if axis == 1:
        return np.exp(-1j * grid.hy * (xbar * Bz))
    return np.exp(-1j * grid.hz * (-xbar * By))


def laplacian_matrix_yz(grid, By, Bz, K):
    """Dense covariant Laplacian for the yz-plane field (Eq. LaplUV_yz)."""
    return _laplacian(grid, lambda a, i, j, k: link_yz(grid, a, i, j, k, By, Bz, K))


def laplacian_matrix(grid, Bx, Bz, K):
    """Dense matrix of the covariant Laplacian with all boundary forms."""
    return _laplacian(grid, lambda a, i, j, k: link(grid, a, i, j, k, Bx, Bz, K))


def _laplacian(grid, linkf):
    N = grid.N
    L = np.zeros((N, N), dtype=np.complex128)
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                m = _m(grid, i, j, k)
                pos = (i, j, k)
                for a, (n, h, op, cf) in enumerate(_axes(grid)):
                    c = cf / (h * h)
                    if op and n == 1:
                        continue
                    L[m, m] += -2.0 * c
                    p = list(pos)
                    fwd = pos[a] + 1
                    bwd = pos[a] - 1
                    # forward neighbour, link on edge m -> m+a
                    U_f = linkf(a, *pos)
                    # backward neighbour, conj of the link on edge m-a -> m
                    pb = list(pos)
                    pb[a] = bwd % n
                    U_b = np.conj(linkf(a, *pb))
                    pf = list(pos)
                    pf[a] = fwd % n
                    if op and pos[a] == 0:
                        L[m, _m(grid, *pf)] += 2.0 * c * U_f
                    elif op and pos[a] == n - 1:
                        L[m, _m(grid, *pb)] += 2.0 * c * U_b
                    else:
                        L[m, _m(grid, *pf)] += c * U_f
                        L[m, _m(grid, *pb)] += c * U_b
    return L


def gl_system(grid, Bx, Bz, K, psi_prev, eps, mu, u, ht):
    """Dense M and vector b (Eq. GL_linearized and Eq. b, noise zero)."""
    L = laplacian_matrix(grid, Bx, Bz, K)
    p = psi_prev.reshape(-1)
    e = eps.reshape(-1)
    mu_ = np.zeros_like(e) if mu is None else mu.reshape(-1)
    a2 = np.abs(p) ** 2
    # M = 1 + (ht/2)[ |psi^-|^2 + i u mu - eps ] - (ht/2) L
    M = np.diag(1.0 + 0.5 * ht * (a2 + 1j * u * mu_ - e)) - 0.5 * ht * L
    b = p + 0.5 * ht * ((e - 1j * u * mu_) * p - a2 * p + L @ p)
    return M, b


def poisson_matrix(grid):
    """Dense 7-point Laplacian of Sec. 3.2 (wrap on periodic axes, Neumann
    reflection on open faces)."""
    N = grid.N
    A = np.zeros((N, N))
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                m = _m(grid, i, j, k)
                pos = (i, j, k)
                for a, (n, h, op, cf) in enumerate(_axes(grid)):
                    c = cf / (h * h)
                    if op and n == 1:
                        continue
                    A[m, m] -= 2.0 * c
                    pf = list(pos)
                    pf[a] = (pos[a] + 1) % n
                    pb = list(pos)
                    pb[a] = (pos[a] - 1) % n
                    if op and pos[a] == 0:
                        A[m, _m(grid, *pf)] += 2.0 * c
                    elif op and pos[a] == n - 1:
                        A[m, _m(grid, *pb)] += 2.0 * c
                    else:
                        A[m, _m(grid, *pf)] += c
                        A[m, _m(grid, *pb)] += c
    return A


def poisson_rhs(grid, Bx, Bz, K, psi):
    """f_m = sum_a (1/h_a^2) Im[psi_m^* (U psi_{m+a} + U^* psi_{m-a})], with
    the open-face ghost rule: written as Im[psi^* (L psi + 2 S psi)], i.e.
    the off-diagonal part of the dense Laplacian."""
    L = laplacian_matrix(grid, Bx, Bz, K)
    off = L - np.diag(np.diag(L))
    p = psi.reshape(-1)
    return np.imag(np.conj(p) * (off @ p))


def weights(grid):
    w = np.ones((grid.nz, grid.ny, grid.nx))
    if grid.open_[0] and grid.nx > 1:
        w[:, :, 0] *= 0.5
        w[:, :, -1] *= 0.5
    if grid.open_[1] and grid.ny > 1:
        w[:, 0, :] *= 0.5
        w[:, -1, :] *= 0.5
    if grid.open_[2] and grid.nz > 1:
        w[0] *= 0.5
        w[-1] *= 0.5
    return w.reshape(-1)


def poisson_solve(grid, f):
    """Least-squares solve of the singular Poisson system, then shift to a
    zero weighted mean."""
    A = poisson_matrix(grid)
    w = weights(grid)
    ff = f.reshape(-1) - (w @ f.reshape(-1)) / w.sum()
    mu, *_ = np.linalg.lstsq(A, ff, rcond=None)
    mu -= (w @ mu) / w.sum()
    return mu


def laplacian_matrix_cut(grid, Bx, Bz, K, mask):
    """Dense covariant Laplacian (xz-plane field) with every edge that
    touches an insulating node (mask != 0) cut out (Sec. 3.4, item (ii)),
    written edge by edge: row m of a superconducting node sums
    c_a (U psi_n - psi_m) over its remaining edges (an open face node's
    single inner edge counted twice, as in Sec. 3.3.2); rows and columns of
    insulating nodes are zero (psi = 0 there)."""
    mask = np.asarray(mask).reshape(-1) != 0
    N = grid.N
    L = np.zeros((N, N), dtype=np.complex128)
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                m = _m(grid, i, j, k)
                if mask[m]:
                    continue
                pos = (i, j, k)
                for a, (n, h, op, cf) in enumerate(_axes(grid)):
                    c = cf / (h * h)
                    if op and n == 1:
                        continue
                    for d in (-1, 1):
                        t = pos[a] + d
                        if op and (t < 0 or t >= n):
                            continue
                        q = list(pos)
                        q[a] = t % n
                        nb = _m(grid, *q)
                        if mask[nb]:
                            continue
                        if d == 1:
                            U = link(grid, a, *pos, Bx, Bz, K)
                        else:
                            U = np.conj(link(grid, a, *q, Bx, Bz, K))
                        w = 2.0 if (op and (pos[a] == 0 or pos[a] == n - 1)) else 1.0
                        L[m, nb] += w * c * U
                        L[m, m] -= w * c
    return L
