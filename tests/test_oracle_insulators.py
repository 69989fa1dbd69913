"""Pins of the oracle's insulating inclusions (Sec. 3.4, item (ii): no-current
boundary conditions across the internal edges that bound them).  The oracle
cuts those edges out of the covariant Laplacian in plain FP64 and holds psi
= 0 on insulating nodes; these tests pin it to a dense operator written edge
by edge, to LAPACK solves of the cut system and to states the cut cannot
change.  CPU only."""
import itertools

import numpy as np
import pytest

from oracle import brute
from oracle import oracle as O
from paper_1409_8340_amd import inputs

MIXES = list(itertools.product([False, True], repeat=3))


def _ids(o):
    return "open" + "".join("xyz"[a] for a in range(3) if o[a]) or "periodic"


def _mask(grid, seed, frac=0.25):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.random(grid.shape) < frac


def _field(grid, open_):
    Bx, Bz = O.quantize_field(grid, 0.37, 0.41)
    if open_[1] or open_[2]:
        Bx = 0.23
    if open_[0] or open_[1]:
        Bz = 0.31
    return Bx, Bz


@pytest.mark.parametrize("open_", MIXES, ids=_ids)
def test_cut_operator_equals_dense(open_):
    """The oracle's cut Laplacian equals the dense operator with every edge
    touching an insulating node removed, for any psi (insulating rows and
    columns are zero), on every boundary mix with g != 1."""
    grid = O.Grid(5, 4, 3, 0.5, 0.6, 0.45, open_, g=1.3)
    Bx, Bz = _field(grid, open_)
    K = 0.2
    mask = _mask(grid, 1)
    psi = inputs.random_complex(grid.shape, 3, 1.0).astype(np.complex128)
    links = O.with_K(O.landau_links(grid, Bx, Bz, 0.0), grid.hx, K)
    Lcut = brute.laplacian_matrix_cut(grid, Bx, Bz, K, mask)
    got = O.cut_laplacian(grid, links, mask, psi).reshape(-1)
    np.testing.assert_allclose(got, Lcut @ psi.reshape(-1), rtol=0, atol=1e-12)
    # an empty mask gives back the uncut operator
    none = np.zeros(grid.shape, bool)
    np.testing.assert_allclose(O.cut_laplacian(grid, links, none, psi),
                               O.laplacian(grid, links, psi), rtol=0, atol=1e-12)


@pytest.mark.parametrize("open_", MIXES, ids=_ids)
def test_one_step_equals_the_cut_system_solved_densely(open_):
    """One exact-mode step of the oracle with insulators equals the
    linearised Crank-Nicolson step of the cut system (Eq. GL_linearized with
    the cut Laplacian) solved by LAPACK on the superconducting nodes; psi is
    exactly 0 on the insulating ones."""
    grid = O.Grid(6, 5, 4, 0.5, 0.55, 0.5, open_, g=1.2)
    Bx, Bz = _field(grid, open_)
    mask = _mask(grid, 7, 0.2)
    eps = inputs.random_real(grid.shape, 8, 0.3, 1.0).astype(np.float64)
    psi0 = inputs.psi_init(6, 5, 4, 9).astype(np.complex128)
    p = O.Params(Bx=Bx, Bz=Bz, tol=1e-14, mode="exact", insulators=mask)
    st = O.new_state(grid, psi0)
    O.step(grid, p, eps, st)
    ht = p.dt / p.u
    L = brute.laplacian_matrix_cut(grid, Bx, Bz, 0.0, mask)
    sc = ~mask.reshape(-1)
    pm = np.where(sc, psi0.reshape(-1), 0.0)
    e = eps.reshape(-1)
    a2 = np.abs(pm) ** 2
    M = np.diag(1.0 + 0.5 * ht * (a2 - e)) - 0.5 * ht * L
    b = pm + 0.5 * ht * (e * pm - a2 * pm + L @ pm)
    x = np.linalg.solve(M[np.ix_(sc, sc)], b[sc])
    np.testing.assert_allclose(st.psi.reshape(-1)[sc], x, rtol=0, atol=1e-12)
    assert np.all(st.psi.reshape(-1)[~sc] == 0)


def test_driven_step_with_a_scalar_potential_equals_dense():
    """A driven step (mu~ from the previous step in M and b, then J_av, K and
    the Poisson right side) against dense algebra of the cut system."""
    grid = O.Grid(6, 5, 4, 0.5, 0.5, 0.5, (False, False, True))
    Bz = O.quantize_field(grid, 0.0, 0.4)[1]
    mask = _mask(grid, 3, 0.2)
    eps = inputs.random_real(grid.shape, 4, 0.3, 1.0).astype(np.float64)
    mu0 = inputs.random_real(grid.shape, 5, -0.2, 0.2).astype(np.float64)
    psi0 = inputs.psi_init(6, 5, 4, 6).astype(np.complex128)
    K0, J, u, dt = 0.3, 0.04, 1.0, 0.1
    p = O.Params(Bz=Bz, J_ext=J, tol=1e-14, mode="exact", driven=True, insulators=mask)
    st = O.new_state(grid, psi0)
    st.mu = mu0.copy()
    st.K = K0
    O.step(grid, p, eps, st)
    ht = dt / u
    sc = ~mask.reshape(-1)
    L = brute.laplacian_matrix_cut(grid, 0.0, Bz, K0, mask)
    pm = np.where(sc, psi0.reshape(-1), 0.0)
    e, m_ = eps.reshape(-1), mu0.reshape(-1)
    a2 = np.abs(pm) ** 2
    M = np.diag(1.0 + 0.5 * ht * (a2 + 1j * u * m_ - e)) - 0.5 * ht * L
    b = pm + 0.5 * ht * ((e - 1j * u * m_) * pm - a2 * pm + L @ pm)
    x = np.zeros(grid.N, np.complex128)
    x[sc] = np.linalg.solve(M[np.ix_(sc, sc)], b[sc])
    np.testing.assert_allclose(st.psi.reshape(-1), x, rtol=0, atol=1e-12)
    # J_av over the remaining x edges, edge by edge
    jav = 0.0
    for k in range(grid.nz):
        for j in range(grid.ny):
            for i in range(grid.nx):
                m = i + grid.nx * (j + grid.ny * k)
                n = (i + 1) % grid.nx + grid.nx * (j + grid.ny * k)
                if sc[m] and sc[n]:
                    U = brute.link(grid, 0, i, j, k, 0.0, Bz, K0)
                    jav += np.imag(np.conj(x[m]) * U * x[n])
    jav /= grid.N * grid.hx
    assert abs(st.last_Jav - jav) < 1e-13
    K1 = O.rewind_K(K0 + dt * (J - jav), grid.hx)
    assert abs(st.K - K1) < 1e-13
    # Poisson right side Im[psi* L_cut psi] at the new K, weighted mean zero
    L1 = brute.laplacian_matrix_cut(grid, 0.0, Bz, K1, mask)
    f = np.imag(np.conj(x) * (L1 @ x))
    assert abs(float(np.sum(brute.weights(grid) * f))) < 1e-12 * max(1.0, np.abs(f).sum())
    np.testing.assert_allclose(O.poisson_apply(grid, st.mu).reshape(-1), f, rtol=0, atol=1e-10)


def test_uniform_state_is_untouched_by_voids():
    """B = 0, eps = 1: psi = 1 on the superconducting nodes stays a fixed
    point next to insulating voids (no current through their surface, so no
    suppression), while the same voids modelled as psi = 0 boundaries of the
    uncut operator suppress psi around them."""
    grid = O.Grid(12, 10, 8, open_=(False, False, True))
    c, d = inputs.sphere_candidates([grid.length(a) for a in range(3)], 6, 4, law="fixed", d=2.5)
    cover, _, _ = O.gen_inclusions(grid, c, d, 0.15)
    mask = cover < 0
    assert mask.any()
    psi0 = np.where(mask, 0.0, 1.0).astype(np.complex128)
    p = O.Params(Bx=0.0, Bz=0.0, tol=1e-14, mode="exact", insulators=mask)
    st = O.new_state(grid, psi0)
    O.run(grid, p, np.ones(grid.shape), st, 5)
    assert np.max(np.abs(st.psi[~mask] - 1)) < 1e-12
    assert np.all(st.psi[mask] == 0)
    st2 = O.new_state(grid, psi0)
    O.run(grid, O.Params(Bx=0.0, Bz=0.0, tol=1e-14, mode="exact"), np.ones(grid.shape), st2, 5)
    assert np.max(np.abs(st2.psi[~mask] - 1)) > 1e-3


def test_current_carrying_state_across_insulating_layers():
    """Insulating planes normal to z cut only z edges.  The uniform
    current-carrying state psi = a (B = 0, x links exp(i hx K)) with
    a^2 = eps - (2 - 2 cos hx K)/hx^2 is stationary and carries
    J_av = (fraction of superconducting nodes) a^2 sin(hx K)/hx: the cut
    z edges change neither."""
    grid = O.Grid(8, 6, 9, open_=(False, False, True))
    mask = np.zeros(grid.shape, bool)
    mask[3] = True          # two insulating planes, k = 3 and k = 6
    mask[6] = True
    K, hx = 0.4, grid.hx
    a2 = 1.0 - (2 - 2 * np.cos(hx * K)) / hx ** 2
    psi0 = np.where(mask, 0.0, np.sqrt(a2)).astype(np.complex128)
    p = O.Params(tol=1e-14, mode="exact", insulators=mask)
    st = O.new_state(grid, psi0)
    links = O.with_K(O.landau_links(grid, 0.0, 0.0, 0.0), hx, K)
    base = O.landau_links(grid, 0.0, 0.0, 0.0)
    st.K = K
    O.step(grid, p, np.ones(grid.shape), st, base_links=base)
    np.testing.assert_allclose(st.psi, psi0, rtol=0, atol=1e-13)
    frac = 1 - mask.mean()
    assert abs(O.cut_jav(grid, links, mask, st.psi) - frac * a2 * np.sin(hx * K) / hx) < 1e-14
