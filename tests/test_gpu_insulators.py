"""Insulating inclusions (Sec. 3.4, item (ii)) on the GPU against the FP64
oracle's cut-edge system (edges with an insulating end removed from the
covariant Laplacian, psi = 0 on insulating nodes).  The library realises the
cut as a shift of eps; nothing here compares that representation itself,
only the states both sides reach."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1409_8340_amd import inputs, tdgl
from tests.harness import Case, rel_maxerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tdgl.load()


def _voids(grid, seed, frac):
    c, d = inputs.sphere_candidates([grid.length(a) for a in range(3)], 400, seed, law="fixed", d=3.0)
    cover, _, _ = O.gen_inclusions(grid, c, d, frac)
    return cover < 0


def _oracle_run(c, mask, nsteps, st=None):
    p = c.oracle_params()
    p.insulators = mask
    if st is None:
        st = c.oracle_state()
    O.run(c.grid, p, c.eps.astype(np.float64), st, nsteps)
    return st


@pytest.mark.parametrize("shape,open_,g", [
    ((48, 40, 12), (False, False, True), 1.0),
    ((70, 37, 9), (True, False, True), 1.3),
    ((32, 24, 12), (False, False, False), 1.0),
    ((40, 30, 1), (False, False, True), 1.0),
    ((20, 2, 7), (False, True, True), 1.0),       # two-node open y: both rows are faces
])
def test_undriven_steps_with_insulators(shape, open_, g):
    """One and three undriven steps with insulating spheres on every kind of
    face (open x, periodic z, a single z plane, two-node open y, g != 1)."""
    c = Case(*shape, open_=open_, g=g)
    c.eps = inputs.random_real(c.grid.shape, 4, -0.5, 1.0)
    mask = _voids(c.grid, 17, 0.2)
    assert mask.any() and not mask.all()
    s = c.solver()
    s.set_insulators(mask)
    s.step(1)
    psi1 = s.get_psi().cpu().numpy()
    s.step(2)
    psi3 = s.get_psi().cpu().numpy()
    s.close()
    st = _oracle_run(c, mask, 1)
    e1 = rel_maxerr(psi1, st.psi)
    _oracle_run(c, mask, 2, st)
    e3 = rel_maxerr(psi3, st.psi)
    scale = float(np.max(np.abs(st.psi)))
    void = float(np.max(np.abs(psi3[mask]))) / scale
    print(f"[insulators {shape} open={open_} g={g}] psi 1 step {e1:.2e}, 3 steps {e3:.2e}, "
          f"|psi| on insulators {void:.1e}")
    assert e1 <= 1e-5
    assert e3 <= 1e-4
    assert void <= 1e-12


def test_driven_steps_with_insulating_voids():
    """Driven steps (J = 0.03): psi, K and mu~ after one and three steps."""
    c = Case(64, 48, 16, Bz=0.12, J=0.03, driven=True, tol=1e-12, mu_tol=1e-6)
    mask = _voids(c.grid, 21, 0.12)
    s = c.solver()
    s.set_insulators(mask)
    got = {}
    for n in (1, 2):
        s.step(n)
        got[n] = (s.get_psi().cpu().numpy(), s.get_mu().cpu().numpy(), s.get_scalars()["K"])
    s.close()
    st = c.oracle_state()
    for n, bar in ((1, 1e-5), (2, 1e-4)):
        _oracle_run(c, mask, n, st)
        psi_g, mu_g, K_g = got[n]
        err = rel_maxerr(psi_g, st.psi)
        mu_err = float(np.max(np.abs(mu_g - st.mu))) / max(1.0, float(np.max(np.abs(st.mu))))
        void = float(np.max(np.abs(psi_g[mask])))
        print(f"[insulators driven, {st.n} steps] psi {err:.2e}, mu {mu_err:.2e}, K {K_g:.9f} vs {st.K:.9f}, "
              f"|psi| on voids {void:.1e}")
        assert err <= bar
        assert abs(K_g - st.K) <= 1e-6
        assert mu_err <= 1e-4
        assert void <= 1e-12


def test_second_call_on_the_same_eps_is_refused():
    """The cut shares go into eps once: a second call before eps is set again
    is refused, and setting eps re-arms the call."""
    c = Case(16, 12, 6)
    mask = _voids(c.grid, 5, 0.1)
    s = c.solver()
    s.set_insulators(mask)
    with pytest.raises(tdgl.TdglError):
        s.set_insulators(mask)
    s.set_eps(torch.from_numpy(c.eps).cuda())
    s.set_insulators(mask)
    s.close()
