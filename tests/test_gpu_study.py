"""The trends of the paper's Jacobi study (Sec. 4, Fig. 5) on a small 2D
free-flowing film: iterations per step grow as the stop tolerance tightens
and as the spacing h shrinks (the Jacobi contraction factor of the implicit
system, h_t S / (1 + h_t S - h_t max(eps) / 2) with S = sum 1/h_a^2, rises
towards 1), and every solve stays below the Gershgorin iteration bound."""
import math

import numpy as np
import pytest

from paper_1409_8340_amd import inputs, tdgl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tdgl.load()


def _sweeps(n, h, tol, warmup=60, steps=20):
    p = tdgl.make_params(n, n, 1, h=h, driven=True, tol=tol, max_iter=256, mu_tol=1e-6, mu_max_cycles=40)
    s = tdgl.Solver(p)
    s.set_field(0.0, 0.1, quantize=True)
    s.set_current(0.02)
    s.set_psi(torch.from_numpy(inputs.psi_init(n, n, 1, 1005)).cuda())
    s.step(warmup, stats=False)
    st = s.step(steps)
    psi = s.get_psi().cpu().numpy()
    s.close()
    assert st["capped_steps"] == 0
    return st, psi


def test_iterations_grow_as_the_tolerance_tightens():
    per = []
    for tol in (1e-4, 1e-8, 1e-12):
        st, _ = _sweeps(256, 0.5, tol)
        per.append(st["sweeps_sum"] / 20)
    print("[study] sweeps per step at tol 1e-4, 1e-8, 1e-12:", per)
    assert per[0] < per[1] < per[2]


def test_iterations_grow_as_the_spacing_shrinks():
    per, bound = [], []
    for h in (1.0, 0.5, 0.3):
        st, psi = _sweeps(192, h, 1e-8)
        per.append(st["sweeps_sum"] / 20)
        # contraction factor of the Jacobi iteration (eps = 1, no pinning;
        # z is a single open plane, so S = 2 / h^2), and the number of
        # sweeps after which the residual of an increment no larger than
        # |psi| + |psi^-| <= 4 must have dropped below sqrt(tol), with the
        # diagonal's spread (1 + ht S + ht |psi|^2 / 2) / (1 + ht S - ht / 2)
        ht, S = 0.1, 2.0 / (h * h)
        rho = ht * S / (1.0 + ht * S - ht / 2.0)
        amax = float(np.max(np.abs(psi))) ** 2
        spread = (1.0 + ht * S + ht * amax / 2.0) / (1.0 + ht * S - ht / 2.0)
        m0 = 4.0 * (1.0 + ht * S + ht * amax / 2.0)
        bound.append(2 + math.ceil(math.log(math.sqrt(1e-8) / (spread * m0)) / math.log(rho)))
        assert st["sweeps_max"] <= bound[-1]
    print("[study] sweeps per step at h 1.0, 0.5, 0.3:", per, "bounds", bound)
    assert per[0] < per[1] < per[2]
