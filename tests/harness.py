"""Shared set-up for GPU-vs-oracle parity tests: the same seeded inputs go to
the HIP path (through the C ABI) and to the FP64 oracle."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O
from paper_1409_8340_amd import inputs, tdgl

OPEN = tdgl.TDGL_OPEN
PER = tdgl.TDGL_PERIODIC


def bc_codes(open_):
    return tuple(OPEN if o else PER for o in open_)


def rel_maxerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


class Case:
    """One instance: grid, field, current, eps and initial state."""

    def __init__(self, nx, ny, nz, h=0.5, open_=(False, False, True), g=1.0, Bx=0.0, Bz=0.1,
                 J=0.0, driven=False, tol=1e-12, max_iter=200, mu_tol=1e-6, mu_max_cycles=40,
                 psi_seed=11, eps=None, mu0=None, K0=0.0, dt=0.1, u=1.0, hx=None, hy=None,
                 hz=None, tile_cz=0, noise_T=0.0, noise_seed=0):
        self.grid = O.Grid(nx, ny, nz, hx or h, hy or h, hz or h, tuple(open_), g)
        self.Bx, self.Bz = O.quantize_field(self.grid, Bx, Bz)
        self.J = J
        self.driven = driven
        self.params = tdgl.make_params(nx, ny, nz, h=h, hx=hx, hy=hy, hz=hz, bc=bc_codes(open_), g=g,
                                       u=u, dt=dt, tol=tol, max_iter=max_iter, driven=driven,
                                       mu_tol=mu_tol, mu_max_cycles=mu_max_cycles, tile_cz=tile_cz,
                                       noise_T=noise_T, noise_seed=noise_seed)
        self.noise_T, self.noise_seed = noise_T, noise_seed
        self.psi0 = inputs.psi_init(nx, ny, nz, psi_seed)
        self.eps = (np.ones(self.grid.shape, np.float32) if eps is None
                    else np.asarray(eps, np.float32).reshape(self.grid.shape))
        self.mu0 = None if mu0 is None else np.asarray(mu0, np.float32).reshape(self.grid.shape)
        self.K0 = K0
        self.dt, self.u = dt, u

    # ---- oracle side
    def oracle_params(self, mode="exact", tol=None):
        return O.Params(Bx=self.Bx, Bz=self.Bz, J_ext=self.J, u=self.u, dt=self.dt,
                        tol=self.params.tol if tol is None else tol, max_iter=self.params.max_iter,
                        mode=mode, driven=self.driven, noise_T=self.noise_T, noise_seed=self.noise_seed)

    def oracle_state(self):
        st = O.new_state(self.grid, self.psi0.astype(np.complex128))
        if self.mu0 is not None:
            st.mu = self.mu0.astype(np.float64).copy()
        st.K = self.K0
        return st

    # ---- GPU side
    def solver(self):
        import torch
        s = tdgl.Solver(self.params)
        self.load_into(s, 0)
        return s

    def load_into(self, s, inst):
        import torch
        bx, bz = s.set_field(self.Bx, self.Bz, inst=inst, quantize=False)
        assert bx == self.Bx and bz == self.Bz
        if self.driven:
            s.set_current(self.J, inst=inst)
        s.set_eps(torch.from_numpy(self.eps).cuda(), inst=inst)
        s.set_psi(torch.from_numpy(self.psi0).cuda(), inst=inst)
        if self.mu0 is not None:
            s.set_mu(torch.from_numpy(self.mu0).cuda(), inst=inst)
        if self.K0:
            sc = s.get_scalars(inst)
            sc["K"] = self.K0
            s.set_scalars(sc, inst)
