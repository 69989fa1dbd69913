"""FP64 reverse-mode derivative of the time-averaged voltage with respect to
the pinning landscape eps(r), for the implicit step of oracle.step.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (same rules as oracle.py).

Loss: Vbar = (1/W) sum_{n in window} E_n,  E_n = J_ext - J_av(psi_n, K_{n-1}).

Convention for complex variables: for a real loss L the adjoint of z is
zbar = dL/dRe z + i dL/dIm z, so that dL = Re sum conj(zbar) dz.

One step maps (psi^-, mu^-, K^-) -> (psi, mu, K) (Sec. 4.1 order):
  psi = M^-1 b                     (Eq. GL_linearized, Eq. b; exact solve)
  J   = J_av(psi, K^-)             (Sec. 3.1.1)
  E   = J_ext - J
  K   = rewind(K^- + dt E)          (Eq. K_ODE; the rewind has derivative 1)
  f   = Im[conj(psi) NS(psi; K)]    (Sec. 3.2 right side)
  mu  = G f                        (exact Poisson solve, zero weighted mean)
Its reverse, given the adjoints of (psi, mu, K) and the loss weight of E:
  fbar   = G^T mubar = W G(W^-1 mubar)      (Delta_h is W-self-adjoint)
  psibar += -i fbar NS(psi) + i NS^H(fbar psi),  Kbar += fbar . df/dK
  Kbar^- += Kbar,  Ebar = dt Kbar + (loss weight),  Jbar = -Ebar
  psibar += -i Jbar T psi / (N hx),  Kbar^- += Jbar dJ/dK
  lambda = M^-H psibar   (solved as M~ nu = W^-1 psibar, lambda = W nu,
                          M~ = M with conjugated diagonal, NS^H = W NS W^-1)
  epsbar += (ht/2) Re[conj(lambda)(psi^- + psi)]
  mubar^- = (u ht/2) Im[conj(lambda)(psi^- + psi)]
  Kbar^- += (ht/2) Re sum conj(lambda) dNS/dK (psi^- + psi)
  psibar^- = conj(alpha) lambda + beta conj(lambda) + (ht/2) L^H lambda,
     alpha = 1 + (ht/2)(eps - i u mu^-) - ht |psi^-|^2 - (ht/2) conj(psi^-) psi,
     beta  = -(ht/2) (psi^-)^2 - (ht/2) psi^- psi.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def ns(grid, links, x):
    return O.neighbour_sum(grid, links, x)


def ns_h(grid, links, w, x):
    """Conjugate transpose of the neighbour sum: W NS W^-1 (W NS is
    Hermitian for every boundary kind)."""
    return w * O.neighbour_sum(grid, links, x / w)


def dns_dK(grid, links, x):
    """Derivative of NS(x; K) with respect to K (x links carry e^{i hx K});
    x must be periodic (the driven case)."""
    lx = links[0]
    fwd = lx * np.roll(x, -1, axis=2)
    bwd = np.conj(np.roll(lx, 1, axis=2)) * np.roll(x, 1, axis=2)
    return (1j * grid.hx / (grid.hx * grid.hx)) * (fwd - bwd)


def tshift(links, x):
    """T x = U x_{+x} - conj(U_{-x}) x_{-x} (periodic x)."""
    lx = links[0]
    return lx * np.roll(x, -1, axis=2) - np.conj(np.roll(lx, 1, axis=2)) * np.roll(x, 1, axis=2)


def poisson_T(grid, w, g):
    """Transpose of the exact Poisson solve: W G(W^-1 g)."""
    return w * O.poisson_exact(grid, g / w)


def forward(grid, p, eps, st0, nsteps, base_links=None):
    """Run nsteps exact steps from st0 (copied) and keep every state."""
    if base_links is None:
        base_links = O.base_links_of(grid, p)
    st = O.State(psi=st0.psi.copy(), mu=st0.mu.copy(), K=st0.K)
    states = [(st.psi.copy(), st.mu.copy(), st.K)]
    Es = []
    q = O.Params(**{**p.__dict__, "mode": "exact"})
    for _ in range(nsteps):
        O.step(grid, q, eps, st, base_links=base_links)
        states.append((st.psi.copy(), st.mu.copy(), st.K))
        Es.append(st.last_E)
    return states, Es


def step_vjp(grid, p, eps, prev, nxt, psibar, mubar, Kbar, Ebar_loss, base_links, w):
    """Reverse of one step.  prev, nxt: (psi, mu, K) before and after.
    Returns (psibar^-, mubar^-, Kbar^-, epsbar)."""
    ht = p.dt / p.u
    u = p.u
    psim, mum, Km = prev
    psi, mu, K = nxt
    links_m = O.with_K(base_links, grid.hx, Km)
    links_n = O.with_K(base_links, grid.hx, K)
    N = grid.N
    psibar = psibar.astype(np.complex128).copy()
    Kbar_m = 0.0
    if p.driven:
        # Poisson and its right side (links at K_n)
        fbar = poisson_T(grid, w, mubar)
        psibar += -1j * fbar * ns(grid, links_n, psi) + 1j * ns_h(grid, links_n, w, fbar * psi)
        Kbar_n = Kbar + float(np.sum(fbar * np.imag(np.conj(psi) * dns_dK(grid, links_n, psi))))
        # K update and the loss
        Kbar_m = Kbar_n
        Ebar = p.dt * Kbar_n + Ebar_loss
        Jbar = -Ebar
        # J_av(psi, K^-)
        psibar += -1j * Jbar * tshift(links_m, psi) / (N * grid.hx)
        dJdK = float(np.sum(np.real(np.conj(psi) * (links_m[0] * np.roll(psi, -1, axis=2)
                                                    + np.conj(np.roll(links_m[0], 1, axis=2))
                                                    * np.roll(psi, 1, axis=2))))) / (2.0 * N)
        Kbar_m += Jbar * dJdK
    # the implicit CN solve
    mu_use = mum if p.driven else None
    _, diag = O.assemble(grid, links_m, psim, eps, mu_use, u, ht)
    nu, _, _ = O.gl_solve(grid, links_m, psibar / w, np.conj(diag), ht, np.zeros_like(psibar), 0.0, 0,
                          "exact")
    lam = w * nu
    s = psim + psi
    epsbar = 0.5 * ht * np.real(np.conj(lam) * s)
    mubar_m = 0.5 * u * ht * np.imag(np.conj(lam) * s) if p.driven else np.zeros(grid.shape)
    if p.driven:
        Kbar_m += 0.5 * ht * float(np.real(np.sum(np.conj(lam) * dns_dK(grid, links_m, s))))
    a2 = np.abs(psim) ** 2
    mu_term = mum if p.driven else 0.0
    alpha = 1 + 0.5 * ht * (eps - 1j * u * mu_term) - ht * a2 - 0.5 * ht * np.conj(psim) * psi
    beta = -0.5 * ht * psim * psim - 0.5 * ht * psim * psi
    lap_h = w * O.laplacian(grid, links_m, lam / w)
    psibar_m = np.conj(alpha) * lam + beta * np.conj(lam) + 0.5 * ht * lap_h
    return psibar_m, mubar_m, Kbar_m, epsbar


def voltage_grad(grid, p, eps, st0, nsteps, window_begin=0):
    """dVbar/deps for Vbar = mean of E_n over steps n >= window_begin
    (0-based within the run), exact forward.  Returns (Vbar, grad)."""
    base = O.base_links_of(grid, p)
    states, Es = forward(grid, p, eps, st0, nsteps, base)
    W = nsteps - window_begin
    Vbar = float(np.mean(Es[window_begin:]))
    w = O.node_weights(grid)
    psibar = np.zeros(grid.shape, np.complex128)
    mubar = np.zeros(grid.shape)
    Kbar = 0.0
    grad = np.zeros(grid.shape)
    for n in range(nsteps, 0, -1):
        ew = 1.0 / W if (n - 1) >= window_begin else 0.0
        psibar, mubar, Kbar, eb = step_vjp(grid, p, eps, states[n - 1], states[n], psibar, mubar, Kbar,
                                           ew, base, w)
        grad += eb
    return Vbar, grad
