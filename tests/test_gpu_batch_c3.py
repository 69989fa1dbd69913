"""The batched workload against the FP64 oracle: 64 instances in one context
(shapes drawn from {64^3, 96x96x48, 128x128x32}, B ~ U[0.05, 0.3] along z,
J ~ U[0, 0.05] along x, one inclusion diameter ~ U[2, 6] and fraction
~ U[0.05, 0.20] per instance, eps = -1 / +1).  Sampled instances -- per shape
the one with the largest J, and the one with the largest B -- are compared
with the oracle run on that instance alone:
  * after one step from the seeded state (tight Jacobi tolerance on both
    sides, exact oracle solve): psi, mu~ and K;
  * over the workload's 1000 steps at its Jacobi stop rule (max|r|^2 < 1e-8;
    the oracle in mirror mode with the same rule), the batch advanced by
    graph-replayed steps after 50 eager ones: E_x of the first 50 steps, and
    the time-averaged field over all 1000 steps and over the last 200,
    against tests/golden/c3_batch_oracle.json (written by
    tests/golden/make_c3_batch.py from oracle/ only).
A driven vortex run has no closed form: parity unpinned beyond the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1409_8340_amd import inputs, tdgl
from tests.harness import rel_maxerr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_batch_oracle.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    tdgl.load()


def _picks(ws):
    picks = []
    for shape in sorted({(w.nx, w.ny, w.nz) for w in ws}):
        cand = [i for i, w in enumerate(ws) if (w.nx, w.ny, w.nz) == shape]
        picks.append(max(cand, key=lambda i: ws[i].J))
    for i in sorted(range(len(ws)), key=lambda i: -ws[i].B):
        if i not in picks:
            picks.append(i)
            break
    return picks


def _batch(tol, max_iter):
    ws = inputs.batch_workloads()
    params = [tdgl.make_params(w.nx, w.ny, w.nz, h=w.h, driven=True, tol=tol, max_iter=max_iter, dt=w.dt)
              for w in ws]
    s = tdgl.Solver(params)
    for i, w in enumerate(ws):
        s.set_field(0.0, w.B, inst=i, quantize=True)
        s.set_current(w.J, inst=i)
        cen, dia = inputs.candidates_for(w)
        s.gen_inclusions(cen, dia, w.fraction, w.eps_in, w.eps_out, inst=i)
        s.set_psi(torch.from_numpy(inputs.psi_init(w.nx, w.ny, w.nz, w.psi_seed)).cuda(), inst=i)
    return s, ws


def test_c3_one_step_sampled_instances_vs_oracle():
    s, ws = _batch(1e-12, 250)
    picks = _picks(ws)
    s.step(1)
    got = {i: (s.get_psi(i).cpu().numpy(), s.get_mu(i).cpu().numpy(), s.get_scalars(i)["K"]) for i in picks}
    s.close()
    for i in picks:
        w = ws[i]
        grid = O.Grid(w.nx, w.ny, w.nz, w.h, w.h, w.h, w.open_)
        Bx, Bz = O.quantize_field(grid, 0.0, w.B)
        cen, dia = inputs.candidates_for(w)
        eps, _, _ = O.gen_inclusions(grid, cen, dia, w.fraction)
        st = O.new_state(grid, inputs.psi_init(w.nx, w.ny, w.nz, w.psi_seed).astype(np.complex128))
        O.step(grid, O.Params(Bx=Bx, Bz=Bz, J_ext=w.J, dt=w.dt, tol=1e-12, mode="exact", driven=True), eps, st)
        psi_g, mu_g, K_g = got[i]
        e = rel_maxerr(psi_g, st.psi)
        mu_e = float(np.max(np.abs(mu_g - st.mu))) / max(1.0, float(np.max(np.abs(st.mu))))
        print(f"[c3 inst {i} {w.nx}x{w.ny}x{w.nz} B {w.B:.3f} J {w.J:.4f}] one step: psi {e:.2e}, "
              f"mu {mu_e:.2e}, K {K_g:.10f} vs {st.K:.10f}")
        assert e <= 1e-5
        assert mu_e <= 1e-4
        assert abs(K_g - st.K) <= 1e-6


def test_c3_voltage_sampled_instances_vs_oracle():
    ref = json.load(open(GOLDEN))
    ws0 = inputs.batch_workloads()
    picks = _picks(ws0)
    assert picks == ref["picks"]
    tol = ws0[0].tol
    s, ws = _batch(tol, 100)
    steps = ws[0].steps
    early = {i: [] for i in picks}
    smax = 0
    for n in range(50):
        smax = max(smax, s.step(1, stats=True)["sweeps_max"])
        for i in picks:
            early[i].append(s.get_scalars(i)["E_last"])
    budget = min(100, smax + max(4, smax // 2))
    rest = s.step_graph(steps - 200 - 50, budget, stats=True)
    mid = {i: s.get_scalars(i) for i in picks}
    tail = s.step_graph(200, budget, stats=True)
    fin = {i: s.get_scalars(i) for i in picks}
    s.close()
    print(f"[c3] graph budget {budget}; capped steps {rest['capped_steps'] + tail['capped_steps']}")
    assert rest["capped_steps"] == 0 and tail["capped_steps"] == 0
    for i in picks:
        r = ref["instances"][str(i)]
        assert r["steps"] == steps
        E_ref = np.asarray(r["E"])
        d_early = float(np.max(np.abs(np.asarray(early[i]) - E_ref[:50])) / np.max(np.abs(E_ref[:50])))
        V_all = fin[i]["V_sum"] / fin[i]["n_avg"]
        V_200 = (fin[i]["V_sum"] - mid[i]["V_sum"]) / (fin[i]["n_avg"] - mid[i]["n_avg"])
        R_all = float(np.mean(E_ref))
        R_200 = float(np.mean(E_ref[-200:]))
        print(f"[c3 inst {i} {ws[i].nx}x{ws[i].ny}x{ws[i].nz} B {ws[i].B:.3f} J {ws[i].J:.4f}] "
              f"first 50 E max rel {d_early:.2e}; Vbar(1000) gpu {V_all:.6e} oracle {R_all:.6e} "
              f"rel {abs(V_all - R_all) / abs(R_all):.2e}; Vbar(last 200) gpu {V_200:.6e} oracle {R_200:.6e} "
              f"rel {abs(V_200 - R_200) / abs(R_200):.2e}")
        assert fin[i]["n_avg"] == steps
        assert d_early <= 1e-3
        assert abs(V_all - R_all) <= 0.01 * abs(R_all)
        assert abs(V_200 - R_200) <= 0.01 * abs(R_200)
