#!/usr/bin/env python3
"""Throughput of the implicit TDGL step on one MI355X.

Workload (default): 1024 x 1024 x 128 nodes, h = 0.5 xi, B = 0.2 Hc2 along z
(rounded to 8344 flux quanta), current J = 0.03 along x, 15 % random
spherical inclusions with lognormal diameters (median 3 xi, sigma 0.3,
eps = -1 inside, +1 outside), x periodic, y quasi-periodic, z open,
dt = 0.1, Jacobi stop max|r|^2 < 1e-8.  Synthetic seeded inputs.

A step is one full pass of the method: assemble, Jacobi sweeps to the stop
rule, J_av / K update, Poisson right side and Poisson solve (spectral for
this box).  The stencil tiling is chosen by tdgl_autotune during set-up.  W untimed
warm-up steps are followed by K timed steps bracketed by device
synchronisation.  value = nodes * K / seconds (cell-updates per second).

The roofline entry is for the dominant kernel, the Jacobi sweep: its launches
are bracketed by HIP events on the solver's stream inside the timed region,
and achieved = algorithmic bytes per pass (32 B per node: read psi, b/M and
(ht/2)/M, write psi, complex64 each; a two-sweep pass makes two iterates
from the same bytes) / mean time of a full pass (total sweep-class time over
the launches that did a full pass).

cpu_baseline times the FP64 oracle (test infrastructure, not the product)
on a bounded sample of the same physics.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SWEEP_BYTES_PER_NODE = 32      # psi in, b/M, (ht/2)/M, psi out (complex64)
ASSEMBLE_BYTES_PER_NODE = 40   # psi^-, eps, mu in; b/M, (ht/2)/M, psi^(1) out
# committed rocprofv3 counter summaries, one per sweep kernel
TRAFFIC_FILES = {"k_stencil_sweep": os.path.join(ROOT, "profiles", "sweep_c5_traffic.txt"),
                 "k_sweep2": os.path.join(ROOT, "profiles", "sweep2_c5_traffic.txt")}
SWEEP_SRCS = [os.path.join(ROOT, "paper_1409_8340_amd", "csrc", f)
              for f in ("k_gl.hip", "k_gl2.hip", "stencil.h", "tdgl_dev.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_sha():
    """Hash of the sources of the two sweep kernels (single and two-sweep)."""
    h = hashlib.sha256()
    for f in SWEEP_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def read_traffic(n_nodes, kernel):
    """HBM bytes per full sweep pass (one launch of the single-sweep kernel,
    or the two kernels of a two-sweep pass) from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the
    plain-copy calibration factor), or None when absent or taken on other
    sources."""
    path = TRAFFIC_FILES[kernel]
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if (kv.get("kernel_source_sha") != kernel_sha() or int(kv.get("nodes", -1)) != n_nodes
                or kv.get("kernel") != kernel):
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def setup(w, tdgl, inputs, torch, tol, mu_rtol, noise_T=0.0):
    p = tdgl.make_params(w.nx, w.ny, w.nz, h=w.h, driven=w.driven, tol=tol, max_iter=100,
                         mu_tol=1e-5, mu_rtol=mu_rtol, mu_max_cycles=20, noise_T=noise_T, noise_seed=0x5EED)
    s = tdgl.Solver(p)
    Bx, Bz = s.set_field(0.0, w.B, quantize=True)
    if w.driven:
        s.set_current(w.J)
    used = frac = None
    if w.fraction > 0:
        cen, dia = inputs.candidates_for(w)
        used, frac = s.gen_inclusions(cen, dia, w.fraction, w.eps_in, w.eps_out)
    psi0 = inputs.psi_init(w.nx, w.ny, w.nz, w.psi_seed)
    s.set_psi(torch.from_numpy(psi0).cuda())
    del psi0
    return s, Bz, used, frac


def variant_bench(w, tdgl, inputs, torch, kind, steps, warmup, mu_rtol):
    """The same workload with one of the paper's options switched on, timed
    like the main line: "noise" -- the Langevin term (Eq. b) at T = 0.02;
    "yz" -- the field turned into the yz plane, (By, Bz) = (0.1, B)."""
    s, Bz, used, frac = setup(w, tdgl, inputs, torch, w.tol, mu_rtol, noise_T=0.02 if kind == "noise" else 0.0)
    if kind == "yz":
        s.set_field_yz(0.1, w.B, quantize=True)
    tiling = s.autotune()
    s.step(warmup, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(steps, stats=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.close()
    N = w.nx * w.ny * w.nz
    return {"steps": steps, "ms_per_step": 1e3 * el / steps, "cell_updates_per_s": N * steps / el,
            "sweeps_per_step": st["sweeps_sum"] / max(st["steps"], 1),
            "tiling": {k: tiling[k] for k in ("rows", "chunk", "chunk2", "streaming", "fused", "persistent",
                                               "rhs_rows", "super_rows")}}


def host_cpu_model():
    """Model name of the host CPU (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds_target=20.0, seconds_1t=12.0):
    """FP64 oracle on a bounded sample: the workload's physics (h, B, J,
    inclusion law and fraction, psi init, Jacobi stop rule) on a
    256 x 256 x min(nz, 128) sub-box, as many steps as fit the time target
    (at least one), on all host threads the oracle is given; then the same
    sample continued on one thread.  Returns the entry for the JSON line."""
    import numpy as np
    from oracle import oracle as O
    from paper_1409_8340_amd import inputs
    nx, ny, nz = min(w.nx, 256), min(w.ny, 256), min(w.nz, 128)
    grid = O.Grid(nx, ny, nz, w.h, w.h, w.h, w.open_)
    Bx, Bz = O.quantize_field(grid, 0.0, w.B)
    sub = inputs.Workload(w.name + "_sample", nx, ny, nz, h=w.h, B=w.B, J=w.J, driven=w.driven,
                          fraction=w.fraction, law=w.law, d=w.d, psi_seed=w.psi_seed,
                          incl_seed=w.incl_seed, extra=w.extra)
    eps = np.ones(grid.shape)
    if w.fraction > 0:
        cen, dia = inputs.candidates_for(sub)
        eps, _, _ = O.gen_inclusions(grid, cen, dia, w.fraction)
    st = O.new_state(grid, inputs.psi_init(nx, ny, nz, w.psi_seed).astype(np.complex128))
    p = O.Params(Bx=Bx, Bz=Bz, J_ext=w.J, dt=w.dt, tol=w.tol, mode="mirror", driven=w.driven)

    def timed(target):
        t0 = time.perf_counter()
        steps = 0
        while True:
            O.step(grid, p, eps, st)
            steps += 1
            el = time.perf_counter() - t0
            if el >= target or steps >= 50:
                break
            if el / steps * (steps + 1) > 1.5 * target:
                break
        return steps, time.perf_counter() - t0

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    O.set_threads(threads)
    steps, el = timed(seconds_target)
    one = None
    if seconds_1t > 0:
        O.set_threads(1)
        s1, e1 = timed(seconds_1t)
        O.set_threads(threads)
        one = {"value": grid.N * s1 / e1, "steps": s1, "seconds": round(e1, 2)}
    return {"value": grid.N * steps / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle, {nx}x{ny}x{nz} sub-box of the workload's physics, {steps} steps from "
                      f"the seeded initial state, Jacobi stop rule max|r|^2<{w.tol:g} (same as GPU), exact "
                      f"Poisson; {el:.1f} s on {threads} OpenMP threads",
            "host_cpu": host_cpu_model(), "one_thread": one}


def adjoint_ratio(tdgl, inputs, torch, nsteps, ckpt, warmup):
    """(forward + adjoint time) / (plain forward time) on the c4 workload
    (128 x 128 x 32, B = 0.1, J = 0.03, 8 % d = 4 inclusions): nsteps
    steps with the voltage averaged over all of them, checkpoint every
    ckpt steps, both timed from the same state after warmup steps."""
    w = inputs.WORKLOADS["c4_adjoint_128x128x32"]
    s, _, _, _ = setup(w, tdgl, inputs, torch, w.tol, 0.0)
    s.autotune()
    s.step(warmup, stats=False)
    torch.cuda.synchronize()
    psi, mu, sc = s.get_psi(), s.get_mu(), s.get_scalars()
    t0 = time.perf_counter()
    s.step(nsteps, stats=True)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    s.set_psi(psi)
    s.set_mu(mu)
    s.set_scalars(sc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v, g = s.voltage_grad(nsteps, 0, ckpt)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    gn = float(torch.linalg.vector_norm(g.double()))
    s.close()
    return {"workload": w.name, "steps": nsteps, "ckpt_every": ckpt, "warmup": warmup,
            "plain_ms_per_step": 1e3 * t_fwd / nsteps, "fwd_adj_ms_per_step": 1e3 * t_adj / nsteps,
            "ratio": t_adj / t_fwd, "Vbar": v, "grad_l2": gn}


def small_bench(tdgl, inputs, torch, name, steps, warmup):
    """A small workload, where launches rather than HBM set the pace: steps
    per second with plain tdgl_step (the host follows convergence) and with
    graph-replayed steps (each step one captured launch sequence with a fixed
    sweep budget taken from the timed eager steps), continuing from the same
    run."""
    w = inputs.WORKLOADS[name]
    s, Bz, used, frac = setup(w, tdgl, inputs, torch, w.tol, 0.03)
    tiling = s.autotune()
    s.step(warmup, stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(steps, stats=True)
    torch.cuda.synchronize()
    t_e = time.perf_counter() - t0
    budget = min(100, st["sweeps_max"] + max(2, st["sweeps_max"] // 4))
    s.step_graph(1, budget, stats=False)  # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sg = s.step_graph(steps, budget, stats=True)
    torch.cuda.synchronize()
    t_g = time.perf_counter() - t0
    s.close()
    n = w.nx * w.ny * w.nz
    return {"workload": w.name, "nodes": n, "driven": w.driven, "steps": steps, "warmup": warmup,
            "tiling": {k: tiling[k] for k in ("rows", "chunk", "chunk2", "streaming", "fused", "persistent",
                                               "rhs_rows", "super_rows")},
            "eager_us_per_step": 1e6 * t_e / steps, "eager_rate": n * steps / t_e,
            "eager_sweeps_per_step": st["sweeps_sum"] / steps,
            "graph_us_per_step": 1e6 * t_g / steps, "graph_rate": n * steps / t_g,
            "graph_sweeps_per_step": sg["sweeps_sum"] / steps, "graph_sweep_budget": budget,
            "graph_capped_steps": sg["capped_steps"]}


def batch_bench(tdgl, inputs, torch, steps, warmup, n=64):
    """Batched form against single-instance steps on the same GPU: n
    instances with shapes drawn from {64^3, 96x96x48, 128x128x32}, per
    instance B, J, inclusion diameter and fraction, in one context advanced
    by graph-replayed steps (one captured launch sequence per step for all
    instances); then the same instances, each in its own context, advanced by
    plain tdgl_step from the same state.  Rates are nodes x steps / s."""
    ws = inputs.batch_workloads(n)
    params = [tdgl.make_params(w.nx, w.ny, w.nz, h=w.h, driven=True, tol=w.tol, max_iter=100,
                               mu_tol=1e-5, mu_rtol=0.03) for w in ws]

    def load(s, i, w, inst):
        s.set_field(0.0, w.B, inst=inst, quantize=True)
        s.set_current(w.J, inst=inst)
        cen, dia = inputs.candidates_for(w)
        s.gen_inclusions(cen, dia, w.fraction, w.eps_in, w.eps_out, inst=inst)
        s.set_psi(torch.from_numpy(inputs.psi_init(w.nx, w.ny, w.nz, w.psi_seed)).cuda(), inst=inst)

    nodes = sum(w.nx * w.ny * w.nz for w in ws)
    b = tdgl.Solver(params)
    for i, w in enumerate(ws):
        load(b, i, w, i)
    tiling = b.autotune()
    wst = b.step(warmup, stats=True)
    budget = min(100, wst["sweeps_max"] + max(4, wst["sweeps_max"] // 2))
    states = [(b.get_psi(i), b.get_mu(i), b.get_scalars(i)) for i in range(n)]
    b.step_graph(1, budget, stats=False)  # capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.step_graph(steps, budget, stats=True)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    b.close()
    t_s = 0.0
    sweeps_s = 0
    for i, w in enumerate(ws):
        s = tdgl.Solver([params[i]])
        load(s, i, w, 0)
        s.autotune()
        s.set_psi(states[i][0])
        s.set_mu(states[i][1])
        s.set_scalars(states[i][2])
        s.step(1, stats=False)
        # the comparison starts one step later than the batch: the same work
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ss = s.step(steps, stats=True)
        torch.cuda.synchronize()
        t_s += time.perf_counter() - t0
        sweeps_s += ss["sweeps_sum"]
        s.close()
    return {"instances": n, "nodes": nodes, "steps": steps, "warmup": warmup, "sweep_budget": budget,
            "tiling": {"rows": tiling["rows"], "chunk": tiling["chunk"], "streaming": tiling["streaming"],
                       "fused": tiling["fused"], "persistent": tiling["persistent"]},
            "batched_rate": nodes * steps / t_b, "batched_ms_per_step": 1e3 * t_b / steps,
            "sequential_rate": nodes * steps / t_s, "sequential_ms_per_step": 1e3 * t_s / steps,
            "speedup": t_s / t_b, "batched_sweeps_sum": st["sweeps_sum"], "capped_steps": st["capped_steps"],
            "sequential_sweeps_sum": sweeps_s}


def iv_study(tdgl, inputs, torch, w, points, steps, window, mu_rtol):
    """The workload's current sweep (Sec. 3.1.1, current-voltage
    characteristics): J = 0 .. 0.06 in `points` equal steps, ascending, the
    state carried from one point to the next; at each point `steps` steps,
    the time-averaged field <E_x> over the last `window`.  One JSON line per
    point (V = Lx <E_x> as well)."""
    s, Bz, used, frac = setup(w, tdgl, inputs, torch, w.tol, mu_rtol)
    tiling = s.autotune()
    Lx = w.nx * w.h
    for q in range(points):
        J = 0.06 * q / max(points - 1, 1)
        s.set_current(J)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        a = s.step(steps - window, stats=True)
        s.window_reset()
        b = s.step(window, stats=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        obs = s.observables()
        print(json.dumps({"study": "iv", "workload": w.name, "J": J, "steps": steps, "window": window,
                          "E_mean": obs["E_mean"], "V_mean": obs["E_mean"] * Lx, "psi2_mean": obs["psi2_mean"],
                          "sweeps_per_step": (a["sweeps_sum"] + b["sweeps_sum"]) / steps,
                          "capped_steps": a["capped_steps"] + b["capped_steps"],
                          "ms_per_step": 1e3 * el / steps, "B_eff": Bz, "inclusions": used,
                          "tiling": {k: tiling[k] for k in ("rows", "chunk", "chunk2", "streaming", "fused")}}),
              flush=True)
    s.close()


def jacobi_study(tdgl, inputs, torch, steps, warmup):
    """The paper's Fig. 5 study on this solver: Jacobi iterations per step
    and time per step of a 2D free-flowing vortex film (one z plane, no
    pinning, B = 0.1 along z, J = 0.02 along x) against the grid size
    (h = 0.5, tol 1e-6), the spacing h (1024 x 1024, tol 1e-6) and the
    stop tolerance (1024 x 1024, h = 0.5).  tol bounds max|r|^2, the
    reading used everywhere in this library.  One JSON line per point."""
    pts = [("N", n, 0.5, 1e-6) for n in (128, 256, 512, 1024, 2048, 4096)]
    pts += [("h", 1024, h, 1e-6) for h in (0.2, 0.3, 0.4, 0.5, 0.7, 1.0)]
    pts += [("tol", 1024, 0.5, t) for t in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10, 1e-12)]
    for axis, n, h, tol in pts:
        p = tdgl.make_params(n, n, 1, h=h, driven=True, tol=tol, max_iter=256, mu_tol=1e-5, mu_rtol=0.03,
                             mu_max_cycles=20)
        s = tdgl.Solver(p)
        Bx, Bz = s.set_field(0.0, 0.1, quantize=True)
        s.set_current(0.02)
        s.set_psi(torch.from_numpy(inputs.psi_init(n, n, 1, 1005)).cuda())
        tiling = s.autotune()
        s.step(warmup, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.step(steps, stats=True)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        s.close()
        rec = {"study": "jacobi_fig5", "vary": axis, "nx": n, "ny": n, "nz": 1, "h": h, "tol": tol,
               "B_eff": Bz, "J": 0.02, "warmup": warmup, "steps": steps,
               "sweeps_per_step": st["sweeps_sum"] / steps, "sweeps_min": st["sweeps_min"],
               "sweeps_max": st["sweeps_max"], "capped_steps": st["capped_steps"],
               "ms_per_step": 1e3 * el / steps, "cell_updates_per_s": n * n * steps / el,
               "tiling": {k: tiling[k] for k in ("rows", "chunk", "chunk2", "streaming", "fused")}}
        log(f"[study] {axis}: n={n} h={h} tol={tol:g}: {rec['sweeps_per_step']:.2f} sweeps/step, "
            f"{rec['ms_per_step']:.4f} ms/step")
        print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c5_1024x1024x128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--breakdown-steps", type=int, default=5,
                    help="extra untimed steps profiled per kernel class")
    ap.add_argument("--mu-rtol", type=float, default=0.03,
                    help="Poisson stop: residual below max(1e-5, mu_rtol * initial residual)")
    ap.add_argument("--adjoint-steps", type=int, default=500,
                    help="steps of the c4 forward+adjoint comparison (0 skips it)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="steps of the 64-instance batched comparison (0 skips it)")
    ap.add_argument("--small-steps", type=int, default=200,
                    help="steps of the small-workload lines (32x32x16 undriven, 256x256x64 driven), eager "
                         "and graph-replayed (0 skips them)")
    ap.add_argument("--variant-steps", type=int, default=10,
                    help="steps of the same workload with Langevin noise and with a yz-plane field (0 skips)")
    ap.add_argument("--tiling", default=None,
                    help="rows,chunk,streaming,fused[,persistent[,chunk2[,rhs_rows[,super_rows]]]]: set the stencil tiling instead of "
                         "tdgl_autotune")
    ap.add_argument("--study", choices=["jacobi", "iv"], default=None,
                    help="instead of the benchmark line: 'jacobi', the Jacobi iteration study (2D film: "
                         "iterations and time per step against grid size, spacing and tolerance); 'iv', the "
                         "workload's current sweep J = 0..0.06 in 13 points (--steps per point, <E> over the "
                         "last half); one JSON line per point")
    ap.add_argument("--flow-warmup", type=int, default=200,
                    help="untimed steps after the timed region before the flowing-state figure (0 skips it)")
    ap.add_argument("--flow-steps", type=int, default=20, help="timed steps of the flowing-state figure")
    ap.add_argument("--copy-calib-gib", type=float, default=0.0,
                    help="run a plain device copy of this size (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this solver runs on one GPU; multi-GPU runs are not part of this build "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1409_8340_amd import inputs, tdgl
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.study == "jacobi":
        jacobi_study(tdgl, inputs, torch, args.steps, args.warmup)
        return
    w = inputs.WORKLOADS[args.workload]
    if args.study == "iv":
        iv_study(tdgl, inputs, torch, w, 13, args.steps, args.steps // 2, args.mu_rtol)
        return
    N = w.nx * w.ny * w.nz

    log(f"[bench] setting up {w.name} ({N} nodes)")
    s, Bz, used, frac = setup(w, tdgl, inputs, torch, w.tol, args.mu_rtol)
    log(f"[bench] B_eff={Bz:.6f} inclusions={used} fraction={frac}")
    if args.tiling:
        v_ = [int(v) for v in args.tiling.split(",")] + [0, 0, 0, 0]
        s.set_tiling(rows=v_[0], chunk=v_[1], streaming=v_[2], fused=v_[3], persistent=v_[4], chunk2=v_[5],
                     rhs_rows=v_[6], super_rows=v_[7])
        tiling = s.tiling()
    else:
        tiling = s.autotune()
    log(f"[bench] stencil tiling {tiling}")
    if args.copy_calib_gib > 0:
        # one elementwise kernel that reads nb bytes and writes nb bytes
        nb = int(args.copy_calib_gib * (1 << 30)) // 4 * 4
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: {nb} bytes read and {nb} bytes written by one mul kernel")
    for i in range(args.warmup):
        s.step(1, stats=False)
        if (i + 1) % 10 == 0:
            torch.cuda.synchronize()
            log(f"[bench] warmup {i + 1}/{args.warmup}")
    torch.cuda.synchronize()

    s.profile_start(["assemble", "sweep"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.step(args.steps, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_stop()
    el = t1 - t0
    log(f"[bench] timed {args.steps} steps in {el:.3f} s; sweeps {st['sweeps_sum']} "
        f"(min {st['sweeps_min']} max {st['sweeps_max']}), mu cycles {st['mu_cycles_sum']}")

    breakdown = None
    if args.breakdown_steps > 0:
        s.profile_start()
        s.step(args.breakdown_steps, stats=True)
        bd = s.profile_stop()
        tot = sum(v["ms"] for v in bd.values())
        breakdown = {k: {"launches": v["launches"], "ms": round(v["ms"], 4),
                         "share": round(v["ms"] / tot, 4) if tot else 0.0} for k, v in bd.items()}
    obs = s.observables()

    flowing = None
    if args.flow_warmup > 0 and args.flow_steps > 0:
        # the same run further on: vortices flowing rather than the start's transient
        s.step(args.flow_warmup, stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fs = s.step(args.flow_steps, stats=True)
        torch.cuda.synchronize()
        fe = time.perf_counter() - t0
        fo = s.observables()
        done = args.warmup + args.steps + args.breakdown_steps + args.flow_warmup
        flowing = {"after_steps": done, "steps": args.flow_steps, "ms_per_step": 1e3 * fe / args.flow_steps,
                   "cell_updates_per_s": N * args.flow_steps / fe,
                   "sweeps_per_step": fs["sweeps_sum"] / max(fs["steps"], 1),
                   "E_last": fo["E_last"], "psi2_mean": fo["psi2_mean"]}
        log(f"[bench] flowing state after {done} steps: {flowing['ms_per_step']:.3f} ms/step, "
            f"{flowing['sweeps_per_step']:.2f} sweeps/step")

    sw = prof["sweep"]
    # Sweep-class launches that did a full pass over the grid (the library
    # counts them: the first iterate of a step comes from the assemble kernel,
    # a two-sweep pass makes two iterates, and the launch that starts before
    # the host has seen convergence exits at once; its few microseconds stay
    # in the total, so the mean below errs on the slow side).  A pass of
    # either kind reads psi, b/M and (ht/2)/M and writes psi once: 32 B/node.
    full = max(st["sweep_passes"], 1)
    sweep_ms = sw["ms"] / full
    achieved = SWEEP_BYTES_PER_NODE * N / (sweep_ms * 1e-3) / 1e9
    asm = prof["assemble"]
    asm_ms = asm["ms"] / max(asm["launches"], 1)
    traffic = read_traffic(N, "k_sweep2" if tiling["fused"] else "k_stencil_sweep")

    adj = None
    if args.adjoint_steps > 0:
        log(f"[bench] c4 forward+adjoint over {args.adjoint_steps} steps")
        adj = adjoint_ratio(tdgl, inputs, torch, args.adjoint_steps, 50, 1000)
        # the same with every state of the window kept in HBM (no recompute)
        whole = adjoint_ratio(tdgl, inputs, torch, args.adjoint_steps, args.adjoint_steps, 1000)
        adj["whole_trajectory"] = {k: whole[k] for k in ("ckpt_every", "fwd_adj_ms_per_step", "plain_ms_per_step",
                                                          "ratio")}
        log(f"[bench] adjoint ratio {adj['ratio']:.3f} (checkpoint every 50), {whole['ratio']:.3f} (whole trajectory)")

    batch = None
    if args.batch_steps > 0:
        log(f"[bench] 64-instance batch over {args.batch_steps} steps")
        batch = batch_bench(tdgl, inputs, torch, args.batch_steps, 10)
        log(f"[bench] batch {batch['batched_rate']:.3e} vs sequential {batch['sequential_rate']:.3e} "
            f"cell-updates/s (x{batch['speedup']:.2f})")

    variants = None
    if args.variant_steps > 0:
        variants = {}
        for kind in ("noise", "yz"):
            variants[kind] = variant_bench(w, tdgl, inputs, torch, kind, args.variant_steps, 3, args.mu_rtol)
            log(f"[bench] variant {kind}: {variants[kind]['ms_per_step']:.3f} ms/step, "
                f"{variants[kind]['sweeps_per_step']:.2f} sweeps/step, tiling {variants[kind]['tiling']}")

    small = None
    if args.small_steps > 0:
        small = {}
        for name in ("c1_small_undriven", "c2_256x256x64_J0.02"):
            small[name] = small_bench(tdgl, inputs, torch, name, args.small_steps, 20)
            r = small[name]
            log(f"[bench] {name}: {r['eager_us_per_step']:.1f} us/step eager, {r['graph_us_per_step']:.1f} "
                f"us/step graph-replayed ({r['eager_sweeps_per_step']:.2f} / {r['graph_sweeps_per_step']:.2f} "
                f"sweeps/step)")

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a bounded sample")
        cpu = cpu_baseline(w, args.cpu_seconds)
        log(f"[bench] oracle {cpu['value']:.3e} cell-updates/s")

    out = {
        "metric": "TDGL cell-updates/s + %HBM roofline; fwd+adjoint step time vs plain step",
        "value": N * args.steps / el,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": [w.nx, w.ny, w.nz], "h": w.h, "B_eff": Bz, "J": w.J,
                   "inclusions": used, "inclusion_fraction": frac, "tol": w.tol, "dt": w.dt,
                   "mu_tol": 1e-5, "mu_rtol": args.mu_rtol,
                   "tiling": {"rows": tiling["rows"], "chunk": tiling["chunk"], "chunk2": tiling["chunk2"],
                              "streaming": tiling["streaming"], "fused": tiling["fused"],
                              "persistent": tiling["persistent"], "rhs_rows": tiling["rhs_rows"], "super_rows": tiling["super_rows"]},
                   "precision": "psi, links and sweeps in FP32 (complex64 storage); residual, J_av, K, "
                                "means and the Poisson z solve in FP64",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": ("tdgl::k_sweep2i + tdgl::k_sweep2 (one two-sweep Jacobi pass: super-tiles, "
                                "and boundary tiles where there are any)" if tiling["fused"]
                                else "tdgl::k_stencil<1> (Jacobi sweep)"),
                     "sweeps_per_pass": 2 if tiling["fused"] else 1,
                     "bytes_per_launch": SWEEP_BYTES_PER_NODE * N, "mean_launch_ms": sweep_ms,
                     "full_launches": full, "launches": sw["launches"]},
        "cpu_baseline": cpu,
        "extra": {
            "sweeps_per_step": st["sweeps_sum"] / max(st["steps"], 1),
            "cell_sweeps_per_s": N * st["sweeps_sum"] / el,
            "mu_cycles_per_step": st["mu_cycles_sum"] / max(st["steps"], 1),
            "assemble_ms": asm_ms,
            "assemble_GBps": ASSEMBLE_BYTES_PER_NODE * N / (asm_ms * 1e-3) / 1e9,
            "kernel_breakdown": breakdown,
            "flowing": flowing,
            "adjoint": adj,
            "batch": batch,
            "variants": variants,
            "small": small,
            "E_mean": obs["E_mean"], "F": obs["F"], "psi2_mean": obs["psi2_mean"],
            "kernel_source_sha": kernel_sha(),
        },
    }
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
