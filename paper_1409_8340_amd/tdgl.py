"""ctypes binding of libtdgl (include/tdgl.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  torch provides the device memory (the workspace and the user
arrays) and the stream.  Loading fails loudly when the library has not been
built; there is no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import re
import weakref
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdgl.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "tdgl.h")

TDGL_PERIODIC = 0
TDGL_OPEN = 1
STATUS = {0: "OK", 1: "EINVAL", 2: "EWS", 3: "ENOCONV", 4: "EDEVICE", 5: "ESTATE"}


class TdglError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("bc", ctypes.c_int * 3), ("g", ctypes.c_double), ("u", ctypes.c_double),
                ("dt", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("driven", ctypes.c_int), ("mu_tol", ctypes.c_double), ("mu_rtol", ctypes.c_double),
                ("mu_max_cycles", ctypes.c_int), ("strict", ctypes.c_int),
                ("tile_cz", ctypes.c_int), ("tile_rows", ctypes.c_int), ("poisson", ctypes.c_int),
                ("reserved0", ctypes.c_int), ("noise_T", ctypes.c_double), ("noise_seed", ctypes.c_ulonglong),
                ("reserved", ctypes.c_int * 2)]


class StepStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("sweeps_min", ctypes.c_int),
                ("sweeps_max", ctypes.c_int), ("sweeps_sum", ctypes.c_longlong),
                ("capped_steps", ctypes.c_int), ("last_res2", ctypes.c_float),
                ("mu_cycles_sum", ctypes.c_int), ("mu_capped_steps", ctypes.c_int),
                ("mu_last_res", ctypes.c_float), ("sweep_passes", ctypes.c_longlong),
                ("single_first_steps", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Scalars(ctypes.Structure):
    _fields_ = [("K", ctypes.c_double), ("t", ctypes.c_double), ("V_sum", ctypes.c_double),
                ("n", ctypes.c_longlong), ("n_avg", ctypes.c_longlong),
                ("E_last", ctypes.c_double), ("J_av_last", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Obs(ctypes.Structure):
    _fields_ = [("F", ctypes.c_double), ("E_last", ctypes.c_double), ("E_mean", ctypes.c_double),
                ("V_mean", ctypes.c_double), ("J_av", ctypes.c_double), ("K", ctypes.c_double),
                ("res2_last", ctypes.c_double), ("mu_mean_w", ctypes.c_double),
                ("psi2_mean", ctypes.c_double), ("n", ctypes.c_longlong),
                ("n_avg", ctypes.c_longlong)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# profile classes, in the order of the TDGL_K_* codes: "poisson" is the solve on the
# full grid (FFT passes and z systems, or the finest multigrid level),
# "poisson_coarse" the coarser multigrid levels
KERNEL_CLASSES = ["assemble", "sweep", "current", "rhs", "poisson", "poisson_coarse", "other"]


class Tiling(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int), ("chunk", ctypes.c_int), ("streaming", ctypes.c_int),
                ("fused", ctypes.c_int), ("persistent", ctypes.c_int), ("sweep_us", ctypes.c_double),
                ("chunk2", ctypes.c_int), ("rhs_rows", ctypes.c_int), ("super_rows", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Prof(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong * 7), ("ms", ctypes.c_double * 7)]

    def as_dict(self):
        return {k: {"launches": self.launches[i], "ms": self.ms[i]}
                for i, k in enumerate(KERNEL_CLASSES)}


_lib = None

_SIGS = {
    "tdgl_last_error": ([], ctypes.c_char_p),
    "tdgl_plan": ([ctypes.c_int, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tdgl_create": ([ctypes.c_int, ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_size_t,
                     ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "tdgl_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "tdgl_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "tdgl_quantize_field": ([ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                            ctypes.c_int),
    "tdgl_quantize_field_yz": ([ctypes.POINTER(Params), ctypes.c_double, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tdgl_set_field_yz": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tdgl_set_field": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tdgl_set_current": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_double], ctypes.c_int),
    "tdgl_set_eps": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_get_eps": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_gen_inclusions": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                             ctypes.c_double, ctypes.c_float, ctypes.c_float, ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tdgl_gen_shapes": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                         ctypes.c_float, ctypes.c_float, ctypes.POINTER(ctypes.c_int),
                         ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tdgl_gen_voronoi": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                          ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "tdgl_set_insulators": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_set_psi": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_get_psi": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_set_mu": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_get_mu": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "tdgl_get_scalars": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Scalars)], ctypes.c_int),
    "tdgl_set_scalars": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Scalars)], ctypes.c_int),
    "tdgl_voltage_window_reset": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "tdgl_step": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(StepStats)], ctypes.c_int),
    "tdgl_observables": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Obs)], ctypes.c_int),
    "tdgl_poisson_solve": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tdgl_step_graph": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(StepStats)], ctypes.c_int),
    "tdgl_adjoint_plan": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                          ctypes.c_int),
    "tdgl_voltage_grad": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_size_t, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p], ctypes.c_int),
    "tdgl_voltage_grad_noalloc": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p], ctypes.c_int),
    "tdgl_autotune": ([ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(Tiling)], ctypes.c_int),
    "tdgl_get_tiling": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Tiling)], ctypes.c_int),
    "tdgl_set_tiling": ([ctypes.c_void_p, ctypes.POINTER(Tiling)], ctypes.c_int),
    "tdgl_profile_start": ([ctypes.c_void_p, ctypes.c_uint], ctypes.c_int),
    "tdgl_profile_stop": ([ctypes.c_void_p, ctypes.POINTER(Prof)], ctypes.c_int),
}


def header_symbols():
    """Entry points declared in include/tdgl.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tdgl_[a-z_]+)\s*\(", txt)))


def load():
    """Load libtdgl.so (must have been built; raises otherwise)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


_live = weakref.WeakSet()


def _close_all():
    """Destroys every context still open and waits for the device at
    interpreter exit.  Python runs this before it tears its modules down and
    before the C runtime's exit handlers, so no context is destroyed by a
    finaliser while the HIP runtime, or a tool attached to it, is already
    shutting down."""
    for s in list(_live):
        try:
            s.close()
        except Exception:
            pass
    try:
        import torch
        if torch.cuda.is_initialized():
            torch.cuda.synchronize()
    except Exception:
        pass


atexit.register(_close_all)


def _check(status):
    if status != 0:
        msg = load().tdgl_last_error()
        raise TdglError(status, msg.decode() if msg else "")


def make_params(nx, ny, nz, h=0.5, hx=None, hy=None, hz=None, bc=(TDGL_PERIODIC, TDGL_PERIODIC, TDGL_OPEN),
                g=1.0, u=1.0, dt=0.1, tol=1e-8, max_iter=100, driven=False, mu_tol=1e-5,
                mu_rtol=0.0, mu_max_cycles=20, strict=False, tile_cz=0, tile_rows=0,
                poisson=0, noise_T=0.0, noise_seed=0) -> Params:
    p = Params()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.hx = h if hx is None else hx
    p.hy = h if hy is None else hy
    p.hz = h if hz is None else hz
    for a in range(3):
        p.bc[a] = int(bc[a])
    p.g, p.u, p.dt, p.tol = g, u, dt, tol
    p.max_iter = max_iter
    p.driven = int(bool(driven))
    p.mu_tol = mu_tol
    p.mu_rtol = mu_rtol
    p.mu_max_cycles = mu_max_cycles
    p.strict = int(bool(strict))
    p.tile_cz = tile_cz
    p.tile_rows = tile_rows
    p.poisson = poisson
    p.noise_T = noise_T
    p.noise_seed = noise_seed
    return p


def plan(params) -> int:
    arr = (Params * len(params))(*params)
    sz = ctypes.c_size_t()
    _check(load().tdgl_plan(len(params), arr, ctypes.byref(sz)))
    return sz.value


def quantize_field(p: Params, Bx: float, Bz: float):
    bx, bz = ctypes.c_double(), ctypes.c_double()
    _check(load().tdgl_quantize_field(ctypes.byref(p), Bx, Bz, ctypes.byref(bx), ctypes.byref(bz)))
    return bx.value, bz.value


def quantize_field_yz(p: Params, By: float, Bz: float):
    by, bz = ctypes.c_double(), ctypes.c_double()
    _check(load().tdgl_quantize_field_yz(ctypes.byref(p), By, Bz, ctypes.byref(by), ctypes.byref(bz)))
    return by.value, bz.value


class Solver:
    """A context of one or more instances on the current torch device."""

    def __init__(self, params, stream=None):
        import torch
        if isinstance(params, Params):
            params = [params]
        self.params = list(params)
        self.n = len(self.params)
        lib = load()
        ws_bytes = plan(self.params)
        self._ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        arr = (Params * self.n)(*self.params)
        ctx = ctypes.c_void_p()
        _check(lib.tdgl_create(self.n, arr, ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(ws_bytes),
                               ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(ctx)))
        self._ctx = ctx
        self.ws_bytes = ws_bytes
        _live.add(self)

    def close(self):
        """Destroys the context (synchronising) and releases its workspace."""
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            load().tdgl_destroy(self._ctx)
            self._ctx = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def shape(self, inst=0):
        p = self.params[inst]
        return (p.nz, p.ny, p.nx)

    def _dev(self, t, dtype):
        import torch
        assert t.device.type == "cuda" and t.dtype == dtype and t.is_contiguous(), (t.device, t.dtype)
        return ctypes.c_void_p(t.data_ptr())

    # -- setters / getters
    def set_field(self, Bx, Bz, inst=0, quantize=True):
        bx, bz = ctypes.c_double(), ctypes.c_double()
        _check(load().tdgl_set_field(self._ctx, inst, Bx, Bz, int(quantize), ctypes.byref(bx),
                                     ctypes.byref(bz)))
        return bx.value, bz.value

    def set_field_yz(self, By, Bz, inst=0, quantize=True):
        """Field in the yz plane (tdgl_set_field_yz); returns (By, Bz) as set."""
        by, bz = ctypes.c_double(), ctypes.c_double()
        _check(load().tdgl_set_field_yz(self._ctx, inst, By, Bz, int(quantize), ctypes.byref(by),
                                        ctypes.byref(bz)))
        return by.value, bz.value

    def set_current(self, J, inst=0):
        _check(load().tdgl_set_current(self._ctx, inst, J))

    def set_eps(self, eps, inst=0):
        import torch
        eps = eps.to(device="cuda", dtype=torch.float32).contiguous()
        torch.cuda.current_stream().synchronize()   # the library reads it on its own stream
        _check(load().tdgl_set_eps(self._ctx, inst, self._dev(eps, torch.float32)))
        self._keep = eps

    def get_eps(self, inst=0):
        import torch
        out = torch.empty(self.shape(inst), dtype=torch.float32, device="cuda")
        _check(load().tdgl_get_eps(self._ctx, inst, self._dev(out, torch.float32)))
        self._stream.synchronize()
        return out

    def gen_inclusions(self, centres, diameters, target, eps_in=-1.0, eps_out=1.0, inst=0):
        import torch
        c = torch.as_tensor(centres, dtype=torch.float64).reshape(-1, 3).contiguous().cuda()
        d = torch.as_tensor(diameters, dtype=torch.float64).reshape(-1).contiguous().cuda()
        torch.cuda.current_stream().synchronize()
        used, frac = ctypes.c_int(), ctypes.c_double()
        _check(load().tdgl_gen_inclusions(self._ctx, inst, self._dev(c, torch.float64),
                                          self._dev(d, torch.float64), int(d.numel()), float(target),
                                          float(eps_in), float(eps_out), ctypes.byref(used),
                                          ctypes.byref(frac)))
        return used.value, frac.value

    def gen_shapes(self, shapes, target, eps_in=-1.0, eps_out=1.0, inst=0):
        """shapes: (nc, 16) doubles per tdgl_gen_shapes (centre, Q, axis, hlen, ext)."""
        import torch
        sh = torch.as_tensor(shapes, dtype=torch.float64).reshape(-1, 16).contiguous().cuda()
        torch.cuda.current_stream().synchronize()
        used, frac = ctypes.c_int(), ctypes.c_double()
        _check(load().tdgl_gen_shapes(self._ctx, inst, self._dev(sh, torch.float64), int(sh.shape[0]),
                                      float(target), float(eps_in), float(eps_out), ctypes.byref(used),
                                      ctypes.byref(frac)))
        return used.value, frac.value

    def gen_voronoi(self, seeds, values, metric=0, axes=7, inst=0):
        """seeds: (ns, 3) positions; values: (ns,) eps per crystallite;
        metric 0 Euclidean, 1 absolute, 2 maximum; axes: bit mask of the
        axes in the distance (per tdgl_gen_voronoi)."""
        import torch
        sd = torch.as_tensor(seeds, dtype=torch.float64).reshape(-1, 3).contiguous().cuda()
        vals = torch.as_tensor(values, dtype=torch.float32).reshape(-1).contiguous().cuda()
        if vals.numel() != sd.shape[0]:
            raise ValueError("one value per seed")
        torch.cuda.current_stream().synchronize()
        _check(load().tdgl_gen_voronoi(self._ctx, inst, self._dev(sd, torch.float64), self._dev(vals, torch.float32),
                                       int(sd.shape[0]), int(metric), int(axes)))

    def set_insulators(self, mask, inst=0):
        """mask: array-like of the instance's shape (nz, ny, nx), nonzero =
        insulating node (tdgl_set_insulators: rewrites eps, zeroes psi there)."""
        import torch
        m = torch.as_tensor(mask).to(dtype=torch.uint8).reshape(-1).contiguous().cuda()
        if m.numel() != self.params[inst].nx * self.params[inst].ny * self.params[inst].nz:
            raise ValueError("mask must have one entry per node")
        torch.cuda.current_stream().synchronize()
        _check(load().tdgl_set_insulators(self._ctx, inst, self._dev(m, torch.uint8)))

    def set_psi(self, psi, inst=0):
        import torch
        psi = psi.to(device="cuda", dtype=torch.complex64).contiguous()
        torch.cuda.current_stream().synchronize()   # the library reads it on its own stream
        _check(load().tdgl_set_psi(self._ctx, inst, self._dev(psi, torch.complex64)))
        self._stream.synchronize()

    def get_psi(self, inst=0):
        import torch
        out = torch.empty(self.shape(inst), dtype=torch.complex64, device="cuda")
        _check(load().tdgl_get_psi(self._ctx, inst, self._dev(out, torch.complex64)))
        self._stream.synchronize()
        return out

    def set_mu(self, mu, inst=0):
        import torch
        mu = mu.to(device="cuda", dtype=torch.float32).contiguous()
        torch.cuda.current_stream().synchronize()   # the library reads it on its own stream
        _check(load().tdgl_set_mu(self._ctx, inst, self._dev(mu, torch.float32)))
        self._stream.synchronize()

    def get_mu(self, inst=0):
        import torch
        out = torch.empty(self.shape(inst), dtype=torch.float32, device="cuda")
        _check(load().tdgl_get_mu(self._ctx, inst, self._dev(out, torch.float32)))
        self._stream.synchronize()
        return out

    def get_scalars(self, inst=0):
        s = Scalars()
        _check(load().tdgl_get_scalars(self._ctx, inst, ctypes.byref(s)))
        return s.as_dict()

    def set_scalars(self, d, inst=0):
        s = Scalars()
        for k, v in d.items():
            setattr(s, k, v)
        _check(load().tdgl_set_scalars(self._ctx, inst, ctypes.byref(s)))

    def window_reset(self, inst=0):
        _check(load().tdgl_voltage_window_reset(self._ctx, inst))

    def step(self, nsteps=1, stats=True):
        st = StepStats()
        _check(load().tdgl_step(self._ctx, int(nsteps), ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def step_graph(self, nsteps=1, budget=None, stats=True):
        """nsteps steps as replays of one captured graph (tdgl_step_graph);
        budget defaults to the largest max_iter of the context."""
        if budget is None:
            budget = max(p.max_iter for p in self.params)
        st = StepStats()
        _check(load().tdgl_step_graph(self._ctx, int(nsteps), int(budget), ctypes.byref(st) if stats else None))
        return st.as_dict() if stats else None

    def poisson_solve(self, f):
        import torch
        f = f.to(device="cuda", dtype=torch.float32).contiguous()
        out = torch.empty(self.shape(0), dtype=torch.float32, device="cuda")
        _check(load().tdgl_poisson_solve(self._ctx, self._dev(f, torch.float32),
                                         self._dev(out, torch.float32)))
        self._stream.synchronize()
        return out

    def autotune(self, cache_path=None):
        """Pick the stencil tiling by timing (tdgl_autotune); returns it."""
        t = Tiling()
        path = None if cache_path is None else str(cache_path).encode()
        _check(load().tdgl_autotune(self._ctx, path, ctypes.byref(t)))
        return t.as_dict()

    def set_tiling(self, rows=2, chunk=0, streaming=0, fused=0, persistent=0, chunk2=0, rhs_rows=0, super_rows=0):
        t = Tiling(rows=rows, chunk=chunk, streaming=streaming, fused=fused, persistent=persistent,
                   sweep_us=0.0, chunk2=chunk2, rhs_rows=rhs_rows, super_rows=super_rows)
        _check(load().tdgl_set_tiling(self._ctx, ctypes.byref(t)))

    def tiling(self, inst=0):
        t = Tiling()
        _check(load().tdgl_get_tiling(self._ctx, inst, ctypes.byref(t)))
        return t.as_dict()

    def voltage_grad(self, nsteps, window_begin=0, ckpt_every=50):
        """(Vbar, dVbar/deps) over nsteps steps; see tdgl_voltage_grad."""
        import torch
        nb = ctypes.c_size_t()
        _check(load().tdgl_adjoint_plan(self._ctx, nsteps, ckpt_every, ctypes.byref(nb)))
        torch.cuda.current_stream().synchronize()
        ws = torch.empty(nb.value + 256, dtype=torch.uint8, device="cuda")
        ptr = (ws.data_ptr() + 255) // 256 * 256
        grad = torch.empty(self.shape(0), dtype=torch.float32, device="cuda")
        v = ctypes.c_double()
        _check(load().tdgl_voltage_grad(self._ctx, nsteps, window_begin, ckpt_every, ctypes.c_void_p(ptr),
                                        nb.value, ctypes.byref(v), self._dev(grad, torch.float32)))
        del ws
        return v.value, grad

    def voltage_grad_noalloc(self, nsteps, window_begin=0, ckpt_every=50, grad=None):
        """tdgl_voltage_grad_noalloc: the adjoint buffers sit in the library's
        fixed device array; grad (float32, the grid's shape) may be given."""
        import torch
        if grad is None:
            grad = torch.empty(self.shape(0), dtype=torch.float32, device="cuda")
        torch.cuda.current_stream().synchronize()
        v = ctypes.c_double()
        _check(load().tdgl_voltage_grad_noalloc(self._ctx, nsteps, window_begin, ckpt_every, ctypes.byref(v),
                                                self._dev(grad, torch.float32)))
        return v.value, grad

    def profile_start(self, classes=None):
        mask = 0
        for c in (classes or KERNEL_CLASSES):
            mask |= 1 << KERNEL_CLASSES.index(c)
        _check(load().tdgl_profile_start(self._ctx, mask))

    def profile_stop(self):
        p = Prof()
        _check(load().tdgl_profile_stop(self._ctx, ctypes.byref(p)))
        return p.as_dict()

    def observables(self, inst=0):
        o = Obs()
        _check(load().tdgl_observables(self._ctx, inst, ctypes.byref(o)))
        return o.as_dict()


_VOLTAGE_FN = None


def _voltage_fn():
    global _VOLTAGE_FN
    if _VOLTAGE_FN is None:
        import torch

        class VoltageFn(torch.autograd.Function):
            """Vbar(eps) of a driven one-instance solver as a torch function.

            The forward runs nsteps implicit steps from the solver's current
            state and, when eps needs a gradient, the checkpointed reverse
            sweep in the same call (the step states exist only while the
            solver replays them), keeping dVbar/deps for the backward."""

            @staticmethod
            def forward(ctx, eps, solver, nsteps, window_begin, ckpt_every):
                solver.set_eps(eps.detach())
                if ctx.needs_input_grad[0]:
                    v, g = solver.voltage_grad(nsteps, window_begin, ckpt_every)
                    ctx.save_for_backward(g)
                else:
                    if window_begin > 0:
                        solver.step(window_begin, stats=False)
                    solver.window_reset()
                    solver.step(nsteps - window_begin, stats=False)
                    v = solver.observables()["E_mean"]
                return torch.tensor(v, dtype=torch.float64, device=eps.device)

            @staticmethod
            def backward(ctx, gout):
                (g,) = ctx.saved_tensors
                return gout.to(g.dtype) * g, None, None, None, None

        _VOLTAGE_FN = VoltageFn
    return _VOLTAGE_FN


def voltage(solver, eps, nsteps, window_begin=0, ckpt_every=50):
    """Time-averaged E_x over steps window_begin..nsteps-1 of a run from the
    solver's current state, differentiable with respect to eps (float32,
    shape (nz, ny, nx), CUDA).  Advances the solver by nsteps steps."""
    return _voltage_fn().apply(eps, solver, nsteps, window_begin, ckpt_every)
