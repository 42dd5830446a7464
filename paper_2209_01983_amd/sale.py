"""Thin ctypes binding of libsale.so (the C ABI in include/sale.h).

The functions named like the C entry points only marshal arguments; every
step of the method runs in the library's HIP kernels. ``SaleRun`` is a small
convenience owner: it allocates the device workspace as a torch uint8 tensor
and passes torch's current HIP stream (PyTorch is used for device memory and
streams only).

torch is imported before the library is loaded so that the process holds a
single HIP runtime (torch's, which has the same soname). A missing build
raises an error: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# SALE_LIB may name another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("SALE_LIB") or os.path.join(HERE, "libsale.so")

# ---- constants (include/sale.h) ----------------------------------------------
SALE_OK, SALE_DONE = 0, 1
SALE_EINVAL, SALE_ENOMEM, SALE_EHIP, SALE_ENUMERIC, SALE_ETANGLE, SALE_EBUSY = -1, -2, -3, -4, -5, -6
SALE_FP64, SALE_MIXED32 = 0, 1
SALE_BC_REFLECT = 0
SALE_SOD_X, SALE_SEDOV_CORNER, SALE_USER, SALE_NOH = 0, 1, 2, 3
SALE_FLAG_TANGLE, SALE_FLAG_NUMERIC = 1, 2
SALE_F_RHO, SALE_F_E, SALE_F_P, SALE_F_Q = 1 << 0, 1 << 1, 1 << 2, 1 << 3
SALE_F_U, SALE_F_V, SALE_F_W = 1 << 4, 1 << 5, 1 << 6
SALE_F_STATE, SALE_F_TOTALS, SALE_F_CLOCK = 1 << 7, 1 << 8, 1 << 9
SALE_F_X, SALE_F_Y, SALE_F_Z = 1 << 10, 1 << 11, 1 << 12
SALE_EULERIAN, SALE_LAGRANGIAN = 0, 1

FIELD_BITS = {"rho": SALE_F_RHO, "e": SALE_F_E, "p": SALE_F_P, "q": SALE_F_Q,
              "u": SALE_F_U, "v": SALE_F_V, "w": SALE_F_W, "x": SALE_F_X, "y": SALE_F_Y, "z": SALE_F_Z}
CELL_FIELDS = ("rho", "e", "p", "q")
NODE_FIELDS = ("u", "v", "w", "x", "y", "z")

# functions the header declares (checked by the tests against include/sale.h)
EXPORTS = ("sale_workspace_bytes", "sale_init", "sale_init_static", "sale_step", "sale_run", "sale_fields",
           "sale_step_timed", "sale_set_launch", "sale_status", "sale_destroy", "sale_strerror")
POOL_EXPORTS = ("sale_pool_create", "sale_pool_admit", "sale_pool_advance", "sale_pool_poll",
                "sale_pool_fields", "sale_pool_release", "sale_pool_destroy")


class sale_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("gamma", C.c_double), ("cfl", C.c_double),
                ("c_quad", C.c_double), ("c_lin", C.c_double),
                ("t_end", C.c_double), ("precision", C.c_int32), ("bc", C.c_int32 * 6),
                ("remap_order", C.c_int32), ("mode", C.c_int32), ("c_hg", C.c_double)]


class sale_problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("sod", C.c_double * 5), ("sedov", C.c_double * 3),
                ("noh", C.c_double * 3), ("noh_dims", C.c_int32), ("rho", C.c_void_p), ("e", C.c_void_p), ("u", C.c_void_p), ("v", C.c_void_p),
                ("w", C.c_void_p), ("user_on_device", C.c_int32), ("t0", C.c_double),
                ("step0", C.c_int64)]


_lib = None


class SaleError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {sale_strerror(code)} ({code})")


def lib():
    """Load libsale.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2209_01983_amd.build`")
        L = C.CDLL(LIB_PATH)
        cp = C.POINTER(sale_config)
        pp = C.POINTER(sale_problem)
        L.sale_workspace_bytes.argtypes = [cp, C.POINTER(C.c_size_t)]
        L.sale_workspace_bytes.restype = C.c_int
        L.sale_init.argtypes = [cp, pp, C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.sale_init.restype = C.c_int
        L.sale_init_static.argtypes = [cp, pp, C.c_void_p, C.POINTER(C.c_size_t), C.c_void_p,
                                       C.POINTER(C.c_void_p)]
        L.sale_init_static.restype = C.c_int
        L.sale_step.argtypes = [C.c_void_p]
        L.sale_step.restype = C.c_int
        L.sale_run.argtypes = [C.c_void_p, C.c_double, C.c_int64]
        L.sale_run.restype = C.c_int
        L.sale_fields.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(C.c_void_p), C.c_int, C.c_int]
        L.sale_fields.restype = C.c_int
        L.sale_step_timed.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_float)]
        L.sale_step_timed.restype = C.c_int
        L.sale_set_launch.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32]
        L.sale_set_launch.restype = C.c_int
        L.sale_status.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
        L.sale_status.restype = C.c_int
        L.sale_destroy.argtypes = [C.c_void_p]
        L.sale_destroy.restype = None
        L.sale_strerror.argtypes = [C.c_int]
        L.sale_strerror.restype = C.c_char_p
        L.sale_pool_create.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.POINTER(C.c_void_p)]
        L.sale_pool_create.restype = C.c_int
        L.sale_pool_admit.argtypes = [C.c_void_p, cp, pp, C.c_int64, C.POINTER(C.c_int32)]
        L.sale_pool_admit.restype = C.c_int
        L.sale_pool_advance.argtypes = [C.c_void_p, C.c_int32]
        L.sale_pool_advance.restype = C.c_int
        L.sale_pool_poll.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)]
        L.sale_pool_poll.restype = C.c_int
        L.sale_pool_fields.argtypes = [C.c_void_p, C.c_int32, C.c_uint32, C.POINTER(C.c_void_p), C.c_int,
                                       C.c_int]
        L.sale_pool_fields.restype = C.c_int
        L.sale_pool_release.argtypes = [C.c_void_p, C.c_int32]
        L.sale_pool_release.restype = C.c_int
        L.sale_pool_destroy.argtypes = [C.c_void_p]
        L.sale_pool_destroy.restype = None
        _lib = L
    return _lib


# ---- C entry points -------------------------------------------------------------
def sale_workspace_bytes(cfg: sale_config) -> int:
    n = C.c_size_t(0)
    rc = lib().sale_workspace_bytes(C.byref(cfg), C.byref(n))
    if rc != SALE_OK:
        raise SaleError(rc, "sale_workspace_bytes")
    return n.value


def sale_init(cfg: sale_config, prob: sale_problem, d_ws: int, ws_bytes: int, stream: int):
    """Returns (code, ctx handle or None)."""
    ctx = C.c_void_p(None)
    rc = lib().sale_init(C.byref(cfg), C.byref(prob), C.c_void_p(d_ws), ws_bytes, C.c_void_p(stream),
                         C.byref(ctx))
    return rc, (ctx if rc == SALE_OK else None)


def sale_init_static(cfg: sale_config, prob: sale_problem, d_state, state_bytes: int, stream: int):
    """Returns (code, ctx handle or None, state bytes). With d_state None: the
    size query (code, None, bytes cfg needs)."""
    ctx = C.c_void_p(None)
    n = C.c_size_t(state_bytes)
    rc = lib().sale_init_static(C.byref(cfg), C.byref(prob), C.c_void_p(d_state), C.byref(n),
                                C.c_void_p(stream), C.byref(ctx))
    return rc, (ctx if rc == SALE_OK and d_state else None), n.value


def sale_step(ctx) -> int:
    return lib().sale_step(ctx)


def sale_run(ctx, t_end: float, max_steps: int) -> int:
    return lib().sale_run(ctx, t_end, max_steps)


def sale_fields(ctx, mask: int, dst_ptrs, dst_on_device: int, as_fp64: int) -> int:
    arr = (C.c_void_p * max(1, len(dst_ptrs)))(*[C.c_void_p(p) for p in dst_ptrs])
    return lib().sale_fields(ctx, mask, arr, dst_on_device, as_fp64)


def sale_step_timed(ctx, n: int):
    """Returns (code, [ms start, ms Lagrange+geometry, ms remap]) summed over n steps."""
    ms = (C.c_float * 3)()
    rc = lib().sale_step_timed(ctx, n, ms)
    return rc, [float(x) for x in ms]


def sale_set_launch(ctx, rows_lagrange: int, rows_remap: int, target_blocks: int) -> int:
    return lib().sale_set_launch(ctx, rows_lagrange, rows_remap, target_blocks)


def sale_status(ctx):
    """Returns (code, flags)."""
    f = C.c_int32(0)
    rc = lib().sale_status(ctx, C.byref(f))
    return rc, f.value


def sale_destroy(ctx) -> None:
    lib().sale_destroy(ctx)


def sale_strerror(code: int) -> str:
    return lib().sale_strerror(code).decode()


def sale_pool_create(precision: int, max_runs: int, d_arena: int, arena_bytes: int, stream: int):
    """Returns (code, pool handle or None)."""
    pool = C.c_void_p(None)
    rc = lib().sale_pool_create(precision, max_runs, C.c_void_p(d_arena), arena_bytes, C.c_void_p(stream),
                                C.byref(pool))
    return rc, (pool if rc == SALE_OK else None)


def sale_pool_admit(pool, cfg: sale_config, prob: sale_problem, n_steps: int):
    """Returns (code, slot)."""
    slot = C.c_int32(-1)
    rc = lib().sale_pool_admit(pool, C.byref(cfg), C.byref(prob), n_steps, C.byref(slot))
    return rc, slot.value


def sale_pool_advance(pool, max_steps_per_run: int) -> int:
    return lib().sale_pool_advance(pool, max_steps_per_run)


def sale_pool_poll(pool, cap: int):
    """Returns (code, list of finished slots)."""
    buf = (C.c_int32 * max(1, cap))()
    n = C.c_int32(0)
    rc = lib().sale_pool_poll(pool, buf, cap, C.byref(n))
    return rc, list(buf[: n.value])


def sale_pool_fields(pool, slot: int, mask: int, dst_ptrs, dst_on_device: int, as_fp64: int) -> int:
    arr = (C.c_void_p * max(1, len(dst_ptrs)))(*[C.c_void_p(p) for p in dst_ptrs])
    return lib().sale_pool_fields(pool, slot, mask, arr, dst_on_device, as_fp64)


def sale_pool_release(pool, slot: int) -> int:
    return lib().sale_pool_release(pool, slot)


def sale_pool_destroy(pool) -> None:
    lib().sale_pool_destroy(pool)


# ---- helpers ------------------------------------------------------------------------
def make_config(nx, ny, nz, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), gamma=1.4, cfl=0.5,
                c_quad=1.0, c_lin=0.5, t_end=1.0, precision=SALE_FP64, remap_order=1,
                mode=SALE_EULERIAN, c_hg=0.1) -> sale_config:
    return sale_config(nx, ny, nz, (C.c_double * 3)(*lo), (C.c_double * 3)(*hi), gamma, cfl, c_quad,
                       c_lin, t_end, precision, (C.c_int32 * 6)(*([SALE_BC_REFLECT] * 6)), remap_order,
                       mode, c_hg)


def sod_problem(x_split=0.5, rhoL=1.0, pL=1.0, rhoR=0.125, pR=0.1, t0=0.0, step0=0) -> sale_problem:
    p = sale_problem()
    p.kind = SALE_SOD_X
    p.sod = (C.c_double * 5)(x_split, rhoL, pL, rhoR, pR)
    p.t0, p.step0 = t0, step0
    return p


def sedov_problem(rho0=1.0, p0=1e-6, edep=0.125, t0=0.0, step0=0) -> sale_problem:
    p = sale_problem()
    p.kind = SALE_SEDOV_CORNER
    p.sedov = (C.c_double * 3)(rho0, p0, edep)
    p.t0, p.step0 = t0, step0
    return p


def noh_problem(rho0=1.0, p0=1e-6, u0=1.0, dims=3, t0=0.0, step0=0) -> sale_problem:
    """Noh implosion toward the corner lo (use gamma = 5/3 in the config)."""
    p = sale_problem()
    p.kind = SALE_NOH
    p.noh = (C.c_double * 3)(rho0, p0, u0)
    p.noh_dims = dims
    p.t0, p.step0 = t0, step0
    return p


def user_problem(rho, e, u, v, w, t0=0.0, step0=0):
    """SALE_USER from numpy float64 arrays (host) or torch float64 CUDA tensors
    (device). Returns (problem, keepalive)."""
    arrs = [rho, e, u, v, w]
    p = sale_problem()
    p.kind = SALE_USER
    p.t0, p.step0 = t0, step0
    if all(isinstance(a, np.ndarray) for a in arrs):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in arrs]
        ptrs = [a.ctypes.data for a in arrs]
        p.user_on_device = 0
    else:
        import torch
        arrs = [a.contiguous().to(torch.float64) for a in arrs]
        if not all(a.is_cuda for a in arrs):
            raise ValueError("user arrays must be all numpy or all CUDA tensors")
        ptrs = [a.data_ptr() for a in arrs]
        p.user_on_device = 1
    p.rho, p.e, p.u, p.v, p.w = ptrs
    return p, arrs


def _field_buffers(torch, device, names, cell_shape, node_shape, on_device):
    names = sorted(names, key=lambda n: FIELD_BITS[n])
    out, ptrs, mask = {}, [], 0
    for n in names:
        shape = cell_shape if n in CELL_FIELDS else node_shape
        if on_device:
            a = torch.empty(shape, dtype=torch.float64, device=device)
            ptrs.append(a.data_ptr())
        else:
            a = np.empty(shape, dtype=np.float64)
            ptrs.append(a.ctypes.data)
        out[n] = a
        mask |= FIELD_BITS[n]
    return out, ptrs, mask


class SaleRun:
    """One run: workspace as a torch uint8 tensor on `device`, torch's current
    stream as the library's stream. With static=True the context comes from
    sale_init_static: the tensor holds only the state part of the workspace,
    the intermediates live in the library's device array."""

    def __init__(self, cfg: sale_config, prob: sale_problem, device="cuda:0", keepalive=None, static=False):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device).cuda_stream
        if static:
            rc, _, self.nbytes = sale_init_static(cfg, prob, None, 0, self.stream)
            if rc != SALE_OK:
                raise SaleError(rc, "sale_init_static")
            self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            rc, self.ctx, _ = sale_init_static(cfg, prob, self.ws.data_ptr(), self.nbytes, self.stream)
        else:
            self.nbytes = sale_workspace_bytes(cfg)
            self.ws = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            rc, self.ctx = sale_init(cfg, prob, self.ws.data_ptr(), self.nbytes, self.stream)
        del keepalive
        if rc != SALE_OK:
            raise SaleError(rc, "sale_init_static" if static else "sale_init")
        self.cell_shape = (cfg.nz, cfg.ny, cfg.nx)
        self.node_shape = (cfg.nz + 1, cfg.ny + 1, cfg.nx + 1)

    def close(self):
        if getattr(self, "ctx", None):
            sale_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        for _ in range(n):
            rc = sale_step(self.ctx)
            if rc != SALE_OK:
                raise SaleError(rc, "sale_step")

    def step_timed(self, n=1):
        """n steps; per-kernel durations (ms) summed over them."""
        rc, ms = sale_step_timed(self.ctx, n)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_step_timed")
        return ms

    def set_launch(self, rows_lagrange=14, rows_remap=14, target_blocks=0):
        rc = sale_set_launch(self.ctx, rows_lagrange, rows_remap, target_blocks)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_set_launch")

    def run(self, t_end=-1.0, max_steps=1 << 40) -> int:
        return sale_run(self.ctx, t_end, max_steps)

    def status(self):
        return sale_status(self.ctx)

    def fields(self, names=("rho", "e", "u", "v", "w"), on_device=False):
        """Dict of float64 arrays in the logical layout (numpy, or torch CUDA
        tensors with on_device=True)."""
        out, ptrs, mask = _field_buffers(self.torch, self.device, names, self.cell_shape, self.node_shape,
                                         on_device)
        rc = sale_fields(self.ctx, mask, ptrs, int(on_device), 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_fields")
        return out

    def state(self):
        """(t, steps, next dt, status flags)."""
        o = np.zeros(4)
        rc = sale_fields(self.ctx, SALE_F_STATE, [o.ctypes.data], 0, 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_fields")
        return float(o[0]), int(o[1]), float(o[2]), int(o[3])

    def totals(self):
        """(total mass, total energy)."""
        o = np.zeros(2)
        rc = sale_fields(self.ctx, SALE_F_TOTALS, [o.ctypes.data], 0, 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_fields")
        return float(o[0]), float(o[1])


class Pool:
    """Many independent runs in one device arena (a torch uint8 tensor of
    `arena_bytes` on `device`), advanced together on torch's current stream
    (the library's persistent kernel or lockstep launches, chosen per advance
    unless SALE_POOL_PERSISTENT forces one)."""

    def __init__(self, arena_bytes, max_runs=256, precision=SALE_FP64, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device).cuda_stream
        rc, self.pool = sale_pool_create(precision, max_runs, self.arena.data_ptr(), int(arena_bytes),
                                         self.stream)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_create")
        self.max_runs = max_runs
        self.shapes = {}

    def close(self):
        if getattr(self, "pool", None):
            sale_pool_destroy(self.pool)
            self.pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, cfg: sale_config, prob: sale_problem, n_steps: int):
        """Slot of the admitted run, or None when the pool is full (SALE_EBUSY)."""
        rc, slot = sale_pool_admit(self.pool, cfg, prob, n_steps)
        if rc == SALE_EBUSY:
            return None
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_admit")
        self.shapes[slot] = ((cfg.nz, cfg.ny, cfg.nx), (cfg.nz + 1, cfg.ny + 1, cfg.nx + 1))
        return slot

    def advance(self, max_steps_per_run: int):
        rc = sale_pool_advance(self.pool, max_steps_per_run)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_advance")

    def poll(self, cap=None):
        rc, done = sale_pool_poll(self.pool, self.max_runs if cap is None else cap)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_poll")
        return done

    def fields(self, slot, names=("rho", "e", "u", "v", "w"), on_device=False):
        cell, node = self.shapes[slot]
        out, ptrs, mask = _field_buffers(self.torch, self.device, names, cell, node, on_device)
        rc = sale_pool_fields(self.pool, slot, mask, ptrs, int(on_device), 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_fields")
        return out

    def state(self, slot):
        """(t, steps, next dt, status flags) of one slot."""
        o = np.zeros(4)
        rc = sale_pool_fields(self.pool, slot, SALE_F_STATE, [o.ctypes.data], 0, 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_fields")
        return float(o[0]), int(o[1]), float(o[2]), int(o[3])

    def clock(self, slot):
        """(first advance, last completed step) of a slot, device wall clock in s."""
        o = np.zeros(2)
        rc = sale_pool_fields(self.pool, slot, SALE_F_CLOCK, [o.ctypes.data], 0, 1)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_fields")
        return float(o[0]), float(o[1])

    def release(self, slot):
        rc = sale_pool_release(self.pool, slot)
        if rc != SALE_OK:
            raise SaleError(rc, "sale_pool_release")
        self.shapes.pop(slot, None)
