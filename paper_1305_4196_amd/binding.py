"""ctypes binding of ``libmd.so`` -- argument marshalling only.

Every function mirrors one entry point of ``include/md.h`` and takes torch
tensors that already live on the GPU (float64, contiguous, [3][N] per-atom
layout); the work itself runs in the HIP kernels.  There is no CPU fallback:
if the library is missing, or no GPU is visible, calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmd.so")

MD_OK, MD_ERR_ARG, MD_ERR_BOX, MD_ERR_CAPACITY, MD_ERR_NONFINITE, MD_ERR_HIP, MD_ERR_STATE, MD_ERR_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7
MD_FP64, MD_MIXED = 0, 1
MD_LIST_FULL, MD_LIST_HALF, MD_LIST_WAVES, MD_LIST_DEPS = 0, 1, 2, 3
MD_POT_LJ, MD_POT_EAM = 0, 1
FLAG_OVERFLOW, FLAG_NONFINITE, FLAG_SCHEDULE = 1, 2, 4

EXPORTS = ["md_create", "md_destroy", "md_build_cells", "md_build_neighbor_list",
           "md_compute_forces", "md_verlet_step", "md_force_vjp", "md_get_status",
           "md_get_neighbor_list", "md_get_cells", "md_get_waves", "md_get_task_graph", "md_set_tuning", "md_query", "md_profile",
           "md_profile_detail", "md_compute_forces_noalloc", "md_last_error"]


class MDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"md error {code}: {msg}")
        self.code = code


class md_spline(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("x0", C.c_double), ("h", C.c_double), ("coef", C.c_void_p)]


class md_potential(C.Structure):
    _fields_ = [("kind", C.c_int32), ("rc", C.c_double), ("lj_params", C.c_void_p),
                ("phi", md_spline), ("rho", md_spline), ("embed", md_spline),
                ("rc_phi", C.c_double), ("rc_rho", C.c_double)]


_lib: Optional[C.CDLL] = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libmd.so (built by ``paper_1305_4196_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: run __graft_entry__.build() first")
    L = C.CDLL(path)
    vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    L.md_create.argtypes = [P(vp), i64, i32, P(i64)]
    L.md_create.restype = C.c_int
    L.md_destroy.argtypes = [vp]
    L.md_destroy.restype = None
    L.md_build_cells.argtypes = [vp, vp, P(d), d, d, vp]
    L.md_build_neighbor_list.argtypes = [vp, i32, vp]
    L.md_compute_forces.argtypes = [vp, P(md_potential), i32, vp, vp, vp, vp]
    L.md_compute_forces_noalloc.argtypes = [vp, P(md_potential), i32, vp, vp, vp, vp]
    L.md_verlet_step.argtypes = [vp, P(md_potential), i32, i32, vp, vp, vp, d, d, i32, vp, i32, vp, vp]
    L.md_force_vjp.argtypes = [vp, P(md_potential), i32, vp, vp, vp, vp, vp, vp]
    L.md_get_status.argtypes = [vp, P(i32), P(i64)]
    L.md_get_neighbor_list.argtypes = [vp, P(i64), P(i32), i64]
    L.md_get_neighbor_list.restype = i64
    L.md_get_cells.argtypes = [vp, P(i32), P(i32), P(i64)]
    L.md_get_waves.argtypes = [vp, P(i32), i64, P(i64)]
    L.md_get_task_graph.argtypes = [vp, P(i32), P(i32), i64]
    L.md_get_task_graph.restype = i64
    L.md_set_tuning.argtypes = [vp, i32, i32]
    L.md_query.argtypes = [vp, i32, P(i64)]
    L.md_profile.argtypes = [vp, i32, P(d), P(i64), P(d), P(i64)]
    L.md_profile_detail.argtypes = [vp, P(d), i32]
    L.md_last_error.argtypes = [vp]
    L.md_last_error.restype = C.c_char_p
    for name in ("md_build_cells", "md_build_neighbor_list", "md_compute_forces", "md_compute_forces_noalloc",
                 "md_verlet_step",
                 "md_force_vjp", "md_get_status", "md_get_cells", "md_set_tuning", "md_query", "md_profile",
                 "md_profile_detail"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(None)
    if not t.is_cuda:
        raise ValueError("tensors handed to the library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors handed to the library must be contiguous")
    return C.c_void_p(t.data_ptr())


def _check(ctx, rc: int):
    if rc != MD_OK:
        msg = load().md_last_error(ctx).decode() if ctx else ""
        raise MDError(rc, msg)


# ----------------------------------------------------------------- potentials
class DevicePotential:
    """A workloads.Potential with its parameters in device memory."""

    def __init__(self, pot, device="cuda", params=None):
        import torch
        self.pot = pot
        self.s = md_potential()
        self.s.kind = MD_POT_LJ if pot.kind == "lj" else MD_POT_EAM
        self.s.rc = pot.rc
        if pot.kind == "lj":
            self.params = (torch.tensor([pot.eps, pot.sigma], dtype=torch.float64, device=device)
                           if params is None else params)
            self.s.lj_params = self.params.data_ptr()
        else:
            if params is None:
                flat = np.concatenate([pot.phi.coef.ravel(), pot.rho.coef.ravel(),
                                       pot.embed.coef.ravel()])
                params = torch.tensor(flat, dtype=torch.float64, device=device)
            self.params = params
            o = 0
            for name in ("phi", "rho", "embed"):
                sp = getattr(pot, name)
                cs = getattr(self.s, name)
                cs.n_knots = sp.n_knots
                cs.x0 = sp.x0
                cs.h = sp.h
                cs.coef = self.params.data_ptr() + 8 * o
                o += sp.coef.size
            self.s.rc_phi = pot.rc_phi
            self.s.rc_rho = pot.rc_rho
        if not (self.params.is_cuda and self.params.dtype == torch.float64 and self.params.is_contiguous()):
            raise ValueError("parameters must be a contiguous float64 GPU tensor")

    @property
    def n_params(self) -> int:
        return int(self.params.numel())


# ----------------------------------------------------------------- entry points
class Context:
    """Owns an md_ctx; destroyed with the object."""

    def __init__(self, n: int, offsets: Sequence[int]):
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        h = C.c_void_p()
        rc = load().md_create(C.byref(h), int(n), int(off.size - 1),
                              off.ctypes.data_as(C.POINTER(C.c_int64)))
        if rc != MD_OK:
            raise MDError(rc, "md_create failed")
        self.h = h
        self.n = int(n)
        self.n_replicas = int(off.size - 1)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.md_destroy(h)
            self.h = None


def md_create(n: int, offsets: Sequence[int]) -> Context:
    return Context(n, offsets)


def md_destroy(ctx: Context):
    if ctx.h is not None and ctx.h.value:
        load().md_destroy(ctx.h)
        ctx.h = None


def md_build_cells(ctx: Context, pos, boxes, rc: float, skin: float, stream=None):
    b = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
    _check(ctx.h, load().md_build_cells(ctx.h, _ptr(pos), b.ctypes.data_as(C.POINTER(C.c_double)),
                                        float(rc), float(skin), _stream(stream)))


def md_build_neighbor_list(ctx: Context, kind: int = MD_LIST_FULL, stream=None):
    _check(ctx.h, load().md_build_neighbor_list(ctx.h, int(kind), _stream(stream)))


def md_compute_forces(ctx: Context, pot: DevicePotential, precision: int, forces, energy=None,
                      virial=None, stream=None):
    _check(ctx.h, load().md_compute_forces(ctx.h, C.byref(pot.s), int(precision), _ptr(forces),
                                           _ptr(energy), _ptr(virial), _stream(stream)))


def md_compute_forces_noalloc(ctx: Context, pot: DevicePotential, precision: int, forces, energy=None,
                              virial=None, stream=None):
    _check(ctx.h, load().md_compute_forces_noalloc(ctx.h, C.byref(pot.s), int(precision), _ptr(forces),
                                                   _ptr(energy), _ptr(virial), _stream(stream)))


def md_verlet_step(ctx: Context, pot: DevicePotential, precision: int, kind: int, pos, vel, forces,
                   dt: float, mass: float, n_steps: int, hist=None, rebuilds=None, stream=None,
                   hist_every: int = 1):
    _check(ctx.h, load().md_verlet_step(ctx.h, C.byref(pot.s), int(precision), int(kind), _ptr(pos),
                                        _ptr(vel), _ptr(forces), float(dt), float(mass), int(n_steps),
                                        _ptr(hist), int(hist_every), _ptr(rebuilds), _stream(stream)))


def md_force_vjp(ctx: Context, pot: DevicePotential, precision: int, pos, u, vE, g_pos=None,
                 g_params=None, stream=None):
    _check(ctx.h, load().md_force_vjp(ctx.h, C.byref(pot.s), int(precision), _ptr(pos), _ptr(u),
                                      _ptr(vE), _ptr(g_pos), _ptr(g_params), _stream(stream)))


def md_get_status(ctx: Context) -> Tuple[int, int, int]:
    """(return code, device flags, capacity); synchronises."""
    f = C.c_int32()
    r = C.c_int64()
    code = load().md_get_status(ctx.h, C.byref(f), C.byref(r))
    return int(code), int(f.value), int(r.value)


def md_get_neighbor_list(ctx: Context) -> Tuple[np.ndarray, np.ndarray]:
    """CSR (start[N+1], nbr) over user indices; synchronises."""
    L = load()
    start = np.zeros(ctx.n + 1, dtype=np.int64)
    tot = L.md_get_neighbor_list(ctx.h, start.ctypes.data_as(C.POINTER(C.c_int64)), None, 0)
    if tot < 0:
        _check(ctx.h, int(tot))
    nbr = np.zeros(max(int(tot), 1), dtype=np.int32)
    tot2 = L.md_get_neighbor_list(ctx.h, start.ctypes.data_as(C.POINTER(C.c_int64)),
                                  nbr.ctypes.data_as(C.POINTER(C.c_int32)), int(tot))
    if tot2 != tot:
        raise MDError(MD_ERR_STATE, "neighbour list changed during export")
    return start, nbr[:tot]


def md_get_cells(ctx: Context) -> Tuple[np.ndarray, np.ndarray]:
    """(cell_start[C+1], order[N]) where order[s] is the user index of sorted slot s."""
    L = load()
    nc = C.c_int64()
    _check(ctx.h, L.md_get_cells(ctx.h, None, None, C.byref(nc)))
    cs = np.zeros(nc.value + 1, dtype=np.int32)
    order = np.zeros(ctx.n, dtype=np.int32)
    _check(ctx.h, L.md_get_cells(ctx.h, cs.ctypes.data_as(C.POINTER(C.c_int32)),
                                 order.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(nc)))
    return cs, order


def md_get_waves(ctx: Context) -> Tuple[np.ndarray, int]:
    """(colour[B], number of waves) of the current wave schedule."""
    L = load()
    nb = C.c_int64()
    _check(ctx.h, min(0, L.md_get_waves(ctx.h, None, 0, C.byref(nb))))
    col = np.zeros(nb.value, dtype=np.int32)
    nw = L.md_get_waves(ctx.h, col.ctypes.data_as(C.POINTER(C.c_int32)), nb.value, None)
    _check(ctx.h, min(0, nw))
    return col, int(nw)


def md_get_task_graph(ctx: Context) -> Tuple[np.ndarray, np.ndarray]:
    """(succ_off[B+1], succ[E]) of the current dependent schedule."""
    L = load()
    ne = L.md_get_task_graph(ctx.h, None, None, 0)
    _check(ctx.h, int(min(0, ne)))
    nb = C.c_int64()
    _check(ctx.h, min(0, L.md_get_waves(ctx.h, None, 0, C.byref(nb))))
    off = np.zeros(nb.value + 1, dtype=np.int32)
    succ = np.zeros(max(int(ne), 1), dtype=np.int32)
    P = C.POINTER(C.c_int32)
    _check(ctx.h, int(min(0, L.md_get_task_graph(ctx.h, off.ctypes.data_as(P), succ.ctypes.data_as(P), int(ne)))))
    return off, succ[:int(ne)]


def md_set_tuning(ctx: Context, key: int, value: int):
    _check(ctx.h, load().md_set_tuning(ctx.h, int(key), int(value)))


def md_query(ctx: Context, key: int) -> int:
    v = C.c_int64()
    _check(ctx.h, load().md_query(ctx.h, int(key), C.byref(v)))
    return int(v.value)


def md_profile(ctx: Context, enable: bool, launches: bool = True):
    """Start (enable=True) or stop event timing; on stop returns
    (force_ms, force_launches, list_ms, list_launches).  launches=False times
    only md_verlet_step's setup and step loop (no event pair per launch)."""
    fm, ln = C.c_double(), C.c_double()
    fn, lc = C.c_int64(), C.c_int64()
    mode = 0 if not enable else (1 if launches else 2)
    _check(ctx.h, load().md_profile(ctx.h, mode, C.byref(fm), C.byref(fn), C.byref(ln), C.byref(lc)))
    if enable:
        return None
    return float(fm.value), int(fn.value), float(ln.value), int(lc.value)


def md_profile_detail(ctx: Context) -> dict:
    """Timings of the profiled md_verlet_step calls (after md_profile(ctx, False))."""
    out = (C.c_double * 8)()
    _check(ctx.h, load().md_profile_detail(ctx.h, out, 8))
    v = list(out)
    return {"loop_ms": v[0], "loop_steps": int(v[1]), "setup_ms": v[2],
            "force_plain_ms": v[3], "force_plain_n": int(v[4]),
            "force_energy_ms": v[5], "force_energy_n": int(v[6]), "force_setup_ms": v[7]}
