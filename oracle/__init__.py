"""CPU FP64 oracle of the short-range MD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it; the two meet only in the seeded input generators.

The arithmetic lives in ``md_oracle.c`` (plain C, binary64, contraction off);
this module is ctypes marshalling plus a few plain-numpy helpers that hold no
method arithmetic of their own.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "md_oracle.c")
_LIB = os.path.join(_HERE, "libmdoracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-std=c99", "-Wall", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib: Optional[C.CDLL] = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.orc_wrap.argtypes = [C.c_int64, _d, _d]
        L.orc_grid.argtypes = [_d, C.c_double, _i32]
        L.orc_grid.restype = C.c_int
        L.orc_bin.argtypes = [C.c_int64, _d, _d, _i32, _i32, _i32, _i32]
        L.orc_pairs_brute.argtypes = [C.c_int64, _d, _d, C.c_double, C.c_int, C.c_int64, _i32, _i32]
        L.orc_pairs_brute.restype = C.c_int64
        L.orc_neighbor_list.argtypes = [C.c_int64, _d, _d, C.c_double, C.c_int, _i64, C.c_int64, _i32]
        L.orc_neighbor_list.restype = C.c_int64
        L.orc_lj.argtypes = [C.c_int64, _d, _d, C.c_double, C.c_double, C.c_double,
                             C.c_int64, _i32, _i32, _d, _d]
        L.orc_lj_atoms.argtypes = [C.c_int64, _d, _d, C.c_double, C.c_double, C.c_double,
                                   C.c_int64, _i32, _d, _d]
        L.orc_spline_eval.argtypes = [C.c_int32, C.c_double, C.c_double, _d, C.c_int, C.c_int64, _d, _d]
        L.orc_eam.argtypes = [C.c_int64, _d, _d, _i32, _d, _d, _d, _d, _d, C.c_double, C.c_double,
                              C.c_int64, _i32, _i32, _d, _d, _d, _d]
        L.orc_verlet.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_int, _d, _i32, _d, _d, _d, _d, _d,
                                 C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_int32, _d, _i32]
        L.orc_verlet.restype = C.c_int
        L.orc_verlet_omp.argtypes = list(L.orc_verlet.argtypes) + [C.c_int32]
        L.orc_verlet_omp.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        L.orc_lj_vjp.argtypes = [C.c_int64, _d, _d, C.c_double, C.c_double, C.c_double,
                                 C.c_int64, _i32, _i32, _d, C.c_double, _d, _d]
        L.orc_eam_vjp.argtypes = [C.c_int64, _d, _d, _i32, _d, _d, _d, _d, _d, C.c_double, C.c_double,
                                  C.c_int64, _i32, _i32, _d, C.c_double, _d, _d, _d, _d]
        _lib = L
    return _lib


def _p(a: np.ndarray, ct=_d):
    return a.ctypes.data_as(ct)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _box(L) -> np.ndarray:
    L = _f64(L).reshape(-1)
    if L.size == 1:
        L = np.repeat(L, 3)
    return np.ascontiguousarray(L)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def wrap(x: np.ndarray, L) -> np.ndarray:
    y = _f64(x).copy()
    lib().orc_wrap(y.shape[1], _p(y), _p(_box(L)))
    return y


def grid(L, rl: float) -> Optional[Tuple[int, int, int]]:
    nc = np.zeros(3, dtype=np.int32)
    if lib().orc_grid(_p(_box(L)), rl, _p(nc, _i32)) != 0:
        return None
    return tuple(int(v) for v in nc)


def bin_cells(x: np.ndarray, L, rl: float) -> Dict[str, np.ndarray]:
    """Cells of wrapped positions: cell_of[n], cell_start[ncell+1], order[n]."""
    x = _f64(x)
    nc = grid(L, rl)
    if nc is None:
        raise ValueError("box shorter than twice the list cutoff")
    n = x.shape[1]
    ncell = nc[0] * nc[1] * nc[2]
    cell_of = np.zeros(n, dtype=np.int32)
    cs = np.zeros(ncell + 1, dtype=np.int32)
    order = np.zeros(n, dtype=np.int32)
    lib().orc_bin(n, _p(x), _p(_box(L)), _p(np.array(nc, dtype=np.int32), _i32),
                  _p(cell_of, _i32), _p(cs, _i32), _p(order, _i32))
    return dict(nc=np.array(nc), cell_of=cell_of, cell_start=cs, order=order)


# --------------------------------------------------------------------------
# pair sets
# --------------------------------------------------------------------------
def pairs_brute(x: np.ndarray, L, cut: float, full: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    x = _f64(x)
    n = x.shape[1]
    m = lib().orc_pairs_brute(n, _p(x), _p(_box(L)), cut, int(full), 0, None, None)
    pi = np.zeros(max(m, 1), dtype=np.int32)
    pj = np.zeros(max(m, 1), dtype=np.int32)
    lib().orc_pairs_brute(n, _p(x), _p(_box(L)), cut, int(full), m, _p(pi, _i32), _p(pj, _i32))
    return pi[:m], pj[:m]


def neighbor_list(x: np.ndarray, L, rl: float, full: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """CSR (start[n+1], nbr[...]) by linked cells; x must be wrapped."""
    x = _f64(x)
    n = x.shape[1]
    start = np.zeros(n + 1, dtype=np.int64)
    tot = lib().orc_neighbor_list(n, _p(x), _p(_box(L)), rl, int(full), _p(start, _i64), 0, None)
    if tot < 0:
        raise ValueError("box shorter than twice the list cutoff")
    nbr = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbor_list(n, _p(x), _p(_box(L)), rl, int(full), _p(start, _i64), tot,
                            _p(nbr, _i32))
    return start, nbr[:tot]


def shell_list(x: np.ndarray, L, rl: float) -> Tuple[np.ndarray, np.ndarray]:
    """CSR of the half list over 14 of the 27 cells (each pair once, held by the
    atom that sees the partner's cell in the forward half); x must be wrapped."""
    x = _f64(x)
    n = x.shape[1]
    start = np.zeros(n + 1, dtype=np.int64)
    tot = lib().orc_neighbor_list(n, _p(x), _p(_box(L)), rl, 2, _p(start, _i64), 0, None)
    if tot < 0:
        raise ValueError("box shorter than twice the list cutoff")
    nbr = np.zeros(max(tot, 1), dtype=np.int32)
    lib().orc_neighbor_list(n, _p(x), _p(_box(L)), rl, 2, _p(start, _i64), tot, _p(nbr, _i32))
    return start, nbr[:tot]


def half_pairs(x: np.ndarray, L, rl: float) -> Tuple[np.ndarray, np.ndarray]:
    """Unordered pairs within rl (each once) from the linked-cell half list."""
    start, nbr = neighbor_list(x, L, rl, full=False)
    n = start.size - 1
    pi = np.repeat(np.arange(n, dtype=np.int32), np.diff(start)).astype(np.int32)
    return pi, nbr.astype(np.int32)


# --------------------------------------------------------------------------
# potentials
# --------------------------------------------------------------------------
def lj(x, L, pi, pj, eps=1.0, sigma=1.0, rc=2.5):
    """(F[3][n], E, W) over unordered pairs."""
    x = _f64(x)
    n = x.shape[1]
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    F = np.zeros((3, n))
    ew = np.zeros(2)
    lib().orc_lj(n, _p(x), _p(_box(L)), rc, eps, sigma, pi.size, _p(pi, _i32), _p(pj, _i32),
                 _p(F), _p(ew))
    return F, float(ew[0]), float(ew[1])


def lj_atoms(x, L, atoms, eps=1.0, sigma=1.0, rc=2.5):
    """Per-atom force and half pair energy of selected atoms, exhaustive over j."""
    x = _f64(x)
    atoms = np.ascontiguousarray(atoms, dtype=np.int32)
    m = atoms.size
    F = np.zeros((3, m))
    e = np.zeros(m)
    lib().orc_lj_atoms(x.shape[1], _p(x), _p(_box(L)), rc, eps, sigma, m, _p(atoms, _i32),
                       _p(F), _p(e))
    return F, e


def spline_eval(sp, xs, extrap: bool = False) -> np.ndarray:
    """(3, m): value, first and second derivative of a table at xs."""
    xs = _f64(xs).reshape(-1)
    out = np.zeros((3, xs.size))
    coef = _f64(sp.coef)
    lib().orc_spline_eval(coef.shape[0] + 1, sp.x0, sp.h, _p(coef), int(extrap), xs.size,
                          _p(xs), _p(out))
    return out


def _eam_args(pot):
    nk = np.array([pot.phi.n_knots, pot.rho.n_knots, pot.embed.n_knots], dtype=np.int32)
    x0 = np.array([pot.phi.x0, pot.rho.x0, pot.embed.x0])
    h = np.array([pot.phi.h, pot.rho.h, pot.embed.h])
    cp, cr, ce = _f64(pot.phi.coef), _f64(pot.rho.coef), _f64(pot.embed.coef)
    return nk, x0, h, cp, cr, ce


def eam(x, L, pi, pj, pot):
    """(F[3][n], E, W, rho[n], F'(rho)[n]) over unordered pairs."""
    x = _f64(x)
    n = x.shape[1]
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    nk, x0, h, cp, cr, ce = _eam_args(pot)
    F = np.zeros((3, n))
    ew = np.zeros(2)
    rho = np.zeros(n)
    Fp = np.zeros(n)
    lib().orc_eam(n, _p(x), _p(_box(L)), _p(nk, _i32), _p(x0), _p(h), _p(cp), _p(cr), _p(ce),
                  pot.rc_phi, pot.rc_rho, pi.size, _p(pi, _i32), _p(pj, _i32), _p(F), _p(ew),
                  _p(rho), _p(Fp))
    return F, float(ew[0]), float(ew[1]), rho, Fp


def forces(x, L, pot, skin: float = 0.0):
    """(F, E, W) of one periodic system; pairs from the linked-cell half list."""
    x = wrap(x, L)
    pi, pj = half_pairs(x, L, pot.rc + skin)
    if pot.kind == "lj":
        return lj(x, L, pi, pj, pot.eps, pot.sigma, pot.rc)
    F, E, W, _, _ = eam(x, L, pi, pj, pot)
    return F, E, W


def verlet(x, v, L, pot, dt: float, mass: float, steps: int, skin: float, threads: int = 0):
    """Velocity Verlet; returns (x, v, F, hist[steps][3] = (E_pot, KE, W), n_rebuild).

    threads = 0: the serial reference (half lists); threads >= 1: the OpenMP
    full-list variant on that many threads (a CPU baseline, tested against the
    serial one)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[1]
    F = np.zeros((3, n))
    hist = np.zeros((max(steps, 1), 3))
    nreb = np.zeros(1, dtype=np.int32)
    lj_par = np.array([pot.eps, pot.sigma])
    if pot.kind == "lj":
        nk = np.zeros(3, dtype=np.int32)
        x0 = h = np.zeros(3)
        cp = cr = ce = np.zeros(4)
        kind, rcp, rcr = 0, 0.0, 0.0
    else:
        nk, x0, h, cp, cr, ce = _eam_args(pot)
        kind, rcp, rcr = 1, pot.rc_phi, pot.rc_rho
    args = (n, _p(x), _p(v), _p(F), _p(_box(L)), kind, _p(lj_par), _p(nk, _i32),
            _p(x0), _p(h), _p(cp), _p(cr), _p(ce), rcp, rcr, pot.rc, skin, dt, mass,
            steps, _p(hist), _p(nreb, _i32))
    rc = lib().orc_verlet_omp(*args, int(threads)) if threads > 0 else lib().orc_verlet(*args)
    if rc != 0:
        raise ValueError("box shorter than twice the list cutoff")
    return x, v, F, hist[:steps], int(nreb[0])


def lj_vjp(x, L, pi, pj, u, vE, eps=1.0, sigma=1.0, rc=2.5):
    """(g_x[3][n], g_theta[2] = d/d(eps, sigma)) of vE*E + u.F."""
    x = _f64(x)
    u = _f64(u)
    n = x.shape[1]
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    gx = np.zeros((3, n))
    gp = np.zeros(2)
    lib().orc_lj_vjp(n, _p(x), _p(_box(L)), rc, eps, sigma, pi.size, _p(pi, _i32), _p(pj, _i32),
                     _p(u), float(vE), _p(gx), _p(gp))
    return gx, gp


def eam_vjp(x, L, pi, pj, pot, u, vE):
    """(g_x[3][n], g_phi, g_rho, g_emb) of vE*E + u.F (tables' shapes)."""
    x = _f64(x)
    u = _f64(u)
    n = x.shape[1]
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    pj = np.ascontiguousarray(pj, dtype=np.int32)
    nk, x0, h, cp, cr, ce = _eam_args(pot)
    gx = np.zeros((3, n))
    gphi = np.zeros_like(cp)
    grho = np.zeros_like(cr)
    gemb = np.zeros_like(ce)
    lib().orc_eam_vjp(n, _p(x), _p(_box(L)), _p(nk, _i32), _p(x0), _p(h), _p(cp), _p(cr), _p(ce),
                      pot.rc_phi, pot.rc_rho, pi.size, _p(pi, _i32), _p(pj, _i32), _p(u), float(vE),
                      _p(gx), _p(gphi), _p(grho), _p(gemb))
    return gx, gphi, grho, gemb


def vjp(x, L, pot, u, vE, skin: float = 0.0):
    """Adjoint of one periodic system; LJ -> (g_x, g[2]); EAM -> (g_x, g_phi, g_rho, g_emb)."""
    x = wrap(x, L)
    pi, pj = half_pairs(x, L, pot.rc + skin)
    if pot.kind == "lj":
        return lj_vjp(x, L, pi, pj, u, vE, pot.eps, pot.sigma, pot.rc)
    return eam_vjp(x, L, pi, pj, pot, u, vE)


def max_threads() -> int:
    """Threads the OpenMP variant uses by default (OMP_NUM_THREADS or the cores)."""
    return int(lib().orc_max_threads())
