"""Seeded synthetic inputs for the short-range MD hot path.

This module only *produces inputs*: lattice sites, thermal velocities, defects,
replica batches and the tabulated potential parameters.  It holds none of the
arithmetic of the method itself (binning, neighbor lists, forces, integration,
adjoints); both the HIP path and the CPU oracle consume what it returns.

The paper benchmarks on copper configurations that are not available
(Sec. III: bulk block, spherical nanoparticle, porous sintered system), so the
workloads here are synthetic stand-ins with the same structure:

* ``lj_fcc``       homogeneous Lennard-Jones fcc crystal (bulk stand-in);
* ``lj_inhomogeneous``  fcc cluster in vacuum plus a voided fcc slab
                   (nanoparticle and porous-system stand-in);
* ``fs_eam``       Finnis-Sinclair-type EAM crystal with vacancies and
                   thermal displacements (the many-body potential family of
                   Sec. II.C);
* ``replica_batch`` uneven-size replicas for batched differentiation (the
                   replica-carrying functor of Sec. II.C).

Seeds: one ``numpy.random.SeedSequence(13054196)`` child per
(workload, purpose), PCG64 generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

SEED = 13054196
PURPOSES = {
    "velocities": 0,
    "voids": 1,
    "vacancies": 2,
    "displacements": 3,
    "sizes": 4,
    "offsets": 5,
    "snapshots": 6,
    "params": 7,
    "cotangents": 8,
    "misc": 9,
}

LJ_DENSITY = 0.8442
LJ_RC = 2.5
SKIN = 0.3
N_KNOTS = 2000

# Finnis-Sinclair-type EAM of the many-body workload.
FS_C = 3.25      # phi cutoff
FS_D = 3.6       # rho cutoff
FS_A = 1.0
FS_LATTICE = 3.3
# Pair-polynomial coefficients.  With c1 = c2 = 0 the fcc lattice at a = 3.3 has
# C11 - C12 < 0 and turns into a bcc-like structure within a few hundred steps
# (the Bain path has no barrier); c1, c2 below make it a stable minimum with
# positive elastic constants and phonon frequencies, c0 then follows from zero
# pressure.
FS_C1 = -3.75
FS_C2 = 0.7


def rng(workload: int, purpose: str) -> np.random.Generator:
    """Independent PCG64 stream for one (workload, purpose)."""
    ss = np.random.SeedSequence(SEED, spawn_key=(int(workload), PURPOSES[purpose]))
    return np.random.Generator(np.random.PCG64(ss))


# --------------------------------------------------------------------------
# lattice and velocity generators
# --------------------------------------------------------------------------
_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def fcc_sites(nx: int, ny: int, nz: int, ax: float, ay: Optional[float] = None,
              az: Optional[float] = None) -> np.ndarray:
    """fcc sites of an nx*ny*nz block of cubic unit cells, SoA (3, 4*nx*ny*nz).

    Order: unit cells with x fastest, then the four basis sites.
    """
    ay = ax if ay is None else ay
    az = ax if az is None else az
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1).astype(np.float64)
    sites = (cells[:, None, :] + _FCC_BASIS[None, :, :]).reshape(-1, 3)
    sites = sites * np.array([ax, ay, az])
    return np.ascontiguousarray(sites.T)


def maxwell_boltzmann(n: int, T: float, mass: float, gen: np.random.Generator) -> np.ndarray:
    """Gaussian N(0, T/m) components, net momentum removed, rescaled to T with 3N-3 dof."""
    v = gen.normal(0.0, math.sqrt(T / mass), size=(3, n))
    v -= v.mean(axis=1, keepdims=True)
    ke2 = mass * float(np.sum(v * v))           # 2 * kinetic energy
    scale = math.sqrt(T * (3 * n - 3) / ke2)
    return np.ascontiguousarray(v * scale)


def wrap_into_box(x: np.ndarray, L: np.ndarray) -> np.ndarray:
    """Input preparation: bring generated sites into [0, L) (numpy mod)."""
    y = np.mod(x, L[:, None])
    y[y >= L[:, None]] = 0.0
    return np.ascontiguousarray(y)


# --------------------------------------------------------------------------
# potentials (parameters handed to both sides)
# --------------------------------------------------------------------------
@dataclass
class Spline:
    """Uniform-knot cubic, power basis per interval: f = a0 + a1 t + a2 t^2 + a3 t^3,
    t = (x - x0)/h - k on interval k; ``coef`` has shape (n_knots - 1, 4)."""
    x0: float
    h: float
    coef: np.ndarray

    @property
    def n_knots(self) -> int:
        return self.coef.shape[0] + 1


@dataclass
class Potential:
    kind: str                       # "lj" or "eam"
    rc: float                       # interaction cutoff (neighbor list uses rc + skin)
    eps: float = 1.0
    sigma: float = 1.0
    phi: Optional[Spline] = None
    rho: Optional[Spline] = None
    embed: Optional[Spline] = None
    rc_phi: float = 0.0
    rc_rho: float = 0.0
    analytic: Dict[str, float] = field(default_factory=dict)


def lj_potential(eps: float = 1.0, sigma: float = 1.0, rc: float = LJ_RC) -> Potential:
    return Potential(kind="lj", rc=rc, eps=eps, sigma=sigma)


def hermite_table(f, fp, x0: float, x1: float, n_knots: int = N_KNOTS,
                  slope0: Optional[float] = None) -> Spline:
    """Cubic Hermite interpolant of (f, f') on n_knots uniform knots in [x0, x1].

    ``slope0`` overrides the slope at the first knot (used where f' is infinite).
    """
    h = (x1 - x0) / (n_knots - 1)
    xk = x0 + h * np.arange(n_knots)
    fk = np.array([f(x) for x in xk], dtype=np.float64)
    mk = np.array([fp(x) for x in xk], dtype=np.float64)
    if slope0 is not None:
        mk[0] = slope0
    f0, f1 = fk[:-1], fk[1:]
    m0, m1 = h * mk[:-1], h * mk[1:]
    coef = np.empty((n_knots - 1, 4))
    coef[:, 0] = f0
    coef[:, 1] = m0
    coef[:, 2] = -3.0 * f0 - 2.0 * m0 + 3.0 * f1 - m1
    coef[:, 3] = 2.0 * f0 + m0 - 2.0 * f1 + m1
    return Spline(x0=float(x0), h=float(h), coef=np.ascontiguousarray(coef))


def fs_shells(a: float = FS_LATTICE):
    """(distance, count) of the first fcc shells used by the FS workload."""
    return [(a / math.sqrt(2.0), 12), (a, 6), (a * math.sqrt(1.5), 24)]


def fs_rho0(a: float = FS_LATTICE, d: float = FS_D) -> float:
    return sum(n * (r - d) ** 2 for r, n in fs_shells(a) if r < d)


def fs_c0_zero_pressure(A: float = FS_A, a: float = FS_LATTICE, c: float = FS_C,
                        d: float = FS_D, c1: float = 0.0, c2: float = 0.0) -> float:
    """c0 that gives the perfect lattice zero virial pressure for given c1, c2.

    Zero pressure means dE/ds = 0 under a uniform scaling r -> s r at s = 1:
    F'(rho0) sum_n n r rho'(r) + 1/2 sum_n n r phi'(r) = 0 over the shells, with
    F'(rho0) = -A / (2 sqrt(rho0)) and rho'(r) = 2 (r - d).  phi'(r) is linear in
    c0 (phi' = 2 (r - c) c0 + terms in c1, c2), which gives c0 directly.
    """
    rho0 = fs_rho0(a, d)
    emb = (2.0 * A / math.sqrt(rho0)) * sum(n * r * (r - d) for r, n in fs_shells(a) if r < d)
    rest = sum(n * r * (2.0 * (r - c) * (c1 * r + c2 * r * r) + (r - c) ** 2 * (c1 + 2.0 * c2 * r))
               for r, n in fs_shells(a) if r < c)
    lin = sum(n * r * 2.0 * (r - c) for r, n in fs_shells(a) if r < c)
    return (emb - rest) / lin


def fs_eam_potential(A: float = FS_A, c0: Optional[float] = None, c1: float = FS_C1,
                     c2: float = FS_C2, c: float = FS_C, d: float = FS_D,
                     n_knots: int = N_KNOTS, rho_max: Optional[float] = None) -> Potential:
    """phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2) [r<c], rho(r) = (r-d)^2 [r<d],
    F(rho) = -A sqrt(rho); tabulated as uniform cubic Hermite splines."""
    if c0 is None:
        c0 = fs_c0_zero_pressure(A=A, c=c, d=d, c1=c1, c2=c2)
    if rho_max is None:
        rho_max = 2.0 * fs_rho0(d=d)

    def phi(r):
        return (r - c) ** 2 * (c0 + c1 * r + c2 * r * r) if r < c else 0.0

    def dphi(r):
        if r >= c:
            return 0.0
        return 2.0 * (r - c) * (c0 + c1 * r + c2 * r * r) + (r - c) ** 2 * (c1 + 2.0 * c2 * r)

    def rho(r):
        return (r - d) ** 2 if r < d else 0.0

    def drho(r):
        return 2.0 * (r - d) if r < d else 0.0

    def emb(p):
        return -A * math.sqrt(p)

    def demb(p):
        return -A / (2.0 * math.sqrt(p)) if p > 0.0 else 0.0

    hF = rho_max / (n_knots - 1)
    # F'(0) is infinite: the first knot takes the secant slope of the first interval.
    slope0 = (emb(hF) - emb(0.0)) / hF
    return Potential(
        kind="eam", rc=max(c, d),
        phi=hermite_table(phi, dphi, 0.0, c, n_knots),
        rho=hermite_table(rho, drho, 0.0, d, n_knots),
        embed=hermite_table(emb, demb, 0.0, rho_max, n_knots, slope0=slope0),
        rc_phi=c, rc_rho=d,
        analytic=dict(A=A, c0=c0, c1=c1, c2=c2, c=c, d=d, rho_max=rho_max),
    )


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    pos: np.ndarray                 # (3, N) float64, user order
    vel: np.ndarray                 # (3, N) float64
    boxes: np.ndarray               # (R, 3) float64 box edge lengths
    offsets: np.ndarray             # (R + 1,) int64 replica atom offsets
    pot: Potential
    skin: float = SKIN
    dt: float = 0.005
    mass: float = 1.0
    steps: int = 100
    T: float = 0.0
    meta: Dict[str, object] = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])

    @property
    def n_replicas(self) -> int:
        return int(self.boxes.shape[0])


def lj_fcc(cells: int, T: float = 0.72, steps: int = 100, workload_id: int = 0,
           name: Optional[str] = None) -> Workload:
    """Homogeneous LJ fcc crystal of cells^3 unit cells at density 0.8442."""
    a = (4.0 / LJ_DENSITY) ** (1.0 / 3.0)
    L = cells * a
    pos = fcc_sites(cells, cells, cells, a)
    vel = maxwell_boltzmann(pos.shape[1], T, 1.0, rng(workload_id, "velocities"))
    box = np.array([[L, L, L]])
    return Workload(name=name or f"lj_fcc_{cells}", pos=pos, vel=vel, boxes=box,
                    offsets=np.array([0, pos.shape[1]], dtype=np.int64),
                    pot=lj_potential(), steps=steps, T=T, meta=dict(a=a, cells=cells))


def lj_small() -> Workload:
    """256-atom LJ fcc (4^3 cells), T = 0.72, 100 steps."""
    return lj_fcc(4, T=0.72, steps=100, workload_id=0, name="lj_fcc_256")


def lj_bulk(cells: int = 64) -> Workload:
    """LJ fcc 64^3 unit cells = 1,048,576 atoms, T = 0.72, 1000 steps."""
    return lj_fcc(cells, T=0.72, steps=1000, workload_id=1, name=f"lj_fcc_{4 * cells ** 3}")


def lj_inhomogeneous(L: float = 160.0, R: float = 55.0, n_voids: int = 40,
                     slab_cells: int = 12, T: float = 0.5) -> Workload:
    """fcc cluster (radius R, centred in the box) in vacuum plus an fcc slab
    ``slab_cells`` unit cells thick around z = 0 (mod L) with random spherical voids."""
    a = (4.0 / LJ_DENSITY) ** (1.0 / 3.0)
    centre = np.array([L / 2, L / 2, L / 2])
    # cluster: lattice origin at the centre
    m = int(math.ceil(R / a)) + 1
    blk = fcc_sites(2 * m, 2 * m, 2 * m, a) - m * a
    r = np.sqrt(np.sum(blk * blk, axis=0))
    cluster = blk[:, r < R] + centre[:, None]
    # slab: x-y period commensurate with L
    nxy = int(round(L / a))
    axy = L / nxy
    slab = fcc_sites(nxy, nxy, slab_cells, axy, axy, a)
    slab[2] -= 0.5 * slab_cells * a
    g = rng(2, "voids")
    half = 0.5 * slab_cells * a
    centres = np.stack([g.uniform(0, L, n_voids), g.uniform(0, L, n_voids),
                        g.uniform(-half, half, n_voids)])
    radii = g.uniform(4.0, 8.0, n_voids)
    keep = np.ones(slab.shape[1], dtype=bool)
    for k in range(n_voids):
        d = slab - centres[:, k:k + 1]
        d -= L * np.round(d / L)          # input prep: periodic distance to the void centre
        keep &= np.sum(d * d, axis=0) >= radii[k] ** 2
    slab = slab[:, keep]
    box = np.array([L, L, L])
    pos = wrap_into_box(np.concatenate([cluster, slab], axis=1), box)
    vel = maxwell_boltzmann(pos.shape[1], T, 1.0, rng(2, "velocities"))
    return Workload(name="lj_cluster_slab", pos=pos, vel=vel, boxes=box[None, :],
                    offsets=np.array([0, pos.shape[1]], dtype=np.int64),
                    pot=lj_potential(), steps=1000, T=T,
                    meta=dict(a=a, n_cluster=int(cluster.shape[1]), n_slab=int(slab.shape[1]),
                              voids=np.concatenate([centres, radii[None]], axis=0)))


def fs_eam(cells: int = 72, vacancy_frac: float = 0.05, sigma_d: float = 0.05,
           steps: int = 500, workload_id: int = 3) -> Workload:
    """FS-EAM fcc crystal (a = 3.3), a fraction of sites vacated, Gaussian displacements."""
    a = FS_LATTICE
    L = cells * a
    sites = fcc_sites(cells, cells, cells, a)
    nsites = sites.shape[1]
    nvac = int(round(vacancy_frac * nsites))
    gv = rng(workload_id, "vacancies")
    gone = gv.choice(nsites, size=nvac, replace=False)
    keep = np.ones(nsites, dtype=bool)
    keep[gone] = False
    pos = sites[:, keep]
    gd = rng(workload_id, "displacements")
    pos = pos + gd.normal(0.0, sigma_d, size=pos.shape)
    box = np.array([L, L, L])
    pos = wrap_into_box(pos, box)
    vel = np.zeros_like(pos)
    return Workload(name=f"fs_eam_{pos.shape[1]}", pos=pos, vel=vel, boxes=box[None, :],
                    offsets=np.array([0, pos.shape[1]], dtype=np.int64),
                    pot=fs_eam_potential(), steps=steps, T=0.0,
                    meta=dict(a=a, cells=cells, n_sites=nsites))


def replica_batch(kind: str = "lj", n_replicas: int = 512, nmin: int = 200, nmax: int = 4000,
                  workload_id: int = 4) -> Workload:
    """Uneven-size replicas, alternating perturbed-fcc and liquid-like snapshots."""
    gs = rng(workload_id, "sizes")
    sizes = gs.integers(nmin, nmax + 1, size=n_replicas)
    gsnap = rng(workload_id, "snapshots")
    pos_list: List[np.ndarray] = []
    boxes = np.zeros((n_replicas, 3))
    for r, n in enumerate(sizes):
        n = int(n)
        if kind == "lj":
            L = (n / LJ_DENSITY) ** (1.0 / 3.0)
            nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
            a = L / nc
            rmin = 0.8
        else:
            nc = int(math.ceil((n / 4.0) ** (1.0 / 3.0)))
            a = FS_LATTICE
            L = nc * a
            rmin = 1.8
        sites = fcc_sites(nc, nc, nc, a)
        drop = gsnap.choice(sites.shape[1], size=sites.shape[1] - n, replace=False)
        keep = np.ones(sites.shape[1], dtype=bool)
        keep[drop] = False
        site = sites[:, keep]
        sd = 0.05 if r % 2 == 0 else 0.15
        x = site + gsnap.normal(0.0, sd, size=site.shape)
        box = np.array([L, L, L])
        if r % 2 == 1:
            x = _resample_close(x, site, box, rmin, sd, gsnap)
        pos_list.append(wrap_into_box(x, box))
        boxes[r] = box
    offsets = np.zeros(n_replicas + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    pos = np.ascontiguousarray(np.concatenate(pos_list, axis=1))
    pot = lj_potential() if kind == "lj" else fs_eam_potential()
    return Workload(name=f"replicas_{kind}_{n_replicas}", pos=pos, vel=np.zeros_like(pos),
                    boxes=boxes, offsets=offsets, pot=pot, steps=1, T=0.0,
                    meta=dict(sizes=sizes))


def _resample_close(x: np.ndarray, base: np.ndarray, box: np.ndarray, rmin: float, sd: float,
                    gen: np.random.Generator, max_rounds: int = 60) -> np.ndarray:
    """Re-draw the displacement (from its site ``base``) of any atom closer than rmin
    to another."""
    from scipy.spatial import cKDTree

    x = x.copy()
    for k in range(max_rounds):
        pts = np.mod(x, box[:, None]).T
        pts[pts >= box] = 0.0
        pairs = cKDTree(pts, boxsize=box).query_pairs(rmin, output_type="ndarray")
        if pairs.size == 0:
            break
        bad = np.unique(pairs.ravel())
        # re-draw with a shrinking spread so that the loop ends after a few rounds
        x[:, bad] = base[:, bad] + gen.normal(0.0, sd * 0.8 ** (k + 1), size=(3, bad.size))
    return x


def perturb_params(pot: Potential, workload_id: int = 4, frac: float = 0.1) -> Potential:
    """Starting point of a fit: parameters scaled by (1 + U[-frac, frac]) (seeded)."""
    g = rng(workload_id, "params")
    if pot.kind == "lj":
        f = 1.0 + g.uniform(-frac, frac, size=2)
        return lj_potential(eps=pot.eps * f[0], sigma=pot.sigma * f[1], rc=pot.rc)
    an = pot.analytic
    f = 1.0 + g.uniform(-frac, frac, size=4)
    return fs_eam_potential(A=an["A"] * f[0], c0=an["c0"] * f[1], c1=an["c1"] * f[2],
                            c2=an["c2"] * f[3], c=an["c"], d=an["d"], rho_max=an["rho_max"])


def random_cotangents(n: int, n_replicas: int, workload_id: int = 9):
    """Seeded cotangents (u on forces, v on energies) for adjoint tests."""
    g = rng(workload_id, "cotangents")
    return (np.ascontiguousarray(g.normal(size=(3, n))),
            np.ascontiguousarray(g.normal(size=n_replicas)))


def thermal_snapshot(w: Workload, sigma_d: float, workload_id: int = 9) -> np.ndarray:
    """Positions displaced by N(0, sigma_d^2) per component (for force-error metrics
    away from the perfect lattice, where every force vanishes)."""
    g = rng(workload_id, "displacements")
    out = w.pos + g.normal(0.0, sigma_d, size=w.pos.shape)
    parts = []
    for r in range(w.n_replicas):
        lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
        parts.append(wrap_into_box(out[:, lo:hi], w.boxes[r]))
    return np.ascontiguousarray(np.concatenate(parts, axis=1))


WORKLOADS = {
    "lj_fcc_256": lj_small,
    "lj_fcc_1048576": lj_bulk,
    "lj_cluster_slab": lj_inhomogeneous,
    "fs_eam_1418342": fs_eam,
    "replicas_lj_512": lambda: replica_batch("lj"),
    "replicas_eam_512": lambda: replica_batch("eam"),
}
