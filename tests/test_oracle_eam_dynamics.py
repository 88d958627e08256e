"""Pins of the oracle's velocity Verlet on the Finnis-Sinclair-type EAM, and of
the reading that makes the EAM workload an fcc crystal that stays one.

The integrator pins repeat, for the many-body potential, what the LJ pins
check: time reversibility, an energy error of second order in dt, and that the
recorded energies and the returned forces are those of the EAM force routine
(itself pinned to closed forms and hand cases) at the integrated positions.

The stability pins check the parameter reading: with c1 = c2 = 0 and c0 for zero
pressure, the fcc lattice at a = 3.3 has C11 - C12 < 0 and turns into another
structure within a few hundred steps; with the workload's c1, c2 it has
C11 - C12 > 0 and a short NVE run keeps its neighbour shells.  C11 - C12 comes
from an independent lattice sum of the analytic functions written here.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W

POT = W.fs_eam_potential()


def minimg(d, L):
    return d - L[:, None] * np.round(d / L[:, None])


def eam_crystal(cells=4, vac=0.05, sd=0.05, T=0.0, seed=0):
    w = W.fs_eam(cells=cells, vacancy_frac=vac, sigma_d=sd, workload_id=60 + seed)
    v = w.vel
    if T > 0:
        v = W.maxwell_boltzmann(w.n, T, 1.0, W.rng(60 + seed, "velocities"))
    return w.pos, v, w.boxes[0]


def test_eam_time_reversibility():
    x0, v0, L = eam_crystal(cells=4, sd=0.08, T=0.05)
    x1, v1, _, _, n1 = oracle.verlet(x0, v0, L, POT, 0.005, 1.0, 100, 0.3)
    x2, v2, _, _, _ = oracle.verlet(x1, -v1, L, POT, 0.005, 1.0, 100, 0.3)
    assert np.max(np.abs(minimg(x2 - oracle.wrap(x0, L), L))) < 1e-9
    assert np.max(np.abs(v2 + v0)) < 1e-9
    assert np.max(np.abs(v1 - v0)) > 1e-2          # the atoms did move and interact


def cluster13_eam(seed=0):
    """A site and its 12 fcc neighbours at a = 3.3 in a large box."""
    nn = np.array([[1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0], [1, 0, 1], [1, 0, -1],
                   [-1, 0, 1], [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]])
    x = np.concatenate([np.zeros((1, 3)), 0.5 * 3.3 * nn]).T + 15.0
    g = np.random.default_rng(seed)
    v = g.normal(0, 0.1, size=x.shape)
    v -= v.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), np.array([30.0, 30.0, 30.0])


def test_eam_energy_error_is_second_order():
    x, v, L = cluster13_eam()
    errs = []
    for dt in (0.008, 0.004):
        steps = int(round(0.8 / dt))
        _, _, _, h, _ = oracle.verlet(x, v, L, POT, dt, 1.0, steps, 0.3)
        e = h[:, 0] + h[:, 1]
        errs.append(np.max(np.abs(e - e[0])))
    ratio = errs[0] / errs[1]
    assert 3.2 < ratio < 4.8, (errs, ratio)


def test_eam_verlet_records_the_eam_routine():
    """Row s of the history is (E_pot, KE, W) after step s: E_pot and W equal the
    EAM routine's at the integrated positions, KE = m/2 sum v^2, and the returned
    forces are the EAM forces there."""
    x0, v0, L = eam_crystal(cells=4, sd=0.08, T=0.05, seed=1)
    for steps in (1, 37):
        x, v, F, h, _ = oracle.verlet(x0, v0, L, POT, 0.005, 1.0, steps, 0.3)
        pi, pj = oracle.half_pairs(x, L, POT.rc + 0.3)
        Fo, Eo, Wo, _, _ = oracle.eam(x, L, pi, pj, POT)
        assert h[-1, 0] == pytest.approx(Eo, rel=1e-12)
        assert h[-1, 2] == pytest.approx(Wo, rel=1e-10, abs=1e-10)
        assert h[-1, 1] == pytest.approx(0.5 * float(np.sum(v * v)), rel=1e-12)
        assert np.max(np.abs(F - Fo)) < 1e-11


# ---------------------------------------------------------------- lattice stability
def lattice_energy(Fm, c0, c1, c2, A=W.FS_A, a=W.FS_LATTICE, c=W.FS_C, d=W.FS_D):
    """E/N of the perfect fcc lattice under the homogeneous deformation Fm, from
    the analytic functions summed over lattice vectors."""
    R = []
    for i, j, k in itertools.product(range(-3, 4), repeat=3):
        for b in ((0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)):
            v = (np.array([i, j, k]) + np.array(b)) * a
            if 0 < np.linalg.norm(v) < 5.5:
                R.append(v)
    r = np.linalg.norm(np.array(R) @ np.asarray(Fm).T, axis=1)
    rho = np.sum(np.where(r < d, (r - d) ** 2, 0.0))
    phi = np.where(r < c, (r - c) ** 2 * (c0 + c1 * r + c2 * r * r), 0.0)
    return -A * math.sqrt(rho) + 0.5 * float(np.sum(phi))


def shear_modulus(pot):
    """C11 - C12 from the lattice sum: E/N(e) = E0 + Omega (C11 - C12) e^2 + O(e^4)
    under diag(1 + e, 1 - e, 1) (volume preserved to first order; the first-order
    term vanishes by cubic symmetry)."""
    an = pot.analytic
    e = 1e-3
    om = W.FS_LATTICE ** 3 / 4
    E0 = lattice_energy(np.eye(3), an["c0"], an["c1"], an["c2"])
    Ep = lattice_energy(np.diag([1 + e, 1 - e, 1]), an["c0"], an["c1"], an["c2"])
    Em = lattice_energy(np.diag([1 - e, 1 + e, 1]), an["c0"], an["c1"], an["c2"])
    return (0.5 * (Ep + Em) - E0) / (om * e * e)


@pytest.mark.parametrize("which", ["workload", "c1=c2=0"])
def test_tetragonal_strain_energy(which):
    pot = POT if which == "workload" else W.fs_eam_potential(c1=0.0, c2=0.0)
    cp = shear_modulus(pot)
    if which == "workload":
        assert cp > 0.2
    else:
        assert cp < -0.4
    # the oracle's energy of a strained 4^3 lattice (box strained with it)
    w = W.fs_eam(cells=4, vacancy_frac=0.0, sigma_d=0.0)
    L0 = w.boxes[0]
    E0 = oracle.forces(w.pos, L0, pot)[1] / w.n
    e = 0.01
    s = np.array([1 + e, 1 - e, 1.0])
    Es = oracle.forces(w.pos * s[:, None], L0 * s, pot)[1] / w.n
    om = W.FS_LATTICE ** 3 / 4
    assert Es - E0 == pytest.approx(om * cp * e * e, rel=0.05)


def mean_neighbours(x, L, cut=3.9):
    start, _ = oracle.neighbor_list(oracle.wrap(x, L), L, cut, full=True)
    return start[-1] / x.shape[1]


def test_eam_crystal_keeps_its_shells_over_500_steps():
    """The workload recipe (5 % vacancies, N(0, 0.05^2) displacements, v = 0) on
    5^3 unit cells: the mean list length within r_list = 3.9 stays within 3 % of
    its start and the total energy is conserved to 1e-5 over 500 steps."""
    w = W.fs_eam(cells=5, workload_id=3)
    L = w.boxes[0]
    n0 = mean_neighbours(w.pos, L)
    x, v, _, h, _ = oracle.verlet(w.pos, w.vel, L, POT, w.dt, w.mass, 500, w.skin)
    n1 = mean_neighbours(x, L)
    assert abs(n1 / n0 - 1) < 0.03, (n0, n1)
    e = h[:, 0] + h[:, 1]
    assert np.max(np.abs(e - e[0])) / abs(e[0]) < 1e-5
    T = 2 * h[:, 1] / (3 * w.n - 3)
    assert 0.005 < T[-1] < 0.03


def test_c1_c2_zero_crystal_transforms():
    """The same run with c1 = c2 = 0: the lattice restructures (the mean list
    length grows by more than 10 %), which is why the workload does not use it."""
    w = W.fs_eam(cells=5, workload_id=3)
    L = w.boxes[0]
    pot = W.fs_eam_potential(c1=0.0, c2=0.0)
    n0 = mean_neighbours(w.pos, L)
    x, _, _, _, _ = oracle.verlet(w.pos, w.vel, L, pot, w.dt, w.mass, 500, w.skin)
    assert mean_neighbours(x, L) > 1.10 * n0
