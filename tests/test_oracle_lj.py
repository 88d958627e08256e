"""Pins of the oracle's Lennard-Jones forces, energy and virial.

V(r) = 4 eps [(sigma/r)^12 - (sigma/r)^6] for r < rc (unshifted).  The pins are
closed forms evaluated here in 40-digit arithmetic (mpmath), lattice sums over
fcc shell counts, Newton's third law, finite differences of the energy and
the scaling laws of the potential -- none of them re-uses the oracle's code.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W

mp.mp.dps = 40


def dimer(r, L=20.0):
    x = np.array([[0.0, r], [5.0, 5.0], [5.0, 5.0]])   # d = -r exactly
    return x, np.array([L, L, L])


def mp_V(r, eps=1, sig=1):
    r = mp.mpf(r)
    s6 = (mp.mpf(sig) / r) ** 6
    return 4 * eps * (s6 * s6 - s6)


def mp_f(r, eps=1, sig=1):
    """radial force -dV/dr"""
    r = mp.mpf(r)
    return -mp.diff(lambda q: mp_V(q, eps, sig), r)


@pytest.mark.parametrize("r", [0.95, 1.0, 2 ** (1 / 6), 1.5, 2.2, 2.4999])
def test_dimer_closed_form(r):
    x, L = dimer(r)
    F, E, Wv = oracle.lj(x, L, [0], [1])
    assert E == pytest.approx(float(mp_V(r)), rel=1e-14, abs=1e-15)
    fr = float(mp_f(r))
    # force on atom 0 points along d = x0 - x1 = -r e_x, magnitude fr (repulsive > 0)
    assert F[0, 0] == pytest.approx(-fr, rel=1e-13, abs=1e-14)
    assert F[1, 0] == 0 and F[2, 0] == 0
    assert np.array_equal(F[:, 1], -F[:, 0])
    assert Wv == pytest.approx(float(mp_f(r) * r), rel=1e-13, abs=1e-14)


def test_special_values():
    x, L = dimer(2 ** (1 / 6))
    F, E, _ = oracle.lj(x, L, [0], [1])
    assert E == pytest.approx(-1.0, rel=1e-15) and abs(F[0, 0]) < 1e-13
    x, L = dimer(1.0)
    assert oracle.lj(x, L, [0], [1])[1] == 0.0
    x, L = dimer(np.nextafter(2.5, 0))
    F, E, _ = oracle.lj(x, L, [0], [1])
    assert E == pytest.approx(-0.016316891136, rel=1e-9)
    assert abs(F[0, 0]) == pytest.approx(0.0389994774528, rel=1e-9)


def test_cutoff_is_strict():
    x, L = dimer(2.5)
    F, E, Wv = oracle.lj(x, L, [0], [1])
    assert E == 0.0 and np.all(F == 0.0) and Wv == 0.0


def test_fcc_lattice_sums():
    """Perfect fcc at density 0.8442: shells 12, 6, 24, 12 lie inside rc = 2.5."""
    w = W.lj_fcc(5)
    L = w.boxes[0]
    F, E, Wv = oracle.forces(w.pos, L, w.pot, skin=0.3)
    a = mp.cbrt(mp.mpf(4) / mp.mpf("0.8442"))
    r1 = a / mp.sqrt(2)
    shells = [(1, 12), (2, 6), (3, 24), (4, 12)]
    e_cf = sum(n * mp_V(r1 * mp.sqrt(s)) for s, n in shells) / 2
    w_cf = sum(n * mp_f(r1 * mp.sqrt(s)) * r1 * mp.sqrt(s) for s, n in shells) / 2
    assert E / w.n == pytest.approx(float(e_cf), rel=1e-12)
    assert Wv / w.n == pytest.approx(float(w_cf), rel=1e-12)
    assert E / w.n == pytest.approx(-6.77337, abs=5e-6)
    assert np.max(np.abs(F)) < 1e-12


def thermal_lj(cells=4, sd=0.08, seed=0):
    w = W.lj_fcc(cells)
    g = np.random.default_rng(seed)
    x = oracle.wrap(w.pos + g.normal(0, sd, size=w.pos.shape), w.boxes[0])
    return x, w.boxes[0], w


def test_newton_third_law():
    x, L, w = thermal_lj()
    F, _, _ = oracle.forces(x, L, w.pot)
    assert np.max(np.abs(F.sum(axis=1))) < 1e-11 * np.sqrt(np.mean(F * F)) * x.shape[1]


def test_force_is_minus_gradient():
    x, L, w = thermal_lj(sd=0.05, seed=3)
    F, _, _ = oracle.forces(x, L, w.pot)
    g = np.random.default_rng(5)
    h = 1e-5
    for _ in range(12):
        i = int(g.integers(x.shape[1]))
        c = int(g.integers(3))
        xp = x.copy(); xp[c, i] += h
        xm = x.copy(); xm[c, i] -= h
        Ep = oracle.forces(xp, L, w.pot)[1]
        Em = oracle.forces(xm, L, w.pot)[1]
        assert -(Ep - Em) / (2 * h) == pytest.approx(F[c, i], rel=2e-6, abs=2e-6)


def test_virial_is_volume_derivative():
    """W = -3V dE/dV under uniform scaling of positions and box."""
    x, L, w = thermal_lj(sd=0.03, seed=4)
    _, _, Wv = oracle.forces(x, L, w.pot)
    h = 1e-6
    Ep = oracle.forces(x * (1 + h), L * (1 + h), w.pot)[1]
    Em = oracle.forces(x * (1 - h), L * (1 - h), w.pot)[1]
    # E(lambda) with lambda = 1 +- h: dE/dlambda = -W
    assert -(Ep - Em) / (2 * h) == pytest.approx(Wv, rel=1e-6)


def test_scaling_laws():
    """E is linear in eps; lengths scaled by lambda (sigma, rc, box) leave E unchanged."""
    x, L, w = thermal_lj(sd=0.05, seed=6)
    pi, pj = oracle.half_pairs(x, L, 2.8)
    F1, E1, W1 = oracle.lj(x, L, pi, pj, eps=1.0, sigma=1.0, rc=2.5)
    F2, E2, W2 = oracle.lj(x, L, pi, pj, eps=2.5, sigma=1.0, rc=2.5)
    assert E2 == pytest.approx(2.5 * E1, rel=1e-14)
    lam = 1.37
    F3, E3, W3 = oracle.lj(x * lam, L * lam, pi, pj, eps=1.0, sigma=lam, rc=2.5 * lam)
    assert E3 == pytest.approx(E1, rel=1e-12)
    assert np.allclose(F3 * lam, F1, rtol=1e-10, atol=1e-10)
    assert W3 == pytest.approx(W1, rel=1e-12)


def test_per_atom_exhaustive_agrees():
    x, L, w = thermal_lj(sd=0.06, seed=8)
    F, E, _ = oracle.forces(x, L, w.pot)
    atoms = np.arange(0, x.shape[1], 7)
    Fa, ea = oracle.lj_atoms(x, L, atoms)
    assert np.allclose(Fa, F[:, atoms], rtol=1e-12, atol=1e-12)
    allF, alle = oracle.lj_atoms(x, L, np.arange(x.shape[1]))
    assert alle.sum() == pytest.approx(E, rel=1e-13)
