"""Pins of the oracle's Finnis-Sinclair-type EAM and of the tabulated functions.

phi(r) = (r-c)^2 (c0 + c1 r + c2 r^2) [r < c], rho(r) = (r-d)^2 [r < d],
F(rho) = -A sqrt(rho), each tabulated on 2,000 uniform knots (cubic Hermite);
the workload takes c1 = -3.75, c2 = 0.7 and c0 from zero pressure.  Pins: the tables against the analytic functions within the Hermite error bound,
perfect-lattice closed forms (rho_0, E/N, zero force, zero virial pressure by
the choice of c0), hand-worked two- and three-atom cases from the analytic
functions, finite differences and Newton's third law.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W

POT = W.fs_eam_potential()
AN = POT.analytic


def phi(r, c0=AN["c0"], c1=AN["c1"], c2=AN["c2"], c=W.FS_C):
    return (r - c) ** 2 * (c0 + c1 * r + c2 * r * r) if r < c else 0.0


def dphi(r, c0=AN["c0"], c1=AN["c1"], c2=AN["c2"], c=W.FS_C):
    if r >= c:
        return 0.0
    return 2 * (r - c) * (c0 + c1 * r + c2 * r * r) + (r - c) ** 2 * (c1 + 2 * c2 * r)


def rho(r, d=W.FS_D):
    return (r - d) ** 2 if r < d else 0.0


def drho(r, d=W.FS_D):
    return 2 * (r - d) if r < d else 0.0


def emb(p, A=W.FS_A):
    return -A * math.sqrt(p)


def demb(p, A=W.FS_A):
    return -A / (2 * math.sqrt(p))


def emb_bound(p):
    """Hermite interpolation bound of the embedding table at rho = p:
    h^4/384 max|F''''| over the interval, F'''' = -(15/16) A rho^(-7/2)."""
    h = POT.embed.h
    lo = max(p - h, h)
    return h ** 4 / 384 * (15 / 16) * lo ** -3.5


def emb_slope_bound(p):
    """Derivative error of the cubic Hermite interpolant, h^3/24 max|F''''|."""
    h = POT.embed.h
    lo = max(p - h, h)
    return h ** 3 / 24 * (15 / 16) * lo ** -3.5


# phi is a quartic with leading coefficient c2, so its fourth derivative is 24 c2 everywhere
PHI_BOUND = POT.phi.h ** 4 / 384 * 24 * abs(AN["c2"])
PHI_SLOPE_BOUND = POT.phi.h ** 3 / 24 * 24 * abs(AN["c2"])


def test_quadratic_tables_are_exact():
    """Cubic Hermite reproduces a quadratic exactly: rho always, phi when c1 = c2 = 0."""
    r = np.linspace(0.5, 3.5999, 4001)
    out = oracle.spline_eval(POT.rho, r)
    assert np.max(np.abs(out[0] - (r - 3.6) ** 2)) < 1e-12
    assert np.max(np.abs(out[1] - 2 * (r - 3.6))) < 1e-10
    assert np.max(np.abs(out[2] - 2.0)) < 1e-6
    quad = W.fs_eam_potential(c1=0.0, c2=0.0)
    r = np.linspace(0.5, 3.2499, 4001)
    out = oracle.spline_eval(quad.phi, r)
    assert np.max(np.abs(out[0] - quad.analytic["c0"] * (r - 3.25) ** 2)) < 1e-12


def test_default_phi_within_hermite_bound():
    r = np.linspace(0.5, 3.2499, 4001)
    out = oracle.spline_eval(POT.phi, r)
    exact = np.array([phi(v) for v in r])
    slope = np.array([dphi(v) for v in r])
    assert np.max(np.abs(out[0] - exact)) <= PHI_BOUND * 1.01 + 1e-13
    assert np.max(np.abs(out[1] - slope)) <= PHI_SLOPE_BOUND * 1.01 + 1e-11


def test_embedding_table_within_hermite_bound():
    p = np.linspace(5.0, AN["rho_max"] * 0.999, 3001)
    out = oracle.spline_eval(POT.embed, p, extrap=True)
    h = POT.embed.h
    # |f - p3| <= h^4/384 max|f''''|,  f'''' = -(15/16) A rho^(-7/2)
    bound = h ** 4 / 384 * (15 / 16) * 5.0 ** -3.5
    assert np.max(np.abs(out[0] + np.sqrt(p))) <= bound * 1.01 + 1e-15
    # derivative error is O(h^3)
    assert np.max(np.abs(out[1] + 0.5 / np.sqrt(p))) < 10 * h ** 3


def test_quartic_phi_within_bound():
    pot = W.fs_eam_potential(c1=0.05, c2=-0.02)
    r = np.linspace(1.0, 3.2499, 2001)
    out = oracle.spline_eval(pot.phi, r)
    exact = (r - 3.25) ** 2 * (pot.analytic["c0"] + 0.05 * r - 0.02 * r * r)
    bound = pot.phi.h ** 4 / 384 * 24 * 0.02
    assert np.max(np.abs(out[0] - exact)) <= bound * 1.01 + 1e-14


def test_embedding_linear_continuation():
    rm = AN["rho_max"]
    at = oracle.spline_eval(POT.embed, [rm], extrap=True)
    beyond = oracle.spline_eval(POT.embed, [rm + 3.0], extrap=True)
    assert beyond[0, 0] == pytest.approx(at[0, 0] + 3.0 * at[1, 0], rel=1e-12)
    assert beyond[1, 0] == pytest.approx(at[1, 0], rel=1e-12)
    assert beyond[2, 0] == 0.0


def test_c0_gives_zero_pressure():
    # c1 = c2 = 0: c0 = A [sum n r (r - d) / sqrt(rho0)] / [sum n r (r - c)] over the shells
    assert W.fs_c0_zero_pressure() == pytest.approx(0.3627, abs=1e-4)
    assert W.fs_rho0() == pytest.approx(19.790, abs=1e-3)
    # the workload's (c1, c2) = (-3.75, 0.7) give c0 = 5.0802; that this c0 makes the
    # virial vanish is checked on the oracle's perfect lattice below
    assert AN["c1"] == -3.75 and AN["c2"] == 0.7
    assert AN["c0"] == pytest.approx(5.0802, abs=1e-4)


def test_perfect_lattice_closed_forms():
    w = W.fs_eam(cells=6, vacancy_frac=0.0, sigma_d=0.0)
    L = w.boxes[0]
    x = oracle.wrap(w.pos, L)
    pi, pj = oracle.half_pairs(x, L, 3.9)
    F, E, Wv, rh, Fp = oracle.eam(x, L, pi, pj, POT)
    r1, r2 = 3.3 / math.sqrt(2), 3.3
    rho0 = 12 * rho(r1) + 6 * rho(r2)
    assert np.allclose(rh, rho0, rtol=1e-13)
    e_cf = emb(rho0) + 6 * phi(r1)
    assert E / w.n == pytest.approx(e_cf, rel=1e-10)
    assert np.max(np.abs(F)) < 1e-11
    # c0 was chosen so that the virial vanishes at this lattice constant
    assert abs(Wv / w.n) < 1e-8


def test_dimer_hand_case():
    r = 2.61
    x = np.array([[0.0, r], [4.0, 4.0], [4.0, 4.0]])
    L = np.array([20.0, 20.0, 20.0])
    F, E, Wv, rh, Fp = oracle.eam(x, L, [0], [1], POT)
    e_cf = 2 * emb(rho(r)) + phi(r)
    assert E == pytest.approx(e_cf, abs=2 * emb_bound(rho(r)) + PHI_BOUND + 1e-13)
    g = dphi(r) + 2 * demb(rho(r)) * drho(r)
    tol = 2 * emb_slope_bound(rho(r)) * abs(drho(r)) + PHI_SLOPE_BOUND + 1e-12
    # d = x0 - x1 = -r e_x; F_0 = -g d/r = g e_x
    assert F[0, 0] == pytest.approx(g, abs=tol)
    assert F[0, 1] == pytest.approx(-g, abs=tol)
    assert Wv == pytest.approx(-g * r, abs=tol * r)


def test_trimer_hand_case():
    """Atoms 0-1 at 2.4 and 1-2 at 3.0 on a line; 0-2 at 5.4 is out of range."""
    x = np.array([[0.0, 2.4, 5.4], [1.0, 1.0, 1.0], [1.0, 1.0, 1.0]])
    L = np.array([30.0, 30.0, 30.0])
    pi, pj = oracle.pairs_brute(x, L, 3.6)
    F, E, Wv, rh, Fp = oracle.eam(x, L, pi, pj, POT)
    rh_cf = [rho(2.4), rho(2.4) + rho(3.0), rho(3.0)]
    assert np.allclose(rh, rh_cf, rtol=1e-12)
    e_cf = sum(emb(p) for p in rh_cf) + phi(2.4) + phi(3.0)
    assert E == pytest.approx(e_cf, abs=sum(2 * emb_bound(p) for p in rh_cf) + 2 * PHI_BOUND + 1e-13)
    fp = [demb(p) for p in rh_cf]
    sb = [emb_slope_bound(p) for p in rh_cf]
    g01 = dphi(2.4) + (fp[0] + fp[1]) * drho(2.4)
    g12 = dphi(3.0) + (fp[1] + fp[2]) * drho(3.0)
    t01 = 2 * (sb[0] + sb[1]) * abs(drho(2.4)) + PHI_SLOPE_BOUND + 1e-12
    t12 = 2 * (sb[1] + sb[2]) * abs(drho(3.0)) + PHI_SLOPE_BOUND + 1e-12
    # F_0 = g01 e_x ; F_2 = -g12 e_x ; F_1 = -g01 e_x + g12 e_x
    assert F[0, 0] == pytest.approx(g01, abs=t01)
    assert F[0, 2] == pytest.approx(-g12, abs=t12)
    assert F[0, 1] == pytest.approx(g12 - g01, abs=t01 + t12)


def thermal_eam(cells=4, vac=0.05, sd=0.05, seed=0):
    w = W.fs_eam(cells=cells, vacancy_frac=vac, sigma_d=sd, workload_id=20 + seed)
    return w.pos, w.boxes[0], w


def test_newton_third_law():
    x, L, w = thermal_eam()
    F, _, _ = oracle.forces(x, L, POT)
    assert np.max(np.abs(F.sum(axis=1))) < 1e-11 * x.shape[1]


def test_force_is_minus_gradient():
    x, L, w = thermal_eam(sd=0.08, seed=1)
    F, _, _ = oracle.forces(x, L, POT)
    g = np.random.default_rng(2)
    h = 1e-5
    for _ in range(12):
        i = int(g.integers(x.shape[1]))
        c = int(g.integers(3))
        xp = x.copy(); xp[c, i] += h
        xm = x.copy(); xm[c, i] -= h
        Ep = oracle.forces(xp, L, POT)[1]
        Em = oracle.forces(xm, L, POT)[1]
        assert -(Ep - Em) / (2 * h) == pytest.approx(F[c, i], rel=1e-6, abs=1e-7)


def test_virial_is_volume_derivative():
    x, L, w = thermal_eam(sd=0.05, seed=3)
    _, _, Wv = oracle.forces(x, L, POT)
    h = 1e-6
    Ep = oracle.forces(x * (1 + h), L * (1 + h), POT)[1]
    Em = oracle.forces(x * (1 - h), L * (1 - h), POT)[1]
    assert -(Ep - Em) / (2 * h) == pytest.approx(Wv, rel=1e-5, abs=1e-6)
