"""Pins of the oracle's velocity-Verlet integrator and displacement-triggered rebuild.

Velocity Verlet is time reversible and symplectic with an O(dt^2) energy error;
free flight is exact; the list is rebuilt exactly when the largest
minimum-image displacement since the last build exceeds skin/2.
"""
import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W


def minimg(d, L):
    return d - L[:, None] * np.round(d / L[:, None])


def test_time_reversibility():
    w = W.lj_small()
    L = w.boxes[0]
    x1, v1, F1, h1, _ = oracle.verlet(w.pos, w.vel, L, w.pot, 0.005, 1.0, 100, w.skin)
    x2, v2, F2, h2, _ = oracle.verlet(x1, -v1, L, w.pot, 0.005, 1.0, 100, w.skin)
    x0 = oracle.wrap(w.pos, L)
    assert np.max(np.abs(minimg(x2 - x0, L))) < 1e-9
    assert np.max(np.abs(v2 + w.vel)) < 1e-9


def cluster13(seed=0):
    """13 atoms (a site and its 12 fcc neighbours) in a large box: every pair
    stays inside rc, so the energy is smooth and only the integrator errs."""
    a = 1.55
    nn = np.array([[1, 1, 0], [1, -1, 0], [-1, 1, 0], [-1, -1, 0], [1, 0, 1], [1, 0, -1],
                   [-1, 0, 1], [-1, 0, -1], [0, 1, 1], [0, 1, -1], [0, -1, 1], [0, -1, -1]])
    x = np.concatenate([np.zeros((1, 3)), 0.5 * a * nn]).T + 15.0
    g = np.random.default_rng(seed)
    v = g.normal(0, 0.2, size=x.shape)
    v -= v.mean(axis=1, keepdims=True)
    return np.ascontiguousarray(x), np.ascontiguousarray(v), np.array([30.0, 30.0, 30.0])


def test_energy_error_is_second_order():
    x, v, L = cluster13()
    pot = W.lj_potential()
    errs = []
    for dt in (0.004, 0.002):
        steps = int(round(0.4 / dt))
        _, _, _, h, _ = oracle.verlet(x, v, L, pot, dt, 1.0, steps, 0.3)
        e = h[:, 0] + h[:, 1]
        errs.append(np.max(np.abs(e - e[0])))
    ratio = errs[0] / errs[1]
    assert 3.2 < ratio < 4.8, (errs, ratio)


def test_free_flight_and_rebuild_count():
    L = np.array([20.0, 20.0, 20.0])
    x = np.array([[1.0, 10.0], [1.0, 10.0], [19.9, 1.0]])
    v = np.array([[1.1, 0.0], [0.0, -0.5], [0.3, 0.0]])
    pot = W.lj_potential()
    dt, steps = 0.005, 100
    x1, v1, F1, h, nreb = oracle.verlet(x, v, L, pot, dt, 1.0, steps, 0.3)
    assert np.all(F1 == 0.0) and np.array_equal(v1, v)
    exact = np.mod(x + v * dt * steps, L[:, None])
    assert np.max(np.abs(minimg(x1 - exact, L))) < 1e-12
    # atom 0 moves |v| dt = 0.005*sqrt(1.21+0.09) = 0.0057 per step: more than 0.15
    # after 27 steps, so rebuilds happen at steps 27, 54, 81
    assert nreb == 3


def test_nve_drift_small_system():
    """1,000 steps of the 256-atom LJ system; the unshifted cutoff lets E jump by
    |V(rc)| = 0.0163 per crossing, the bar is set by the oracle itself."""
    w = W.lj_small()
    L = w.boxes[0]
    _, _, _, h, nreb = oracle.verlet(w.pos, w.vel, L, w.pot, 0.005, 1.0, 1000, w.skin)
    e = h[:, 0] + h[:, 1]
    drift = np.max(np.abs(e - e[0])) / abs(e[0])
    assert drift < 5e-3
    assert nreb > 10
    # the temperature stays in the liquid range
    T = 2 * h[:, 1] / (3 * w.n - 3)
    assert 0.3 < T.mean() < 1.2
