"""The threaded CPU baseline (OpenMP over atoms, full lists, each thread
writing only its own atoms) against the serial oracle it stands beside.

The two sum each atom's force in a different order (full list in list order
against the half list's pair order), so trajectories agree to rounding growth,
not bit for bit; rebuild counts and the recorded energies agree.
"""
import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W


def minimg(d, L):
    return d - L[:, None] * np.round(d / L[:, None])


@pytest.mark.parametrize("threads", [1, 4])
def test_lj_small_matches_serial(threads):
    w = W.lj_small()
    L = w.boxes[0]
    xs, vs, Fs, hs, ns = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 100, w.skin)
    xp, vp, Fp, hp, npb = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 100, w.skin, threads=threads)
    assert ns == npb and ns > 0
    assert np.max(np.abs(minimg(xp - xs, L))) < 1e-10
    assert np.max(np.abs(vp - vs)) < 1e-9
    assert np.max(np.abs(Fp - Fs)) < 1e-8
    assert np.allclose(hp, hs, rtol=1e-11, atol=1e-9)


def test_eam_crystal_matches_serial():
    w = W.fs_eam(cells=4, vacancy_frac=0.05, sigma_d=0.08, workload_id=61)
    L = w.boxes[0]
    v = W.maxwell_boltzmann(w.n, 0.05, 1.0, W.rng(61, "velocities"))
    xs, vs, Fs, hs, ns = oracle.verlet(w.pos, v, L, w.pot, w.dt, w.mass, 60, w.skin)
    xp, vp, Fp, hp, npb = oracle.verlet(w.pos, v, L, w.pot, w.dt, w.mass, 60, w.skin, threads=3)
    assert ns == npb
    assert np.max(np.abs(minimg(xp - xs, L))) < 1e-10
    assert np.max(np.abs(Fp - Fs)) < 1e-8
    assert np.allclose(hp, hs, rtol=1e-11, atol=1e-9)


def test_zero_steps_is_the_initial_state():
    """0 steps: wrap, list and F(x0) only (the part the baseline timing subtracts)."""
    w = W.lj_small()
    L = w.boxes[0]
    x, v, F, h, nreb = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 0, w.skin, threads=2)
    Fo, _, _ = oracle.forces(w.pos, L, w.pot, skin=w.skin)
    assert nreb == 0 and np.array_equal(v, w.vel)
    assert np.max(np.abs(F - Fo)) < 1e-10
