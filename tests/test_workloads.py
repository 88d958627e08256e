"""The seeded synthetic inputs: sizes, densities, determinism and structure."""
import math

import numpy as np
import pytest

from paper_1305_4196_amd import workloads as W


def test_seeded_streams_are_deterministic_and_independent():
    a = W.rng(1, "velocities").normal(size=5)
    b = W.rng(1, "velocities").normal(size=5)
    c = W.rng(1, "voids").normal(size=5)
    assert np.array_equal(a, b) and not np.allclose(a, c)


def test_small_lj():
    w = W.lj_small()
    assert w.n == 256 and w.steps == 100
    L = w.boxes[0, 0]
    assert w.n / L ** 3 == pytest.approx(0.8442, rel=1e-12)
    T = w.vel.var(axis=1).sum() / 3
    ke = 0.5 * np.sum(w.vel ** 2)
    assert 2 * ke / (3 * w.n - 3) == pytest.approx(0.72, rel=1e-12)
    assert np.allclose(w.vel.sum(axis=1), 0, atol=1e-12)


def test_bulk_lj_size():
    w = W.lj_bulk()
    assert w.n == 1048576
    assert w.boxes[0, 0] == pytest.approx(107.494, abs=1e-3)
    assert w.pos.min() >= 0 and w.pos.max() < w.boxes[0, 0]


def test_inhomogeneous_lj_structure():
    w = W.lj_inhomogeneous()
    assert 950_000 < w.n < 1_050_000
    assert 580_000 < w.meta["n_cluster"] < 600_000
    assert np.all(w.pos >= 0) and np.all(w.pos < 160.0)
    # the cluster sits in vacuum: no atom in the gaps between cluster and slab
    z = w.pos[2]
    r = np.sqrt(np.sum((w.pos - 80.0) ** 2, axis=0))
    gap = (z > 12.0) & (z < 148.0) & (r > 55.5)
    assert not np.any(gap)


def test_fs_eam_structure():
    w = W.fs_eam()
    assert w.n == 1_492_992 - 74_650 == 1_418_342
    assert w.boxes[0, 0] == pytest.approx(237.6)
    assert np.all(w.vel == 0)


def test_fs_eam_potential_tables():
    p = W.fs_eam_potential()
    for sp in (p.phi, p.rho, p.embed):
        assert sp.coef.shape == (1999, 4)
    assert p.rc == 3.6 and p.rc_phi == 3.25 and p.rc_rho == 3.6
    assert p.analytic["rho_max"] == pytest.approx(2 * W.fs_rho0())


@pytest.mark.parametrize("kind", ["lj", "eam"])
def test_replica_batch(kind):
    w = W.replica_batch(kind, n_replicas=24)
    sizes = np.diff(w.offsets)
    assert np.all((sizes >= 200) & (sizes <= 4000))
    assert w.offsets[-1] == w.n
    rl = w.pot.rc + w.skin
    assert np.all(w.boxes >= 2 * rl)
    for r in range(w.n_replicas):
        x = w.pos[:, w.offsets[r]:w.offsets[r + 1]]
        assert np.all(x >= 0) and np.all(x < w.boxes[r][:, None])
    if kind == "lj":
        dens = sizes / np.prod(w.boxes, axis=1)
        assert np.allclose(dens, 0.8442, rtol=1e-9)
