"""Parity at the full workload sizes, in the launch configuration the benchmark
uses (default brick shape, workgroup size and LDS stage chosen by the library).

Lists are compared exactly on sampled atoms against the oracle's linked-cell
lists; forces against the oracle's exhaustive per-atom sums (LJ) or its full
evaluation (EAM); a short velocity-Verlet run against the oracle's run.
"""
import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def sample_atoms(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=k, replace=False)).astype(np.int32)


def check_list_sample(s, w, sample):
    L = w.boxes[0]
    x = oracle.wrap(w.pos, L)
    start, nbr = s.neighbor_list()
    os_, on = oracle.neighbor_list(x, L, w.pot.rc + w.skin, full=True)
    for u in sample:
        got = np.sort(nbr[start[u]:start[u + 1]])
        want = np.sort(on[os_[u]:os_[u + 1]])
        assert np.array_equal(got, want), f"atom {u}: neighbour sets differ"
    assert start[-1] == os_[-1], "total list length differs"


def check_lj_forces_sample(s, w, snap, sample):
    L = w.boxes[0]
    Fo, _ = oracle.lj_atoms(snap, L, sample, w.pot.eps, w.pot.sigma, w.pot.rc)
    s.pos.copy_(s.pos.new_tensor(snap))
    F64 = s.forces(B.MD_FP64)[0].cpu().numpy()
    Fmx = s.forces(B.MD_MIXED, rebuild=False)[0].cpu().numpy()
    assert rel(F64[:, sample], Fo) <= FP64_TOL
    err = rel(Fmx[:, sample], Fo)
    print(f"{w.name}: mixed force error {err:.3e} on {sample.size} atoms")
    assert err <= MIXED_TOL


def test_lj_crystal_1048576():
    w = W.lj_bulk()
    s = MDSystem.from_workload(w)
    s.build(B.MD_LIST_FULL)
    check_list_sample(s, w, sample_atoms(w.n, 4096, 1))
    snap = W.thermal_snapshot(w, 0.05)
    check_lj_forces_sample(s, w, snap, sample_atoms(w.n, 2048, 2))


def test_lj_crystal_1048576_verlet_10_steps():
    w = W.lj_bulk()
    L = w.boxes[0]
    s = MDSystem.from_workload(w)
    F, hist, nreb = s.run(10, w.dt, w.mass, B.MD_FP64)
    xo, vo, Fo, ho, nrebo = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 10, w.skin)
    assert np.allclose(hist.cpu().numpy(), ho, rtol=1e-10, atol=1e-8)
    sample = sample_atoms(w.n, 4096, 3)
    d = s.pos.cpu().numpy()[:, sample] - xo[:, sample]
    d -= L[:, None] * np.round(d / L[:, None])
    assert np.max(np.abs(d)) < 1e-10
    assert rel(F.cpu().numpy()[:, sample], Fo[:, sample]) < 1e-9
    assert nreb == nrebo


def test_lj_cluster_and_voided_slab():
    w = W.lj_inhomogeneous()
    s = MDSystem.from_workload(w)
    s.build(B.MD_LIST_FULL)
    check_list_sample(s, w, sample_atoms(w.n, 4096, 4))
    snap = W.thermal_snapshot(w, 0.05)
    check_lj_forces_sample(s, w, snap, sample_atoms(w.n, 2048, 5))


def test_fs_eam_1418342():
    w = W.fs_eam()
    L = w.boxes[0]
    s = MDSystem.from_workload(w)
    F64, E64, W64 = s.forces(B.MD_FP64)
    Fmx, Emx, _ = s.forces(B.MD_MIXED, rebuild=False)
    Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F64.cpu().numpy(), Fo) <= 1e-11
    assert E64.item() == pytest.approx(Eo, rel=1e-12)
    assert W64.item() == pytest.approx(Wo, rel=1e-10)
    err = rel(Fmx.cpu().numpy(), Fo)
    print(f"fs_eam: mixed force error {err:.3e}")
    assert err <= MIXED_TOL
    assert Emx.item() == pytest.approx(Eo, rel=1e-7)


@pytest.mark.parametrize("name", ["lj_cluster_slab", "fs_eam_1418342"])
def test_verlet_10_steps_inhomogeneous_and_eam(name):
    """10 binary64 velocity-Verlet steps of the full cluster + voided slab and
    of the full EAM crystal against the oracle's run: energies of every step,
    sampled positions and forces, rebuild counts."""
    w = W.WORKLOADS[name]()
    L = w.boxes[0]
    s = MDSystem.from_workload(w)
    F, hist, nreb = s.run(10, w.dt, w.mass, B.MD_FP64)
    xo, vo, Fo, ho, nrebo = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 10, w.skin)
    assert np.allclose(hist.cpu().numpy(), ho, rtol=1e-10, atol=1e-8)
    sample = sample_atoms(w.n, 4096, 6)
    d = s.pos.cpu().numpy()[:, sample] - xo[:, sample]
    d -= L[:, None] * np.round(d / L[:, None])
    assert np.max(np.abs(d)) < 1e-10
    v = s.vel.cpu().numpy()[:, sample]
    assert np.max(np.abs(v - vo[:, sample])) < 1e-9
    assert rel(F.cpu().numpy()[:, sample], Fo[:, sample]) < 1e-9
    assert nreb == nrebo
