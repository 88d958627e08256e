"""The wave-scheduled half list (MD_LIST_WAVES) through the C ABI against the
oracle: the brick colouring exactly (integer work), forces, energies, virials
and trajectories to the FP64 (1e-12) and mixed (1e-5) bounds."""
import numpy as np
import pytest

import oracle
from oracle import waves as OW
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem
from test_gpu_parity import FP64_TOL, MIXED_TOL, lj_cases, materialise, rel

pytestmark = pytest.mark.gpu

# (bx, by, bz) cells per task; (1, 1, 1) are the paper's cell tasks; a 64-candidate
# LDS stage sends part of every halo through the global-memory path
SHAPES = [((1, 1, 1), 0), ((2, 2, 3), 0), ((4, 3, 2), 0), ((2, 2, 2), 64)]
NAMES = ["box_2x3x5", "fcc2048_thermal", "ragged_6859"]


def shaped(w, shape, cap):
    s = MDSystem.from_workload(w)
    B.md_set_tuning(s.ctx, 3, shape[0] | shape[1] << 8 | shape[2] << 16)
    if cap:
        B.md_set_tuning(s.ctx, 0, cap)
    return s


def expected_colours(w, shape):
    cols, n = [], 0
    for r in range(w.n_replicas):
        nc = oracle.grid(w.boxes[r], w.pot.rc + w.skin)
        bd = [min(shape[d], nc[d]) for d in range(3)]
        c, k = OW.brick_colours(nc, bd)
        cols += c
        n = max(n, k)
    return np.array(cols, dtype=np.int32), n


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("shape,cap", SHAPES)
def test_schedule_equals_the_oracle(name, shape, cap):
    w = materialise(lj_cases()[name])
    s = shaped(w, shape, cap)
    s.build(B.MD_LIST_WAVES)
    col, n = B.md_get_waves(s.ctx)
    exp, ne = expected_colours(w, shape)
    assert n == ne and B.md_query(s.ctx, 11) == n
    assert np.array_equal(col, exp)


def test_cell_tasks_on_a_4_cell_grid_take_64_waves():
    w = materialise(lj_cases()["fcc2048_thermal"])          # 4 x 4 x 4 cells
    s = shaped(w, (1, 1, 1), 0)
    s.build(B.MD_LIST_WAVES)
    assert B.md_get_waves(s.ctx)[1] == 64


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("shape,cap", SHAPES)
def test_forces_energy_virial_fp64(name, shape, cap):
    w = materialise(lj_cases()[name])
    L = w.boxes[0]
    s = shaped(w, shape, cap)
    F, E, Wv = s.forces(B.MD_FP64, B.MD_LIST_WAVES)
    Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= FP64_TOL
    assert E.item() == pytest.approx(Eo, rel=FP64_TOL, abs=1e-12)
    assert Wv.item() == pytest.approx(Wo, rel=FP64_TOL, abs=1e-12)


@pytest.mark.parametrize("shape,cap", [((4, 3, 2), 0), ((1, 1, 1), 0)])
def test_forces_mixed(shape, cap):
    w = materialise(lj_cases()["fcc2048_thermal"])
    L = w.boxes[0]
    s = shaped(w, shape, cap)
    F, E, _ = s.forces(B.MD_MIXED, B.MD_LIST_WAVES)
    Fo, Eo, _ = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= MIXED_TOL
    assert E.item() == pytest.approx(Eo, rel=1e-6)


def test_replica_batch_forces_and_energies():
    w = W.replica_batch("lj", n_replicas=6, nmin=200, nmax=1200)
    s = MDSystem.from_workload(w)
    F, E, Wv = s.forces(B.MD_FP64, B.MD_LIST_WAVES)
    Fg = F.cpu().numpy()
    for r in range(w.n_replicas):
        lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
        L = w.boxes[r]
        Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos[:, lo:hi], L), L, w.pot, skin=w.skin)
        assert rel(Fg[:, lo:hi], Fo) <= 1e-11
        assert E[r].item() == pytest.approx(Eo, rel=1e-12)
        assert Wv[r].item() == pytest.approx(Wo, rel=1e-10, abs=1e-10)


@pytest.mark.parametrize("shape", [(4, 3, 2), (1, 1, 1)])
def test_verlet_matches_the_oracle(shape):
    w = W.lj_small()
    L = w.boxes[0]
    s = shaped(w, shape, 0)
    F, hist, nreb = s.run(100, w.dt, w.mass, B.MD_FP64, B.MD_LIST_WAVES)
    xo, vo, Fo, ho, nrebo = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 100, w.skin)
    assert np.allclose(hist.cpu().numpy(), ho, rtol=1e-9, atol=1e-9)
    d = s.pos.cpu().numpy() - xo
    d -= L[:, None] * np.round(d / L[:, None])
    assert np.max(np.abs(d)) < 1e-8
    assert rel(F.cpu().numpy(), Fo) < 1e-8
    assert nreb == nrebo


def test_verlet_larger_crystal_tracks_the_full_list():
    """Wave and full-list trajectories agree to rounding over 40 steps of a
    2,048-atom thermal crystal (the full list is checked against the oracle
    elsewhere)."""
    w = materialise(lj_cases()["fcc2048_thermal"])
    sa = MDSystem.from_workload(w)
    Fa, ha, na = sa.run(40, w.dt, w.mass, B.MD_FP64, B.MD_LIST_FULL)
    w = materialise(lj_cases()["fcc2048_thermal"])
    sb = MDSystem.from_workload(w)
    Fb, hb, nb = sb.run(40, w.dt, w.mass, B.MD_FP64, B.MD_LIST_WAVES)
    assert na == nb
    assert np.allclose(hb.cpu().numpy(), ha.cpu().numpy(), rtol=1e-10, atol=1e-10)
    assert rel(Fb.cpu().numpy(), Fa.cpu().numpy()) < 1e-9


def test_waves_reject_eam():
    w = W.replica_batch("eam", n_replicas=2, nmin=200, nmax=400)
    s = MDSystem.from_workload(w)
    s.build(B.MD_LIST_WAVES)
    with pytest.raises(B.MDError):
        s.forces(B.MD_FP64, B.MD_LIST_WAVES, rebuild=False)
