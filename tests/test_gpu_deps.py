"""The dependent schedule (MD_LIST_DEPS) through the C ABI against the oracle:
the task graph exactly (integer work; the oracle's backward method over the
same wave order), forces, energies, virials and trajectories to the FP64 (1e-12)
and mixed (1e-5) bounds, and the bounded wait of its persistent launch (forced
from the host with a zero wait limit: every workgroup still leaves normally)."""
import numpy as np
import pytest

import oracle
from oracle import waves as OW
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem
from test_gpu_parity import FP64_TOL, MIXED_TOL, lj_cases, materialise, rel

pytestmark = pytest.mark.gpu

SHAPES = [((1, 1, 1), 0), ((2, 2, 3), 0), ((4, 3, 2), 0), ((2, 2, 2), 64)]
NAMES = ["box_2x3x5", "fcc2048_thermal", "ragged_6859"]


def shaped(w, shape, cap):
    s = MDSystem.from_workload(w)
    B.md_set_tuning(s.ctx, 3, shape[0] | shape[1] << 8 | shape[2] << 16)
    if cap:
        B.md_set_tuning(s.ctx, 0, cap)
    return s


def expected_graph(w, shape):
    """Successor lists of every replica's bricks (global brick numbering)."""
    out, off = [], 0
    for r in range(w.n_replicas):
        nc = oracle.grid(w.boxes[r], w.pot.rc + w.skin)
        bd = [min(shape[d], nc[d]) for d in range(3)]
        succ, order = OW.brick_task_graph(nc, bd)
        out += [sorted(off + s for s in succ[t]) for t in range(len(order))]
        off += len(order)
    return out


def check_status_ok(s):
    code, flags, _ = B.md_get_status(s.ctx)
    assert code == B.MD_OK and flags == 0, (code, flags)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("shape,cap", SHAPES)
def test_task_graph_equals_the_oracle(name, shape, cap):
    w = materialise(lj_cases()[name])
    s = shaped(w, shape, cap)
    s.build(B.MD_LIST_DEPS)
    off, succ = B.md_get_task_graph(s.ctx)
    exp = expected_graph(w, shape)
    assert len(off) == len(exp) + 1
    got = [list(succ[off[t]:off[t + 1]]) for t in range(len(exp))]
    assert got == exp
    assert B.md_query(s.ctx, 12) == len(succ)


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("shape,cap", SHAPES)
def test_forces_energy_virial_fp64(name, shape, cap):
    w = materialise(lj_cases()[name])
    L = w.boxes[0]
    s = shaped(w, shape, cap)
    F, E, Wv = s.forces(B.MD_FP64, B.MD_LIST_DEPS)
    check_status_ok(s)
    Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= FP64_TOL
    assert E.item() == pytest.approx(Eo, rel=FP64_TOL, abs=1e-12)
    assert Wv.item() == pytest.approx(Wo, rel=FP64_TOL, abs=1e-12)


@pytest.mark.parametrize("shape,cap", [((4, 3, 2), 0), ((1, 1, 1), 0)])
def test_forces_mixed(shape, cap):
    w = materialise(lj_cases()["fcc2048_thermal"])
    L = w.boxes[0]
    s = shaped(w, shape, cap)
    F, E, _ = s.forces(B.MD_MIXED, B.MD_LIST_DEPS)
    check_status_ok(s)
    Fo, Eo, _ = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= MIXED_TOL
    assert E.item() == pytest.approx(Eo, rel=1e-6)


def test_repeated_launches_agree():
    """The launch resets its queue and counts: ten evaluations on one list give
    the same forces to rounding (the on-chip partner sums are unordered)."""
    w = materialise(lj_cases()["ragged_6859"])
    s = shaped(w, (2, 2, 2), 0)
    F0, _, _ = s.forces(B.MD_FP64, B.MD_LIST_DEPS)
    for _ in range(10):
        F, _, _ = s.forces(B.MD_FP64, B.MD_LIST_DEPS, rebuild=False)
        assert rel(F.cpu().numpy(), F0.cpu().numpy()) <= 1e-14
    check_status_ok(s)


def test_replica_batch_forces_and_energies():
    w = W.replica_batch("lj", n_replicas=6, nmin=200, nmax=1200)
    s = MDSystem.from_workload(w)
    F, E, Wv = s.forces(B.MD_FP64, B.MD_LIST_DEPS)
    check_status_ok(s)
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
    F, hist, nreb = s.run(100, w.dt, w.mass, B.MD_FP64, B.MD_LIST_DEPS)
    xo, vo, Fo, ho, nrebo = oracle.verlet(w.pos, w.vel, L, w.pot, w.dt, w.mass, 100, w.skin)
    assert np.allclose(hist.cpu().numpy(), ho, rtol=1e-9, atol=1e-9)
    d = s.pos.cpu().numpy() - xo
    d -= L[:, None] * np.round(d / L[:, None])
    assert np.max(np.abs(d)) < 1e-8
    assert rel(F.cpu().numpy(), Fo) < 1e-8
    assert nreb == nrebo


def test_verlet_larger_crystal_tracks_the_full_list():
    w = materialise(lj_cases()["fcc2048_thermal"])
    sa = MDSystem.from_workload(w)
    Fa, ha, na = sa.run(40, w.dt, w.mass, B.MD_FP64, B.MD_LIST_FULL)
    w = materialise(lj_cases()["fcc2048_thermal"])
    sb = MDSystem.from_workload(w)
    Fb, hb, nb = sb.run(40, w.dt, w.mass, B.MD_FP64, B.MD_LIST_DEPS)
    assert na == nb
    assert np.allclose(hb.cpu().numpy(), ha.cpu().numpy(), rtol=1e-10, atol=1e-10)
    assert rel(Fb.cpu().numpy(), Fa.cpu().numpy()) < 1e-9


def test_zero_wait_limit_reports_a_timeout_then_recovers():
    """Cell tasks on a 4 x 4 x 4 grid form one chain of 64 tasks, so every
    workgroup but the first finds its slot empty; with a zero limit they give
    up at once, raise the flag and leave.  With the limit restored the next
    evaluation is exact again."""
    w = materialise(lj_cases()["fcc2048_thermal"])
    L = w.boxes[0]
    s = shaped(w, (1, 1, 1), 0)
    s.build(B.MD_LIST_DEPS)
    B.md_set_tuning(s.ctx, 5, 0)
    s.forces(B.MD_FP64, B.MD_LIST_DEPS, rebuild=False)
    code, flags, _ = B.md_get_status(s.ctx)
    assert code == B.MD_ERR_TIMEOUT and flags & B.FLAG_SCHEDULE
    B.md_set_tuning(s.ctx, 5, 2_000_000)
    F, E, _ = s.forces(B.MD_FP64, B.MD_LIST_DEPS, rebuild=False)
    check_status_ok(s)
    Fo, Eo, _ = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= FP64_TOL
    assert E.item() == pytest.approx(Eo, rel=FP64_TOL)


def test_deps_reject_eam():
    w = W.replica_batch("eam", n_replicas=2, nmin=200, nmax=400)
    s = MDSystem.from_workload(w)
    s.build(B.MD_LIST_DEPS)
    with pytest.raises(B.MDError):
        s.forces(B.MD_FP64, B.MD_LIST_DEPS, rebuild=False)
