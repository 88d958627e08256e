"""The two brick schedules of the force and adjoint kernels (md_set_tuning key
7): static cost-balanced ranges and a queue.  A brick's atoms are summed by
their own lanes in list order whichever workgroup takes the brick, so forces
and position gradients are bitwise equal under both; energies and virials are
summed over workgroups and agree to rounding.  The automatic choice follows
the fraction of empty cells."""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem
from test_gpu_parity import FP64_TOL, lj_cases, materialise, rel

pytestmark = pytest.mark.gpu


def voided_box():
    """The 2,048-atom thermal fcc crystal with its upper half (z > L/2) removed:
    half of the cells are empty."""
    w = materialise(lj_cases()["fcc2048_thermal"])
    L = w.boxes[0]
    x = oracle.wrap(w.pos, L)
    keep = x[2] < 0.5 * L[2]
    w.pos = np.ascontiguousarray(x[:, keep])
    w.vel = np.zeros_like(w.pos)
    w.offsets = np.array([0, w.n], dtype=np.int64)
    return w


def system(w, mode):
    s = MDSystem.from_workload(w)
    B.md_set_tuning(s.ctx, 7, mode)
    return s


@pytest.mark.parametrize("name", ["fcc2048_thermal", "ragged_6859", "voided"])
@pytest.mark.parametrize("precision", [B.MD_FP64, B.MD_MIXED])
def test_lj_forces_bitwise_equal_under_both_schedules(name, precision):
    w = voided_box() if name == "voided" else materialise(lj_cases()[name])
    out = []
    for mode in (1, 2):
        s = system(w, mode)
        F, E, Wv = s.forces(precision, B.MD_LIST_FULL)
        assert B.md_query(s.ctx, 14) == mode
        out.append((F.clone(), E.item(), Wv.item()))
    assert torch.equal(out[0][0], out[1][0])
    assert out[1][1] == pytest.approx(out[0][1], rel=1e-13, abs=1e-12)
    assert out[1][2] == pytest.approx(out[0][2], rel=1e-13, abs=1e-12)


def test_queue_schedule_matches_the_oracle():
    w = voided_box()
    L = w.boxes[0]
    s = system(w, 2)
    F, E, Wv = s.forces(B.MD_FP64, B.MD_LIST_FULL)
    Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert rel(F.cpu().numpy(), Fo) <= FP64_TOL
    assert E.item() == pytest.approx(Eo, rel=FP64_TOL)
    assert Wv.item() == pytest.approx(Wo, rel=FP64_TOL)


def test_eam_forces_and_adjoint_bitwise_equal_under_both_schedules():
    w = W.replica_batch("eam", n_replicas=3, nmin=300, nmax=900)
    u = np.random.default_rng(3).normal(size=(3, w.n))
    out = []
    for mode in (1, 2):
        s = system(w, mode)
        F, E, _ = s.forces(B.MD_FP64, B.MD_LIST_FULL)
        g, gp = s.vjp(u, precision=B.MD_FP64)
        out.append((F.clone(), E.clone(), g.clone(), gp.clone()))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.allclose(out[0][1], out[1][1], rtol=1e-13, atol=1e-12)
    assert torch.equal(out[0][2], out[1][2])
    assert torch.allclose(out[0][3], out[1][3], rtol=1e-12, atol=1e-12 * float(out[0][3].abs().max()))


def test_lj_adjoint_bitwise_equal_under_both_schedules():
    w = materialise(lj_cases()["fcc2048_thermal"])
    u = np.random.default_rng(5).normal(size=(3, w.n))
    out = []
    for mode in (1, 2):
        s = system(w, mode)
        g, gp = s.vjp(u, precision=B.MD_FP64)
        out.append((g.clone(), gp.clone()))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.allclose(out[0][1], out[1][1], rtol=1e-12, atol=0)


def test_trajectories_bitwise_equal_under_both_schedules():
    w = voided_box()
    res = []
    for mode in (1, 2):
        s = system(w, mode)
        s.vel = torch.tensor(np.random.default_rng(2).normal(scale=0.5, size=(3, w.n)), dtype=torch.float64,
                             device="cuda")
        F, hist, nreb = s.run(60, 0.002, 1.0, B.MD_FP64, B.MD_LIST_FULL)
        res.append((s.pos.clone(), F.clone(), hist.clone(), nreb))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    assert res[0][3] == res[1][3]
    assert torch.allclose(res[0][2], res[1][2], rtol=1e-12, atol=1e-12)


def test_automatic_choice_follows_the_empty_cells():
    dense = system(materialise(lj_cases()["fcc2048_thermal"]), 0)
    dense.build(B.MD_LIST_FULL)
    assert B.md_query(dense.ctx, 14) == 1
    sparse = system(voided_box(), 0)
    sparse.build(B.MD_LIST_FULL)
    assert B.md_query(sparse.ctx, 14) == 2
    with pytest.raises(B.MDError):
        B.md_set_tuning(sparse.ctx, 7, 3)
