"""md_compute_forces_noalloc (the entry point for callers that cannot allocate)
against md_compute_forces, through the C ABI.

Both run the same kernels on the same list and grid, so forces, energies and
virials must agree to the FP64 parity bar (they are expected to agree bit for
bit).  Two calls in a row share the library's static scratch: a large system,
then a smaller one, each checked; a system whose scratch would not fit is
rejected on the host.
"""
import numpy as np
import pytest
import torch

from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel(a, b):
    a = a.cpu().numpy()
    b = b.cpu().numpy()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def thermal_system(w, sd=0.05, seed=0):
    snap = W.thermal_snapshot(w, sd, workload_id=seed)
    return MDSystem(snap, w.boxes, w.offsets, w.pot, w.skin)


def both(s, precision):
    """(reference F, E, W) from md_compute_forces and the same from the no-alloc call."""
    s.build(B.MD_LIST_FULL)
    F0, E0, W0 = s.forces(precision, rebuild=False)
    F1 = torch.full_like(F0, float("nan"))
    E1 = torch.full_like(E0, float("nan"))
    W1 = torch.full_like(W0, float("nan"))
    B.md_compute_forces_noalloc(s.ctx, s.dpot, precision, F1, E1, W1)
    code = B.md_get_status(s.ctx)[0]
    assert code == B.MD_OK, code
    return (F0, E0, W0), (F1, E1, W1)


def check(ref, got):
    for a, b in zip(got, ref):
        assert torch.isfinite(a).all()
        assert rel(a, b) <= TOL, rel(a, b)


@pytest.mark.parametrize("precision", [B.MD_FP64, B.MD_MIXED])
def test_two_calls_lj_then_smaller_eam(precision):
    big = thermal_system(W.lj_fcc(20), seed=11)                       # 32,000 atoms
    small = thermal_system(W.fs_eam(cells=6, workload_id=12), seed=12)  # 821 atoms
    assert small.n < big.n
    ref, got = both(big, precision)
    check(ref, got)
    ref, got = both(small, precision)
    check(ref, got)
    # and the large one again after the small one used the scratch
    ref, got = both(big, precision)
    check(ref, got)


def test_two_calls_replica_batch_energies():
    big = MDSystem.from_workload(W.replica_batch("lj", n_replicas=24))
    small = MDSystem.from_workload(W.replica_batch("eam", n_replicas=6, workload_id=5))
    assert small.n < big.n
    for s in (big, small):
        ref, got = both(s, B.MD_FP64)
        check(ref, got)


def test_forces_only_call():
    s = thermal_system(W.lj_fcc(8), seed=13)
    s.build(B.MD_LIST_FULL)
    F0, _, _ = s.forces(B.MD_FP64, rebuild=False)
    F1 = torch.empty_like(F0)
    B.md_compute_forces_noalloc(s.ctx, s.dpot, B.MD_FP64, F1, None, None)
    assert B.md_get_status(s.ctx)[0] == B.MD_OK
    assert rel(F1, F0) <= TOL


def test_rejects_a_system_beyond_the_scratch():
    s = thermal_system(W.lj_fcc(8), seed=14)
    limit = B.md_query(s.ctx, 16)
    assert limit == 48 << 20
    n = limit // 24 + 1000                       # 24 bytes per atom of sorted forces alone
    L = (n / 0.05) ** (1.0 / 3.0)                # a dilute random gas keeps the list small
    g = np.random.default_rng(15)
    pos = torch.tensor(g.uniform(0.0, L, size=(3, n)), dtype=torch.float64, device="cuda")
    w = W.lj_fcc(2)
    big = MDSystem(pos, np.array([[L, L, L]]), np.array([0, n]), w.pot, w.skin)
    big.build(B.MD_LIST_FULL)
    F = torch.empty_like(pos)
    with pytest.raises(B.MDError) as e:
        B.md_compute_forces_noalloc(big.ctx, big.dpot, B.MD_FP64, F, None, None)
    assert e.value.code == B.MD_ERR_ARG
    assert "scratch" in str(e.value)


def test_rejects_a_half_list():
    s = thermal_system(W.lj_fcc(8), seed=16)
    s.build(B.MD_LIST_HALF)
    F = torch.empty_like(s.pos)
    with pytest.raises(B.MDError) as e:
        B.md_compute_forces_noalloc(s.ctx, s.dpot, B.MD_FP64, F, None, None)
    assert e.value.code == B.MD_ERR_STATE
