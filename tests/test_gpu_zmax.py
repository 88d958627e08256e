"""The largest system a context accepts: 2^26 = 67,108,864 atoms (list entries
hold a 26-bit atom index; gathers use 32-bit byte offsets of sorted indices).
An fcc crystal of 256^3 unit cells, thermally displaced, is binned, listed and
its forces computed on both paths; sampled atoms, among them the eight highest
in z (the last cells, so the highest sorted indices), are checked against the
oracle's exhaustive per-atom sums, and a few velocity-Verlet steps run clean.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu

N_MAX = 1 << 26


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def test_largest_context_lj_crystal():
    w = W.lj_fcc(256, workload_id=11, name="lj_fcc_67108864")
    assert w.n == N_MAX
    snap = W.thermal_snapshot(w, 0.05)
    g = np.random.default_rng(5)
    top = np.argsort(snap[2])[-8:]
    sample = np.unique(np.concatenate([g.choice(w.n, 24, replace=False), top])).astype(np.int32)
    print(f"{w.name}: {w.n} atoms, {sample.size} sampled", flush=True)
    s = MDSystem.from_workload(w, pos=snap)
    idx = torch.as_tensor(sample.astype(np.int64), device="cuda")
    F64 = s.forces(B.MD_FP64)[0].index_select(1, idx).cpu().numpy()
    nbar = B.md_query(s.ctx, 10) / w.n
    Fmx = s.forces(B.MD_MIXED, rebuild=False)[0].index_select(1, idx).cpu().numpy()
    assert s.status()[0] == B.MD_OK
    Fo, _ = oracle.lj_atoms(snap, w.boxes[0], sample, w.pot.eps, w.pot.sigma, w.pot.rc)
    e64, emx = rel(F64, Fo), rel(Fmx, Fo)
    print(f"{w.name}: mean list {nbar:.2f}, FP64 error {e64:.2e}, mixed {emx:.2e}", flush=True)
    assert 70.0 < nbar < 85.0
    assert e64 <= 1e-12
    assert emx <= 1e-5
    # a few steps of the integrator at this size: no error, energy conserved
    F, hist, nreb = s.run(4, w.dt, w.mass, B.MD_MIXED)
    h = hist.cpu().numpy()
    etot = h[:, 0] + h[:, 1]
    assert np.all(np.isfinite(h))
    assert abs(etot[-1] - etot[0]) <= 2e-4 * abs(etot[0])      # 2.6e-5 on a 2,048-atom analogue
