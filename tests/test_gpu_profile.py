"""Event timing of md_verlet_step (md_profile, md_profile_detail) through the C ABI.

The library records HIP events around the step loop, its setup and every force
and list launch; the counts must match the call and the times must be
positive.  The calls run on torch's current stream, which here is the default
(null) stream, and md_profile(0) synchronises it itself.
"""
import numpy as np
import pytest
import torch

from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("every", [1, 7])
def test_step_loop_timing_counts(every):
    w = W.lj_fcc(8)
    s = MDSystem.from_workload(w)
    F = torch.empty_like(s.pos)
    n = 30
    hist = torch.zeros(((n + every - 1) // every, 3), dtype=torch.float64, device="cuda")
    B.md_build_cells(s.ctx, s.pos, s.boxes, w.pot.rc, w.skin)
    B.md_profile(s.ctx, True)
    B.md_verlet_step(s.ctx, s.dpot, B.MD_MIXED, B.MD_LIST_FULL, s.pos, s.vel, F, w.dt, w.mass, n, hist, None,
                     hist_every=every)
    fms, fn, lms, ln = B.md_profile(s.ctx, False)          # no torch synchronisation before it
    d = B.md_profile_detail(s.ctx)
    assert B.md_get_status(s.ctx)[0] == B.MD_OK
    recorded = len([k for k in range(1, n + 1) if k % every == 0 or k == n])
    assert d["loop_steps"] == n
    assert d["force_energy_n"] == recorded and d["force_plain_n"] == n - recorded
    assert fn == n + 1                                   # F(x0) and one per step
    assert ln == n                                       # one (possibly empty) list launch per step
    assert d["loop_ms"] > 0 and d["setup_ms"] > 0 and d["force_setup_ms"] > 0
    assert d["force_plain_ms"] + d["force_energy_ms"] + d["force_setup_ms"] == pytest.approx(fms, rel=1e-9)
    assert d["force_plain_ms"] + d["force_energy_ms"] < d["loop_ms"]
    # a second profiled call reports only itself
    B.md_profile(s.ctx, True)
    B.md_verlet_step(s.ctx, s.dpot, B.MD_MIXED, B.MD_LIST_FULL, s.pos, s.vel, F, w.dt, w.mass, 5, None, None)
    B.md_profile(s.ctx, False)
    assert B.md_profile_detail(s.ctx)["loop_steps"] == 5


@pytest.mark.gpu
def test_loop_only_timing_records_no_launch_pairs():
    w = W.lj_fcc(8)
    s = MDSystem.from_workload(w)
    F = torch.empty_like(s.pos)
    B.md_build_cells(s.ctx, s.pos, s.boxes, w.pot.rc, w.skin)
    B.md_profile(s.ctx, True, launches=False)
    B.md_verlet_step(s.ctx, s.dpot, B.MD_MIXED, B.MD_LIST_FULL, s.pos, s.vel, F, w.dt, w.mass, 12, None, None)
    fms, fn, lms, ln = B.md_profile(s.ctx, False)
    d = B.md_profile_detail(s.ctx)
    assert B.md_get_status(s.ctx)[0] == B.MD_OK
    assert d["loop_steps"] == 12 and d["loop_ms"] > 0 and d["setup_ms"] > 0
    assert fn == 0 and ln == 0 and fms == 0.0 and lms == 0.0
    assert d["force_plain_n"] == 0 and d["force_energy_n"] == 0 and d["force_setup_ms"] == 0.0
