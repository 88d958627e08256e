"""Batched differentiation (replica batches, graph replay) and the autotuner on the GPU."""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import tune
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.fit import BatchedFit
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu


def flat_params(pot):
    if pot.kind == "lj":
        return torch.tensor([pot.eps, pot.sigma], dtype=torch.float64, device="cuda")
    return torch.tensor(np.concatenate([pot.phi.coef.ravel(), pot.rho.coef.ravel(), pot.embed.coef.ravel()]),
                        dtype=torch.float64, device="cuda")


def make_fit(kind, n_replicas, window=-1, tune_fit=False):
    w = W.replica_batch(kind, n_replicas=n_replicas, nmin=200, nmax=1200)
    s = MDSystem.from_workload(w)
    B.md_set_tuning(s.ctx, 8, window)
    F_star, _, _ = s.forces(B.MD_FP64)                      # targets at the reference parameters
    start = W.perturb_params(w.pot)
    fit = BatchedFit(s, F_star, flat_params(start), tune=tune_fit)
    return w, s, start, fit


def oracle_gradient(w, pot, F_star, theta_pot):
    """d/dtheta of sum |F - F*|^2 / (3N), replica by replica with the oracle."""
    n = w.n
    F = np.zeros_like(w.pos)
    parts = []
    for r in range(w.n_replicas):
        lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
        L = w.boxes[r]
        x = oracle.wrap(w.pos[:, lo:hi], L)
        Fr, _, _ = oracle.forces(x, L, theta_pot, skin=w.skin)
        F[:, lo:hi] = Fr
    u = 2.0 * (F - F_star) / (3.0 * n)
    for r in range(w.n_replicas):
        lo, hi = int(w.offsets[r]), int(w.offsets[r + 1])
        L = w.boxes[r]
        x = oracle.wrap(w.pos[:, lo:hi], L)
        res = oracle.vjp(x, L, theta_pot, u[:, lo:hi], 0.0, skin=w.skin)
        parts.append(np.asarray(res[1]) if theta_pot.kind == "lj"
                     else np.concatenate([res[1].ravel(), res[2].ravel(), res[3].ravel()]))
    return np.sum(parts, axis=0)


@pytest.mark.parametrize("kind", ["lj", "eam"])
def test_graph_replays_match_eager(kind):
    w, s, start, fit = make_fit(kind, 16)
    g_eager = fit.gradient_eager().clone()
    F_eager = fit.F.clone()
    fit.capture()
    for rep in range(4):
        # eager work and a synchronisation between replays
        _ = s.forces(B.MD_FP64, rebuild=False)[0].sum().item()
        g = fit.gradient().clone()
        torch.cuda.synchronize()
        assert torch.equal(fit.F, F_eager), f"replay {rep}: forces differ"
        if kind == "lj":
            assert torch.equal(g, g_eager), f"replay {rep}: gradient differs"
        else:   # table histograms use atomics: equal up to summation order
            assert torch.allclose(g, g_eager, rtol=1e-12, atol=1e-14 * float(g_eager.abs().max()))


# (EAM also with its parameter gradient summed without LDS, key 8 = 0)
@pytest.mark.parametrize("kind,window", [("lj", -1), ("eam", -1), ("eam", 0)])
def test_batch_gradient_matches_oracle(kind, window):
    w, s, start, fit = make_fit(kind, 8 if kind == "eam" else 12, window)
    g = fit.gradient().cpu().numpy()
    go = oracle_gradient(w, w.pot, fit.F_star.cpu().numpy(), start)
    assert np.linalg.norm(g - go) <= 1e-10 * np.linalg.norm(go)


def test_batch_gradient_finite_differences_lj():
    w, s, start, fit = make_fit("lj", 12)
    theta0 = fit.params.clone()
    g = fit.gradient().clone().cpu().numpy()
    h = 1e-5
    for k in range(2):
        vals = []
        for sgn in (1.0, -1.0):
            th = theta0.clone()
            th[k] += sgn * h
            fit.set_params(th)
            fit.gradient()
            vals.append(fit.loss())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert fd == pytest.approx(g[k], rel=1e-6, abs=1e-12)
    fit.set_params(theta0)


def test_batch_gradient_finite_differences_eam_direction():
    w, s, start, fit = make_fit("eam", 6)
    theta0 = fit.params.clone()
    g = fit.gradient().clone().cpu().numpy()
    gen = np.random.default_rng(31)
    d = gen.normal(size=g.size)
    d /= np.linalg.norm(d)
    dt = torch.tensor(d, dtype=torch.float64, device="cuda")
    h = 1e-6
    vals = []
    for sgn in (1.0, -1.0):
        fit.set_params(theta0 + sgn * h * dt)
        fit.gradient()
        vals.append(fit.loss())
    fd = (vals[0] - vals[1]) / (2 * h)
    assert fd == pytest.approx(float(g @ d), rel=1e-5, abs=1e-12)
    fit.set_params(theta0)


def test_tuner_picks_a_working_configuration(tmp_path):
    w = W.lj_fcc(8)
    w.pos = np.ascontiguousarray(oracle.wrap(w.pos + np.random.default_rng(3).normal(0, 0.05, w.pos.shape),
                                             w.boxes[0]))
    s = MDSystem.from_workload(w)
    best = tune.tune(s, precision=B.MD_FP64, top=3, reps=1, cache_path=str(tmp_path / "t.json"))
    assert best["threads"] % 64 == 0 and len(best["candidates"]) >= 3
    F, E, Wv = s.forces(B.MD_FP64)
    L = w.boxes[0]
    Fo, Eo, Wo = oracle.forces(oracle.wrap(w.pos, L), L, w.pot, skin=w.skin)
    assert np.linalg.norm(F.cpu().numpy() - Fo) <= 1e-12 * np.linalg.norm(Fo)
    shape = B.md_query(s.ctx, 3)
    assert [shape & 255, (shape >> 8) & 255, (shape >> 16) & 255] == [min(b, 4) for b in best["shape"]]
    # a second call takes the cached entry
    again = tune.tune(s, precision=B.MD_FP64, top=3, reps=1, cache_path=str(tmp_path / "t.json"))
    assert again["shape"] == best["shape"] and again["threads"] == best["threads"]


def test_energies_on_request_leave_the_gradient_unchanged():
    """The forward pass skips the energy sums unless asked; with them the force
    arithmetic is the same, so forces and gradient agree bit for bit and E
    equals a direct evaluation at the same parameters."""
    w, s, start, fit = make_fit("lj", 6)
    g0 = fit.gradient().clone()
    F0 = fit.F.clone()
    fit_e = BatchedFit(s, fit.F_star, fit.params, with_energy=True, tune=False)
    g1 = fit_e.gradient().clone()
    torch.cuda.synchronize()
    assert torch.equal(fit_e.F, F0)
    assert torch.equal(g1, g0)
    F = torch.empty_like(s.pos)
    E = torch.zeros(s.R, dtype=torch.float64, device=s.device)
    B.md_compute_forces(s.ctx, fit_e.dpot, B.MD_FP64, F, E)
    assert torch.equal(fit_e.E, E)


@pytest.mark.parametrize("kind", ["lj", "eam"])
def test_batch_gradient_matches_oracle_at_workload_sizes(kind):
    """64 replicas drawn from the timed batch's size range (200 to 4,000 atoms,
    up to 5 cells per axis for LJ and 8 for EAM), so that the multi-replica
    brick tasks run their 16-bit staged-image path in the forward and adjoint
    kernels; gradient against the oracle's, replica by replica."""
    w = W.replica_batch(kind, n_replicas=64)
    sizes = np.diff(w.offsets)
    assert sizes.max() > 3500 and sizes.min() < 500
    s = MDSystem.from_workload(w)
    F_star, _, _ = s.forces(B.MD_FP64)
    ncell = np.floor(w.boxes / (w.pot.rc + w.skin)).max()
    assert ncell >= (5 if kind == "lj" else 8)
    assert B.md_query(s.ctx, 15) > 0, "no list entries in the 16-bit layout"
    start = W.perturb_params(w.pot)
    fit = BatchedFit(s, F_star, flat_params(start))          # autotuned for forces + adjoint
    assert fit.tuning is not None and fit.tuning["objective"] == "fit"
    g = fit.gradient().cpu().numpy()
    go = oracle_gradient(w, w.pot, F_star.cpu().numpy(), start)
    assert np.linalg.norm(g - go) <= 1e-10 * np.linalg.norm(go)
