"""Pins of the oracle's hand-derived adjoints.

For cotangents u (on the forces) and vE (on the energy) the oracle returns
g_x = d(vE E + u.F)/dx = -vE F - H u and the parameter gradient.  Pins:
central finite differences (h = 1e-5, FP64), symmetry of the Hessian,
translation invariance, the LJ closed forms dE/deps = E/eps,
sigma dE/dsigma = W, d(u.F)/deps = u.F/eps, the EAM pair-distance histogram,
and an independent re-statement of the energies in plain torch (CPU, FP64)
differentiated twice by torch.autograd.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1305_4196_amd import workloads as W


def lj_state(cells=4, sd=0.07, seed=0):
    w = W.lj_fcc(cells)
    g = np.random.default_rng(seed)
    L = w.boxes[0]
    x = oracle.wrap(w.pos + g.normal(0, sd, size=w.pos.shape), L)
    u = g.normal(size=x.shape)
    return x, L, u


def eam_state(cells=3, seed=0, sd=0.08):
    w = W.fs_eam(cells=cells, vacancy_frac=0.05, sigma_d=sd, workload_id=30 + seed)
    g = np.random.default_rng(seed)
    u = g.normal(size=w.pos.shape)
    return w.pos, w.boxes[0], u, w.pot


def objective(x, L, pot, u, vE, pairs):
    pi, pj = pairs
    if pot.kind == "lj":
        F, E, _ = oracle.lj(x, L, pi, pj, pot.eps, pot.sigma, pot.rc)
    else:
        F, E, _, _, _ = oracle.eam(x, L, pi, pj, pot)
    return vE * E + float(np.sum(u * F))


# ---------------------------------------------------------------- LJ
@pytest.mark.parametrize("vE", [0.0, 0.7])
def test_lj_positions_fd(vE):
    x, L, u = lj_state()
    pot = W.lj_potential()
    pairs = oracle.half_pairs(x, L, 2.8)
    gx, _ = oracle.lj_vjp(x, L, *pairs, u, vE)
    g = np.random.default_rng(1)
    for _ in range(4):
        wdir = g.normal(size=x.shape)
        h = 1e-5
        fd = (objective(x + h * wdir, L, pot, u, vE, pairs)
              - objective(x - h * wdir, L, pot, u, vE, pairs)) / (2 * h)
        assert np.sum(gx * wdir) == pytest.approx(fd, rel=1e-6)


def test_lj_params_fd():
    x, L, u = lj_state(seed=2)
    pairs = oracle.half_pairs(x, L, 2.8)
    vE = 0.3
    _, gp = oracle.lj_vjp(x, L, *pairs, u, vE, eps=1.1, sigma=0.97)
    h = 1e-6
    for k in range(2):
        pp = [1.1, 0.97]
        pm = [1.1, 0.97]
        pp[k] += h
        pm[k] -= h
        fp = objective(x, L, W.lj_potential(*pp), u, vE, pairs)
        fm = objective(x, L, W.lj_potential(*pm), u, vE, pairs)
        assert gp[k] == pytest.approx((fp - fm) / (2 * h), rel=1e-6)


def test_lj_param_closed_forms():
    x, L, u = lj_state(seed=3)
    pi, pj = oracle.half_pairs(x, L, 2.8)
    eps, sig = 1.3, 1.05
    F, E, Wv = oracle.lj(x, L, pi, pj, eps, sig)
    _, gE = oracle.lj_vjp(x, L, pi, pj, np.zeros_like(u), 1.0, eps, sig)
    assert gE[0] == pytest.approx(E / eps, rel=1e-12)
    assert sig * gE[1] == pytest.approx(Wv, rel=1e-12)
    _, gF = oracle.lj_vjp(x, L, pi, pj, u, 0.0, eps, sig)
    assert gF[0] == pytest.approx(np.sum(u * F) / eps, rel=1e-11)


def test_lj_hessian_symmetric_and_translation_invariant():
    x, L, u = lj_state(seed=4)
    pi, pj = oracle.half_pairs(x, L, 2.8)
    w = np.random.default_rng(9).normal(size=x.shape)
    Hu = -oracle.lj_vjp(x, L, pi, pj, u, 0.0)[0]
    Hw = -oracle.lj_vjp(x, L, pi, pj, w, 0.0)[0]
    assert np.sum(w * Hu) == pytest.approx(np.sum(u * Hw), rel=1e-11)
    gx, _ = oracle.lj_vjp(x, L, pi, pj, u, 0.8)
    assert np.max(np.abs(gx.sum(axis=1))) < 1e-10 * np.abs(gx).max() * x.shape[1]


# ---------------------------------------------------------------- torch re-statement
def torch_minimg(d, L):
    hL = 0.5 * L
    return torch.where(d > hL, d - L, torch.where(d < -hL, d + L, d))


def torch_pairs(x, L, cut):
    n = x.shape[1]
    i, j = torch.triu_indices(n, n, 1)
    d = torch_minimg(x[:, i] - x[:, j], L[:, None])
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    m = r2 < cut * cut
    return i[m], j[m], d[:, m], r2[m]


def torch_lj_energy(x, L, eps, sig, rc=2.5):
    i, j, d, r2 = torch_pairs(x, L, rc)
    s6 = (sig * sig / r2) ** 3
    return torch.sum(4 * eps * (s6 * s6 - s6))


def test_lj_against_torch_autograd():
    x, L, u = lj_state(cells=3, sd=0.1, seed=5)
    # 108 atoms, L = 5.04: the minimum image is unique for rc = 2.5 (no list skin)
    L = L * 1.0
    xt = torch.tensor(x, requires_grad=True)
    Lt = torch.tensor(L)
    eps = torch.tensor(1.2, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(0.95, dtype=torch.float64, requires_grad=True)
    E = torch_lj_energy(xt, Lt, eps, sig)
    F = -torch.autograd.grad(E, xt, create_graph=True)[0]
    vE = 0.4
    obj = vE * E + torch.sum(torch.tensor(u) * F)
    gx_t, ge_t, gs_t = torch.autograd.grad(obj, (xt, eps, sig))
    pi, pj = oracle.pairs_brute(x, L, 2.5)
    gx, gp = oracle.lj_vjp(x, L, pi, pj, u, vE, 1.2, 0.95)
    assert np.allclose(gx, gx_t.numpy(), rtol=1e-10, atol=1e-10)
    assert gp[0] == pytest.approx(ge_t.item(), rel=1e-11)
    assert gp[1] == pytest.approx(gs_t.item(), rel=1e-11)


def torch_spline(coef, x0, h, x, extrap=False):
    n = coef.shape[0] + 1
    u = (x - x0) * (1.0 / h)
    k = torch.clamp(torch.floor(u.detach()).long(), 0, n - 2)
    t = u - k.to(u.dtype)
    a = coef[k]
    val = a[:, 0] + a[:, 1] * t + a[:, 2] * t * t + a[:, 3] * t * t * t
    if extrap:
        last = coef[n - 2]
        e = u - (n - 1)
        lin = (last.sum() + (last[1] + 2 * last[2] + 3 * last[3]) * e)
        val = torch.where(u > n - 1, lin, val)
    return val


def torch_eam_energy(x, L, cp, cr, ce, pot):
    i, j, d, r2 = torch_pairs(x, L, pot.rc)
    r = torch.sqrt(r2)
    mphi = r2 < pot.rc_phi ** 2
    mrho = r2 < pot.rc_rho ** 2
    phi = torch_spline(cp, pot.phi.x0, pot.phi.h, r[mphi])
    rho_p = torch_spline(cr, pot.rho.x0, pot.rho.h, r[mrho])
    n = x.shape[1]
    rho = torch.zeros(n, dtype=x.dtype)
    rho = rho.index_add(0, i[mrho], rho_p).index_add(0, j[mrho], rho_p)
    emb = torch_spline(ce, pot.embed.x0, pot.embed.h, rho, extrap=True)
    return emb.sum() + phi.sum()


def test_eam_against_torch_autograd():
    x, L, u, pot = eam_state(cells=3, seed=1, sd=0.1)
    xt = torch.tensor(x, requires_grad=True)
    cp = torch.tensor(pot.phi.coef, requires_grad=True)
    cr = torch.tensor(pot.rho.coef, requires_grad=True)
    ce = torch.tensor(pot.embed.coef, requires_grad=True)
    E = torch_eam_energy(xt, torch.tensor(L), cp, cr, ce, pot)
    F = -torch.autograd.grad(E, xt, create_graph=True)[0]
    vE = -0.6
    obj = vE * E + torch.sum(torch.tensor(u) * F)
    gx_t, gp_t, gr_t, ge_t = torch.autograd.grad(obj, (xt, cp, cr, ce))
    pi, pj = oracle.pairs_brute(x, L, pot.rc)
    gx, gphi, grho, gemb = oracle.eam_vjp(x, L, pi, pj, pot, u, vE)
    scale = np.abs(gx_t.numpy()).max()
    assert np.allclose(gx, gx_t.numpy(), rtol=1e-9, atol=1e-10 * scale)
    for mine, ref in ((gphi, gp_t), (grho, gr_t), (gemb, ge_t)):
        ref = ref.numpy()
        assert np.allclose(mine, ref, rtol=1e-9, atol=1e-10 * max(np.abs(ref).max(), 1e-300))


# ---------------------------------------------------------------- EAM
@pytest.mark.parametrize("vE", [0.0, 1.3])
def test_eam_positions_fd(vE):
    x, L, u, pot = eam_state(seed=2)
    pairs = oracle.half_pairs(x, L, pot.rc)
    gx, _, _, _ = oracle.eam_vjp(x, L, *pairs, pot, u, vE)
    g = np.random.default_rng(3)
    for _ in range(4):
        wdir = g.normal(size=x.shape)
        h = 1e-5
        fd = (objective(x + h * wdir, L, pot, u, vE, pairs)
              - objective(x - h * wdir, L, pot, u, vE, pairs)) / (2 * h)
        assert np.sum(gx * wdir) == pytest.approx(fd, rel=1e-6)


def with_coef(pot, name, k, delta):
    import copy
    p = copy.deepcopy(pot)
    sp = getattr(p, name)
    sp.coef = sp.coef.copy()
    sp.coef.reshape(-1)[k] += delta
    return p


def test_eam_params_fd():
    x, L, u, pot = eam_state(seed=4)
    pairs = oracle.half_pairs(x, L, pot.rc)
    vE = 0.5
    _, gphi, grho, gemb = oracle.eam_vjp(x, L, *pairs, pot, u, vE)
    grads = {"phi": gphi, "rho": grho, "embed": gemb}
    g = np.random.default_rng(5)
    h = 1e-5
    # 32 seeded coefficients among those the configuration touches
    for _ in range(32):
        name = ["phi", "rho", "embed"][int(g.integers(3))]
        gr = grads[name].reshape(-1)
        live = np.nonzero(gr != 0)[0]
        k = int(live[g.integers(live.size)])
        fp = objective(x, L, with_coef(pot, name, k, h), u, vE, pairs)
        fm = objective(x, L, with_coef(pot, name, k, -h), u, vE, pairs)
        assert gr[k] == pytest.approx((fp - fm) / (2 * h), rel=1e-6, abs=1e-9)
    # one random direction in the whole coefficient space
    import copy
    dirs = {n: g.normal(size=getattr(pot, n).coef.shape) for n in grads}
    norm = np.sqrt(sum(np.sum(v * v) for v in dirs.values()))
    dirs = {n: v / norm for n, v in dirs.items()}
    def shifted(s):
        p = copy.deepcopy(pot)
        for n in grads:
            getattr(p, n).coef = getattr(pot, n).coef + s * dirs[n]
        return p
    fd = (objective(x, L, shifted(h), u, vE, pairs) - objective(x, L, shifted(-h), u, vE, pairs)) / (2 * h)
    an = sum(np.sum(grads[n] * dirs[n]) for n in grads)
    assert an == pytest.approx(fd, rel=1e-6)


def test_eam_hessian_symmetric_and_translation_invariant():
    x, L, u, pot = eam_state(seed=6)
    pi, pj = oracle.half_pairs(x, L, pot.rc)
    w = np.random.default_rng(7).normal(size=x.shape)
    Hu = -oracle.eam_vjp(x, L, pi, pj, pot, u, 0.0)[0]
    Hw = -oracle.eam_vjp(x, L, pi, pj, pot, w, 0.0)[0]
    assert np.sum(w * Hu) == pytest.approx(np.sum(u * Hw), rel=1e-10)
    gx = oracle.eam_vjp(x, L, pi, pj, pot, u, 0.9)[0]
    assert np.max(np.abs(gx.sum(axis=1))) < 1e-10 * np.abs(gx).max() * x.shape[1]


def test_eam_phi_gradient_is_distance_histogram():
    """dE/d(phi coefficient k, p) = sum over pairs with r in interval k of t^p."""
    x, L, u, pot = eam_state(seed=8)
    pi, pj = oracle.pairs_brute(x, L, pot.rc)
    _, gphi, _, _ = oracle.eam_vjp(x, L, pi, pj, pot, np.zeros_like(u), 1.0)
    d = x[:, pi] - x[:, pj]
    d -= L[:, None] * np.round(d / L[:, None])
    r = np.sqrt(np.sum(d * d, axis=0))
    r = r[r < pot.rc_phi]
    uu = r / pot.phi.h
    k = np.floor(uu).astype(int)
    t = uu - k
    hist = np.zeros_like(gphi)
    for p in range(4):
        np.add.at(hist[:, p], k, t ** p)
    assert np.allclose(gphi, hist, rtol=1e-10, atol=1e-10)
