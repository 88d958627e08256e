"""Pairs within one rounding of the LJ cutoff, through the C ABI.

The list build and the rebuild test form r2 exactly as the oracle does
((dx*dx + dy*dy) + dz*dz, every operation rounded), so lists are bit-exact.
The force kernels form r2 with fused multiply-adds (one rounding fewer), and
for a brick staged through its cell images they subtract the partner's
already shifted position; their cutoff test can therefore differ from the
oracle's for a pair whose r2 lies within a few roundings of rc^2.  Both
answers are valid results of the method (the cutoff is a modelling choice,
not a quantity known to an ulp); what is pinned here:

  - an exact tie r = rc is outside on both sides (strict test);
  - for pairs of interior atoms, the force kernels decide on the fused r2:
    the GPU forces, energy and virial equal the oracle's with the pair counted
    by that decision (also where the oracle's own decision differs);
  - across a periodic face, the GPU result equals the oracle's with the pair
    counted or not counted;
  - in every case the list holds the pair (it lies well inside rc + skin).
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from paper_1305_4196_amd import binding as B
from paper_1305_4196_amd import workloads as W
from paper_1305_4196_amd.system import MDSystem

pytestmark = pytest.mark.gpu

RC = 2.5
RC2 = RC * RC
L = 14.0


def fused_r2(d):
    """fma(dz, dz, fma(dy, dy, dx*dx)) with each step rounded once."""
    def fma(a, b, c):
        return float(Fraction(a) * Fraction(b) + Fraction(c))
    return fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]))


def s2_r2(d):
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]


def find_pairs():
    """Seeded search for interior pairs within two units in the last place of
    rc^2, one for each combination of the oracle's and the fused decision."""
    g = np.random.default_rng(1)
    xj = np.array([6.0, 6.0, 6.0])
    found = {}
    for _ in range(20000):
        u = g.normal(size=3)
        u /= np.linalg.norm(u)
        for k in range(-6, 7):
            xi = xj + RC * u * (1 + k * 2.0 ** -52)
            d = xi - xj
            s, f = s2_r2(d), fused_r2(d)
            if abs(s - RC2) > 2 * np.spacing(RC2):
                continue
            key = (bool(s < RC2), bool(f < RC2))
            found.setdefault(key, xi)
        if len(found) == 4:
            break
    assert len(found) == 4
    return xj, found


def system(xi, xj):
    pos = np.ascontiguousarray(np.stack([xi, xj], axis=1))
    w = W.lj_fcc(2)
    return pos, MDSystem(pos, np.array([[L, L, L]]), np.array([0, 2]), w.pot, w.skin)


def oracle_with(pos, counted):
    """The oracle's (F, E, W) with the pair counted or not: its cutoff moved by
    one unit in the last place so that its own test takes that decision."""
    rc = np.nextafter(RC, np.inf) if counted else np.nextafter(RC, 0.0)
    return oracle.lj(pos, np.array([L, L, L]), np.array([0], np.int32), np.array([1], np.int32),
                     1.0, 1.0, rc)


def gpu(s, precision):
    F, E, Wv = s.forces(precision)
    return F.cpu().numpy(), E.item(), Wv.item()


def close(got, want, tol):
    F, E, Wv = got
    Fo, Eo, Wo = want
    scale = max(np.abs(Fo).max(), 1.0)
    return (np.abs(F - Fo).max() <= tol * scale and abs(E - Eo) <= tol * max(abs(Eo), 1.0)
            and abs(Wv - Wo) <= tol * max(abs(Wo), 1.0))


def test_exact_tie_is_outside():
    xj = np.array([6.0, 6.0, 6.0])
    xi = xj + np.array([1.5, 2.0, 0.0])          # r2 = 6.25 exactly, in every order
    pos, s = system(xi, xj)
    for prec in (B.MD_FP64, B.MD_MIXED):
        F, E, Wv = gpu(s, prec)
        assert np.all(F == 0.0) and E == 0.0 and Wv == 0.0
    start, nbr = s.neighbor_list()
    assert start.tolist() == [0, 1, 2] and nbr.tolist() == [1, 0]


@pytest.mark.parametrize("key", [(True, True), (False, False), (True, False), (False, True)],
                         ids=["both_in", "both_out", "oracle_in_fused_out", "oracle_out_fused_in"])
def test_interior_pair_follows_the_fused_r2(key):
    xj, found = find_pairs()
    pos, s = system(found[key], xj)
    oracle_in, fused_in = key
    s.build()
    start, nbr = s.neighbor_list()
    assert nbr.tolist() == [1, 0], "the pair is in both lists"
    want = oracle_with(pos, fused_in)
    for prec, tol in ((B.MD_FP64, 1e-12), (B.MD_MIXED, 1e-5)):
        got = gpu(s, prec)
        assert close(got, want, tol), (key, prec, got, want)
    if fused_in:
        assert np.abs(want[0]).max() > 0.03          # |f(rc)| = 0.039: the decision matters
    # where both decisions agree the GPU equals the oracle's own result
    if oracle_in == fused_in:
        Fo, Eo, Wo = oracle.forces(pos, np.array([L, L, L]), W.lj_potential(), skin=0.3)
        assert close(gpu(s, B.MD_FP64), (Fo, Eo, Wo), 1e-12)


def test_pair_across_a_face_is_one_of_the_two_results():
    """The same near-cutoff pairs moved so that they straddle the periodic
    face at x = 0: the staged image differs from the oracle's minimum image by
    a rounding of L's size, so either decision is a valid result."""
    xj0, found = find_pairs()
    for key, xi0 in found.items():
        shift = np.array([-xj0[0] + 0.4, 0.0, 0.0])
        xj = xj0 + shift
        xi = xi0 + shift
        pos = oracle.wrap(np.stack([xi, xj], axis=1), np.array([L, L, L]))
        s = MDSystem(pos, np.array([[L, L, L]]), np.array([0, 2]), W.lj_potential(), 0.3)
        got = gpu(s, B.MD_FP64)
        ok = close(got, oracle_with(pos, True), 1e-12) or close(got, oracle_with(pos, False), 1e-12)
        assert ok, (key, got)
        start, nbr = s.neighbor_list()
        assert nbr.tolist() == [1, 0]
