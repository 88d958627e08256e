"""Pins of the oracle's periodic geometry, linked cells and pair sets.

The pair set has a plain definition (every pair whose minimum-image distance
is below the cutoff); the linked-cell enumeration of Sec. II.A must reproduce
it exactly.  Two exhaustive enumerations pin it: the oracle's own O(N^2) loop
and an independent vectorised numpy one written here.
"""
import numpy as np
import pytest

import oracle
from paper_1305_4196_amd import workloads as W


def numpy_pairs(x, L, cut, full):
    """Exhaustive pair set, vectorised: {(i, j) : |minimage(x_i - x_j)| < cut}."""
    x = np.asarray(x)
    L = np.asarray(L, dtype=np.float64)
    d = x[:, :, None] - x[:, None, :]
    hL = (0.5 * L)[:, None, None]
    d = np.where(d > hL, d - L[:, None, None], np.where(d < -hL, d + L[:, None, None], d))
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    n = x.shape[1]
    ii, jj = np.nonzero(r2 < cut * cut)
    keep = ii != jj if full else ii < jj
    return set(zip(ii[keep].tolist(), jj[keep].tolist()))


def random_box(seed, n, L):
    g = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64)
    return g.uniform(0, 1, size=(3, n)) * L[:, None], L


def csr_pairs(start, nbr):
    n = start.size - 1
    return {(i, int(j)) for i in range(n) for j in nbr[start[i]:start[i + 1]]}


# ---------------------------------------------------------------- wrap
def test_wrap_boundaries():
    L = np.array([5.0, 7.0, 3.0])
    x = np.array([[5.0, -1e-300, 0.0, np.nextafter(5.0, 0), 12.5, -2.5],
                  [7.0, -7.0, 14.0, 3.5, -0.0, 1e-17],
                  [3.0, 6.0, -3.0, 2.9999999999999996, 1.5, -1e-17]])
    y = oracle.wrap(x, L)
    assert np.all(y >= 0) and np.all(y < L[:, None])
    assert y[0, 0] == 0.0 and y[0, 1] == 0.0 and y[0, 3] == np.nextafter(5.0, 0)
    assert y[0, 4] == 2.5 and y[0, 5] == 2.5
    assert y[1, 0] == 0.0 and y[1, 1] == 0.0 and y[1, 2] == 0.0
    # a tiny negative coordinate rounds up to L and must come back to 0
    assert y[2, 5] == 0.0


def test_wrap_is_periodic_shift():
    g = np.random.default_rng(1)
    L = np.array([6.5, 9.25, 11.0])
    x = g.uniform(-40, 40, size=(3, 500))
    y = oracle.wrap(x, L)
    k = (x - y) / L[:, None]
    assert np.all(y >= 0) and np.all(y < L[:, None])
    assert np.max(np.abs(k - np.round(k))) < 1e-12


# ---------------------------------------------------------------- cells
@pytest.mark.parametrize("L,rl", [((6.72, 6.72, 6.72), 2.8), ((9.0, 12.5, 17.3), 2.8),
                                  ((8.4, 8.4, 8.4), 2.8), ((40.0, 23.0, 11.7), 3.9)])
def test_binning_invariants(L, rl):
    x, L = random_box(7, 800, L)
    x = oracle.wrap(x, L)
    c = oracle.bin_cells(x, L, rl)
    nc = c["nc"]
    assert tuple(nc) == tuple(int(np.floor(l / rl)) for l in L)
    cs, order, cell_of = c["cell_start"], c["order"], c["cell_of"]
    assert cs[0] == 0 and cs[-1] == x.shape[1] and np.all(np.diff(cs) >= 0)
    assert np.array_equal(np.sort(order), np.arange(x.shape[1]))
    for cell in range(nc.prod()):
        members = order[cs[cell]:cs[cell + 1]]
        assert np.all(np.diff(members) > 0), "within a cell, ascending atom id"
        assert np.all(cell_of[members] == cell)
    # each atom lies inside its cell (cell width L/nc), x fastest flattening
    cx = cell_of % nc[0]
    cy = (cell_of // nc[0]) % nc[1]
    cz = cell_of // (nc[0] * nc[1])
    for d, cc in enumerate((cx, cy, cz)):
        w = L[d] / nc[d]
        assert np.all(x[d] >= cc * w - 1e-12) and np.all(x[d] < (cc + 1) * w + 1e-12)


def test_binning_on_cell_faces():
    L = np.array([8.4, 8.4, 8.4])   # 3 cells of width 2.8 per dimension
    faces = np.array([0.0, 2.8, 5.6, np.nextafter(8.4, 0)])
    g = np.stack(np.meshgrid(faces, faces, faces, indexing="ij")).reshape(3, -1)
    c = oracle.bin_cells(g, L, 2.8)
    cx = c["cell_of"] % 3
    expect = np.minimum(np.floor(g[0] * 3 / 8.4), 2).astype(int)
    assert np.array_equal(cx, expect)
    assert set(np.unique(cx)) == {0, 1, 2}


def test_grid_rejects_small_box():
    assert oracle.grid((5.5, 10, 10), 2.8) is None
    assert oracle.grid((5.6, 10, 10), 2.8) == (2, 3, 3)


# ---------------------------------------------------------------- pair sets
CASES = [((6.2, 6.2, 6.2), 2.8, 160),      # 2 cells per dimension (stencil aliases)
         ((8.5, 6.0, 11.9), 2.8, 300),     # mixed 3/2/4
         ((12.0, 12.0, 12.0), 2.8, 700),
         ((16.8, 9.3, 7.8), 3.9, 400)]


@pytest.mark.parametrize("L,rl,n", CASES)
def test_brute_force_matches_numpy(L, rl, n):
    x, L = random_box(3, n, L)
    pi, pj = oracle.pairs_brute(x, L, rl, full=True)
    assert set(zip(pi.tolist(), pj.tolist())) == numpy_pairs(x, L, rl, True)
    pi, pj = oracle.pairs_brute(x, L, rl, full=False)
    assert set(zip(pi.tolist(), pj.tolist())) == numpy_pairs(x, L, rl, False)


@pytest.mark.parametrize("L,rl,n", CASES)
def test_cell_lists_match_brute_force(L, rl, n):
    x, L = random_box(11, n, L)
    x = oracle.wrap(x, L)
    start, nbr = oracle.neighbor_list(x, L, rl, full=True)
    full = csr_pairs(start, nbr)
    assert full == numpy_pairs(x, L, rl, True)
    # symmetry j in N(i) <=> i in N(j)
    assert all((j, i) in full for (i, j) in full)
    # half list: each pair once, held by the atom earlier in the cell-sorted order
    hs, hn = oracle.neighbor_list(x, L, rl, full=False)
    half = csr_pairs(hs, hn)
    assert 2 * len(half) == len(full)
    assert {(min(i, j), max(i, j)) for i, j in half} == numpy_pairs(x, L, rl, False)
    rank = np.empty(x.shape[1], dtype=np.int64)
    rank[oracle.bin_cells(x, L, rl)["order"]] = np.arange(x.shape[1])
    assert all(rank[j] > rank[i] for i, j in half)
    # per-atom lists ascending
    for i in range(x.shape[1]):
        assert np.all(np.diff(nbr[start[i]:start[i + 1]]) > 0)


def test_exact_tie_is_outside():
    """r2 == rl^2 exactly is not a neighbour (strict test)."""
    L = np.array([12.0, 12.0, 12.0])
    x = np.array([[1.0, 3.75, 6.0, 6.0], [1.0, 1.0, 6.0, 6.0], [1.0, 1.0, 1.0, 3.5]])
    # atoms 0-1: d = 2.75 = rl exactly; atoms 2-3: d = 2.5 < rl
    start, nbr = oracle.neighbor_list(x, L, 2.75, full=True)
    got = csr_pairs(start, nbr)
    assert (0, 1) not in got and (2, 3) in got and (3, 2) in got
    pi, pj = oracle.pairs_brute(x, L, 2.75)
    assert set(zip(pi.tolist(), pj.tolist())) == {(2, 3)}


def test_minimum_image_across_faces():
    L = np.array([10.0, 10.0, 10.0])
    x = np.array([[0.1, 9.9, 5.0], [5.0, 5.0, 0.05], [5.0, 5.0, 9.0]])
    # 0-1 are 0.2 apart through the x face
    pi, pj = oracle.pairs_brute(x, L, 1.0)
    assert set(zip(pi.tolist(), pj.tolist())) == {(0, 1)}


def test_fcc_neighbour_shells():
    """fcc at density 0.8442: 78 neighbours within 2.8 (12+6+24+12+24), 54 within 2.5."""
    w = W.lj_fcc(5)
    L = w.boxes[0]
    x = oracle.wrap(w.pos, L)
    start, _ = oracle.neighbor_list(x, L, 2.8, full=True)
    assert np.all(np.diff(start) == 78)
    start, _ = oracle.neighbor_list(x, L, 2.5, full=True)
    assert np.all(np.diff(start) == 54)


# ---------------------------------------------------------------- the 14-cell half list
def unwrapped_offset(x, L, nc, coords, i, j):
    """Cell offset of j's minimum image from i's cell, per axis."""
    o = []
    for a in range(3):
        d = x[a, i] - x[a, j]
        s = 1 if d > 0.5 * L[a] else (-1 if d < -0.5 * L[a] else 0)
        o.append(int(coords[a, j] + s * nc[a] - coords[a, i]))
    return tuple(o)


@pytest.mark.parametrize("L,rl,n", CASES)
def test_shell_list_holds_every_pair_once_within_a_3x3x2_block(L, rl, n):
    x, L = random_box(17, n, L)
    x = oracle.wrap(x, L)
    start, nbr = oracle.shell_list(x, L, rl)
    sh = csr_pairs(start, nbr)
    ref = numpy_pairs(x, L, rl, False)
    assert len(sh) == len(ref)
    assert {(min(i, j), max(i, j)) for i, j in sh} == ref
    b = oracle.bin_cells(x, L, rl)
    nc, cell = b["nc"], b["cell_of"]
    coords = np.stack([cell % nc[0], (cell // nc[0]) % nc[1], cell // (nc[0] * nc[1])])
    seen = set()
    for i, j in sh:
        o = unwrapped_offset(x, L, nc, coords, i, j)
        assert all(-1 <= v <= 1 for v in o)
        assert o[2] in (0, 1)              # never a partner in the layer below
        seen.add(o)
    # of two mirrored cell offsets only one is ever used: 13 + the own cell
    assert not any(tuple(-v for v in o) in seen for o in seen if o != (0, 0, 0))
    assert len(seen) <= 14
    if min(nc) >= 3:
        assert len(seen) == 14


def test_shell_list_gives_the_half_list_forces():
    """Same pairs, other owners: forces, energy and virial agree to rounding."""
    x, L = random_box(5, 700, (12.0, 12.0, 12.0))
    x = oracle.wrap(x, L)
    rl = 2.8
    hs, hn = oracle.neighbor_list(x, L, rl, full=False)
    ss, sn = oracle.shell_list(x, L, rl)
    out = []
    for st, nb in ((hs, hn), (ss, sn)):
        pi = np.repeat(np.arange(x.shape[1], dtype=np.int32), np.diff(st)).astype(np.int32)
        out.append(oracle.lj(x, L, pi, nb.astype(np.int32), rc=2.5))
    (Fa, Ea, Wa), (Fb, Eb, Wb) = out
    assert np.max(np.abs(Fa - Fb)) <= 1e-12 * np.max(np.abs(Fa))
    assert Eb == pytest.approx(Ea, rel=1e-13)
    assert Wb == pytest.approx(Wa, rel=1e-12)
