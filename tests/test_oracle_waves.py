"""The oracle's task waves against the paper's worked examples (appendix) and
the invariants the paper states for them; the brick separation rule on
hand-checked axes.  The paper counts cells from 1; the oracle from 0."""
import itertools

import pytest

from oracle import waves as W


def one_based(sets):
    return [[x + 1 for x in S] for S in sets]


def test_non_periodic_14_cells_three_sets():
    assert one_based(W.axis_sets(14, 3, periodic=False)) == [
        [1, 4, 7, 10, 13], [2, 5, 8, 11, 14], [3, 6, 9, 12]]


def test_periodic_14_cells_four_sets():
    assert one_based(W.axis_sets(14, 3, periodic=True)) == [
        [1, 4, 7, 10], [13, 2, 5, 8], [11, 14, 3, 6], [9, 12]]


@pytest.mark.parametrize("periodic,row", [
    (False, [1, 2, 3, 1, 2, 3, 1, 2, 3, 1, 2, 3, 1, 2]),
    (True, [1, 2, 3, 1, 2, 3, 1, 2, 4, 1, 3, 4, 2, 3]),
])
def test_coverage_rows_of_the_14_cell_examples(periodic, row):
    wave_of = {}
    for w, S in enumerate(W.axis_sets(14, 3, periodic)):
        for x in S:
            wave_of[x + 1] = w + 1
    assert [wave_of[x] for x in range(1, 15)] == row


def test_periodic_14_by_6_first_five_waves():
    """x (14 cells) innermost, y (6 cells) outer: four waves on the y set {1, 4},
    then the fifth repeats the fourth x pattern {9, 12} completed to {9, 12, 1, 4}
    on the y set {2, 5}.  (The sixth wave's printed pattern is garbled; the
    text's rule gives {7, 10, 13, 2}, tested as a reading below.)"""
    ws = W.waves([14, 6], [3, 3], [True, True])
    xs = [sorted({x + 1 for x, _ in w}) for w in ws]
    ys = [sorted({y + 1 for _, y in w}) for w in ws]
    assert xs[:5] == [[1, 4, 7, 10], [2, 5, 8, 13], [3, 6, 11, 14], [9, 12], [1, 4, 9, 12]]
    assert ys[:4] == [[1, 4]] * 4 and ys[4] == [2, 5]
    assert xs[5] == [2, 7, 10, 13] and ys[5] == [2, 5]


def test_invalid_set_from_the_paper_overlaps():
    a, b = (2 - 1, 2 - 1), (4 - 1, 2 - 1)     # {2,4} x {2,5}: cells (2,2) and (4,2)
    assert W.overlapping(a, b, [14, 14], [True, True])
    assert not W.overlapping((1, 1), (4, 1), [14, 14], [True, True])


@pytest.mark.parametrize("dims,count", [
    ((6, 6, 6), 27), ((7, 6, 6), 36), ((6, 7, 8), 48), ((7, 8, 10), 64), ((9, 12, 15), 27),
    ((38, 38, 38), 64), ((14, 6, 9), 36),
])
def test_wave_counts_27_36_48_64(dims, count):
    assert len(W.waves(dims, [3, 3, 3])) == count


@pytest.mark.parametrize("dims", [(6, 6, 6), (7, 8, 10), (14, 6, 9), (5, 7, 11), (4, 4, 13)])
def test_waves_cover_every_cell_once_and_never_overlap(dims):
    ws = W.waves(dims, [3, 3, 3])
    seen = [c for w in ws for c in w]
    assert len(seen) == len(set(seen)) == dims[0] * dims[1] * dims[2]
    for w in ws:
        for a, b in itertools.combinations(w, 2):
            assert not W.overlapping(a, b, dims, [True] * 3)


def test_inner_axis_passes_each_cover_the_axis():
    ax = W.AxisPasses(14, 3)
    for _ in range(5):
        p = ax.next_pass()
        assert sorted(x for S in p for x in S) == list(range(14))
        assert len(p) == 4


def test_small_periodic_axes_fall_back_to_single_positions():
    assert W.axis_sets(5, 3) == [[0], [3], [1], [4], [2]]
    assert W.axis_sets(2, 3) == [[0], [1]]
    assert W.axis_sets(3, 3) == [[0], [1], [2]]


@pytest.mark.parametrize("nc,b,sep", [
    (38, 1, 3),      # cell tasks: the paper's separation
    (38, 2, 2), (38, 3, 2), (38, 4, 2),
    (13, 4, 3),      # bricks 4, 4, 4, 1: bricks 0 and 2 share cell 12 (the 1-cell brick's)
    (17, 4, 3),      # bricks 4, 4, 4, 4, 1: bricks 0 and 3 (two apart across the ring) share cell 16
    (9, 4, 2),       # three bricks: no two are two apart, every set is one brick
    (4, 2, 2),       # two bricks: likewise
    (3, 1, 2),       # three 1-cell bricks whose halos cover the axis: likewise
])
def test_brick_axis_separation(nc, b, sep):
    assert W.axis_separation(nc, b) == sep


def test_brick_colours_keep_write_sets_disjoint():
    for nc, shape in [((38, 38, 38), (4, 3, 2)), ((9, 10, 11), (4, 4, 4)), ((7, 5, 13), (1, 1, 1)),
                      ((6, 6, 6), (2, 3, 1)), ((13, 17, 9), (4, 4, 4)), ((3, 4, 5), (1, 2, 2))]:
        colour, n = W.brick_colours(nc, shape)
        nb = [len(W.brick_ranges(nc[d], shape[d])) for d in range(3)]
        sets = [[W.write_set(o, e, nc[d]) for o, e in W.brick_ranges(nc[d], shape[d])] for d in range(3)]
        by = {}
        for idx, c in enumerate(colour):
            by.setdefault(c, []).append((idx % nb[0], (idx // nb[0]) % nb[1], idx // (nb[0] * nb[1])))
        assert sorted(by) == list(range(n))
        for members in by.values():
            for p, q in itertools.combinations(members, 2):
                assert any(not (sets[d][p[d]] & sets[d][q[d]]) for d in range(3)), (nc, shape, p, q)


# ---------------------------------------------------------------- dependent schedule (Sec. II.B)
GRIDS = [((6, 6, 6), (1, 1, 1)), ((7, 5, 4), (1, 1, 1)), ((9, 10, 11), (4, 4, 4)),
         ((13, 7, 6), (4, 3, 2)), ((4, 4, 4), (1, 1, 1)), ((5, 6, 3), (2, 2, 1))]


def cells_of(nc, shape):
    return lambda t: W.brick_write_cells(nc, shape, t)


@pytest.mark.parametrize("nc,shape", GRIDS)
def test_forward_and_backward_methods_give_the_same_graph(nc, shape):
    colour, _ = W.brick_colours(nc, shape)
    order = W.wave_order(colour)
    pred = W.predecessors_forward(order, cells_of(nc, shape))
    succ = W.successors_backward(order, cells_of(nc, shape))
    transposed = {t: set() for t in order}
    for t, S in succ.items():
        for s in S:
            transposed[s].add(t)
    assert transposed == pred


@pytest.mark.parametrize("nc,shape", GRIDS[:4])
def test_direct_predecessors_by_their_definition(nc, shape):
    """t -> s exactly when t comes before s, both write some cell c, and no
    task between them in wave order writes c (brute force over all pairs)."""
    succ, order = W.brick_task_graph(nc, shape)
    pos = {t: k for k, t in enumerate(order)}
    cells = {t: set(W.brick_write_cells(nc, shape, t)) for t in order}
    for t in order:
        expect = set()
        for s in order[pos[t] + 1:]:
            for c in cells[t] & cells[s]:
                if not any(c in cells[u] for u in order[pos[t] + 1:pos[s]]):
                    expect.add(s)
                    break
        assert succ[t] == expect, t


@pytest.mark.parametrize("nc,shape", GRIDS)
def test_the_graph_orders_every_pair_that_shares_a_cell(nc, shape):
    """The paper's argument: waiting for the last earlier writer of each cell
    orders a task after every earlier task it shares a cell with."""
    succ, order = W.brick_task_graph(nc, shape)
    reach = {}
    for t in reversed(order):                 # successors come later in the order
        r = set()
        for s in succ[t]:
            r |= {s} | reach[s]
        reach[t] = r
    cells = {t: set(W.brick_write_cells(nc, shape, t)) for t in order}
    for i, t in enumerate(order):
        for s in order[i + 1:]:
            if cells[t] & cells[s]:
                assert s in reach[t], (t, s)


@pytest.mark.parametrize("nc,shape", GRIDS)
def test_no_edge_inside_a_wave_and_depth_within_the_wave_count(nc, shape):
    colour, nw = W.brick_colours(nc, shape)
    succ, order = W.brick_task_graph(nc, shape)
    depth = {}
    for t in reversed(order):
        for s in succ[t]:
            assert colour[s] > colour[t]
        depth[t] = 1 + max((depth[s] for s in succ[t]), default=0)
    assert max(depth.values()) <= nw


def test_cell_tasks_have_at_most_27_direct_predecessors():
    nc = (7, 8, 10)
    pred = W.predecessors_forward(W.wave_order(W.brick_colours(nc, (1, 1, 1))[0]),
                                  cells_of(nc, (1, 1, 1)))
    assert max(len(p) for p in pred.values()) <= 27
    assert sum(len(p) == 0 for p in pred.values()) == sum(
        1 for c in W.brick_colours(nc, (1, 1, 1))[0] if c == 0)


# ---------------------------------------------------------------- stricter overlap (Sec. II.D.3)
def test_stricter_overlap_puts_50_percent_more_cell_tasks_in_a_wave():
    """With the 3 x 3 x 2 overlap, cell tasks on a 6 x 6 x 6 grid need 18 waves
    of 12 tasks instead of 27 waves of 8 (the paper's figure of up to 50 %)."""
    c27, n27 = W.brick_colours((6, 6, 6), (1, 1, 1))
    c18, n18 = W.brick_colours((6, 6, 6), (1, 1, 1), shell=True)
    assert (n27, n18) == (27, 18)
    assert all(c27.count(k) == 8 for k in range(27))
    assert all(c18.count(k) == 12 for k in range(18))
    assert W.axis_separation(6, 1, below=0) == 2 and W.axis_separation(6, 1) == 3


@pytest.mark.parametrize("nc,shape", [((38, 38, 38), (1, 1, 1)), ((9, 10, 11), (4, 4, 4)),
                                      ((7, 5, 13), (1, 1, 1)), ((6, 6, 5), (2, 3, 1)),
                                      ((3, 4, 5), (1, 2, 2)), ((13, 7, 6), (4, 3, 2))])
def test_shell_colours_keep_the_3x3x2_write_sets_disjoint(nc, shape):
    colour, n = W.brick_colours(nc, shape, shell=True)
    nb = [len(W.brick_ranges(nc[d], shape[d])) for d in range(3)]
    lo = W.below_layers(True)
    sets = [[W.write_set(o, e, nc[d], lo[d]) for o, e in W.brick_ranges(nc[d], shape[d])] for d in range(3)]
    by = {}
    for idx, c in enumerate(colour):
        by.setdefault(c, []).append((idx % nb[0], (idx // nb[0]) % nb[1], idx // (nb[0] * nb[1])))
    assert sorted(by) == list(range(n))
    for members in by.values():
        for p, q in itertools.combinations(members, 2):
            assert any(not (sets[d][p[d]] & sets[d][q[d]]) for d in range(3)), (nc, shape, p, q)
    assert n <= W.brick_colours(nc, shape)[1]


@pytest.mark.parametrize("nc,shape", GRIDS[:4])
def test_shell_graph_by_its_definition(nc, shape):
    succ, order = W.brick_task_graph(nc, shape, shell=True)
    pos = {t: k for k, t in enumerate(order)}
    cells = {t: set(W.brick_write_cells(nc, shape, t, shell=True)) for t in order}
    for t in order:
        expect = set()
        for s in order[pos[t] + 1:]:
            for c in cells[t] & cells[s]:
                if not any(c in cells[u] for u in order[pos[t] + 1:pos[s]]):
                    expect.add(s)
                    break
        assert succ[t] == expect, t
