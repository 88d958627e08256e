"""Task waves of the cell-task method (Sec. II.B and the appendix) -- TEST INFRASTRUCTURE ONLY.

Plain Python, indices 0-based (the paper counts from 1).  Used by the tests to
pin the wave construction to the paper's worked examples and to check the
library's brick colouring against an independent statement of it.

One dimension, D positions, minimum separation s (3 for cell tasks, whose
3-cell neighbourhoods must not overlap):
  * a non-periodic axis, or D a multiple of s: s residue classes
    {0, s, 2s, ...}, {1, 1+s, ...}, ... in that order;
  * a periodic axis with D not a multiple of s: walk 0, s, 2s, ... modulo D and
    cut the walk into sets, opening a new set whenever the next position lies
    closer than s (cyclically) to a member of the current one.
Several dimensions: nested loops, the first axis innermost.  An inner loop is
not reset when an outer one advances: its next pass starts with the last set of
its previous pass, completed along the same walk, and goes on from there, each
position once per pass (the reading of the appendix used here; the appendix's
figure of the sixth wave of the 14 x 6 example is garbled, the text's rule --
further steps of s along the walk -- is followed).

Dependent schedule (Sec. II.B): instead of a barrier after every wave, a task
waits only for its direct predecessors -- for each cell it writes, the last
earlier task (in wave order) that writes the same cell.  Two ways to find them,
both as the paper describes: the forward method keeps, per cell, the last task
seen so far while walking the tasks first to last (predecessor lists); the
backward method keeps, per cell, the next task while walking last to first
(successor lists).

Stricter overlap (Sec. II.D.3): with the half list over 14 of the 27 cells an
atom's partners never lie in the layer below its cell, so a cell task writes a
3 x 3 x 2 block instead of 3 x 3 x 3, and tasks two cells apart along z no
longer overlap (below = 0 along z in write_set).

Brick colouring (this design's GPU tasks are bricks of cells): a brick writes
the cells of its halo (its cells and one layer around them, the same
coordinates the brick record uses); two bricks may share a wave only if their
write sets are disjoint.  Along each axis the separation is 2 when every pair of
bricks two apart has disjoint write sets, else 3 when that holds for three
apart, else every brick of the axis is a set of its own.
"""
from __future__ import annotations

import itertools
import math
from typing import List, Sequence, Tuple


def cyc_dist(a: int, b: int, D: int) -> int:
    d = abs(a - b) % D
    return min(d, D - d)


class AxisPasses:
    """Successive passes of the index sets of one axis (the not-reset loop)."""

    def __init__(self, D: int, s: int, periodic: bool = True):
        self.D, self.s, self.periodic = D, s, periodic
        self.residue = (not periodic) or D % s == 0
        if not self.residue and math.gcd(D, s) != 1:
            raise ValueError("periodic walk needs gcd(D, s) = 1")
        self.last = None          # last set of the previous pass

    def _far(self, x: int, members: Sequence[int]) -> bool:
        if self.periodic:
            return all(cyc_dist(x, m, self.D) >= self.s for m in members)
        return all(abs(x - m) >= self.s for m in members)

    def next_pass(self) -> List[List[int]]:
        D, s = self.D, self.s
        if self.residue:
            classes = [list(range(r, D, s)) for r in range(min(s, D))]
            if self.last is None:
                order = list(range(len(classes)))
            else:
                k = self.last
                order = [(k + t) % len(classes) for t in range(len(classes))]
            self.last = order[-1]
            return [classes[k] for k in order]
        start = 0 if self.last is None else self.last[0]
        walk = [(start + t * s) % D for t in range(D)]
        sets: List[List[int]] = [[walk[0]]]
        for x in walk[1:]:
            if self._far(x, sets[-1]):
                sets[-1].append(x)
            else:
                sets.append([x])
        self.last = sets[-1]
        return sets


def axis_sets(D: int, s: int = 3, periodic: bool = True) -> List[List[int]]:
    """The first pass of one axis (the appendix's one-dimensional sets)."""
    return AxisPasses(D, s, periodic).next_pass()


def waves(dims: Sequence[int], seps: Sequence[int], periodic: Sequence[bool] = (True, True, True)
          ) -> List[List[Tuple[int, ...]]]:
    """All waves of a grid of 1 to 3 axes (axis 0 innermost); each wave is the
    list of its positions (tuples, axis 0 first)."""
    nd = len(dims)
    gens = [AxisPasses(dims[d], seps[d], periodic[d]) for d in range(nd)]
    out: List[List[Tuple[int, ...]]] = []

    def rec(d: int, outer: Tuple[List[int], ...]):
        for S in gens[d].next_pass():
            sets = (S,) + outer
            if d == 0:
                out.append(_product(sets))
            else:
                rec(d - 1, sets)

    rec(nd - 1, ())
    return out


def _product(sets: Tuple[List[int], ...]) -> List[Tuple[int, ...]]:
    return [tuple(t) for t in itertools.product(*sets)]


def overlapping(a: Tuple[int, ...], b: Tuple[int, ...], dims: Sequence[int], periodic: Sequence[bool]) -> bool:
    """True if the 3^d-cell neighbourhoods of cell tasks a and b share a cell."""
    for d in range(len(dims)):
        dist = cyc_dist(a[d], b[d], dims[d]) if periodic[d] else abs(a[d] - b[d])
        if dist >= 3:
            return False
    return True


# ---------------------------------------------------------------- bricks
def brick_ranges(nc: int, b: int) -> List[Tuple[int, int]]:
    """(origin, extent) of the bricks along an axis of nc cells, bricks of b cells."""
    return [(o, min(b, nc - o)) for o in range(0, nc, b)]


def write_set(o: int, e: int, nc: int, below: int = 1) -> set:
    """Cells a brick writes along one axis: its cells, `below` layers under them
    and one above, (o - below + t) mod nc.  below = 1 for a list whose partners
    lie on both sides; below = 0 along z for the 14-cell half list (Sec. II.D.3:
    the 3 x 3 x 2 overlap)."""
    return {(o - below + t) % nc for t in range(min(e + 1 + below, nc))}


def axis_separation(nc: int, b: int, below: int = 1) -> int:
    """Smallest separation (2, then 3) such that any two bricks of the axis at
    least that far apart (cyclically, in brick index) have disjoint write sets;
    the number of bricks when neither works (each brick a set of its own)."""
    br = brick_ranges(nc, b)
    D = len(br)
    ws = [write_set(o, e, nc, below) for o, e in br]
    for s in (2, 3):
        if all(not (ws[p] & ws[q]) for p in range(D) for q in range(p + 1, D) if cyc_dist(p, q, D) >= s):
            return s
    return D


def below_layers(shell: bool) -> List[int]:
    """Layers under a brick that it writes, per axis: one on every axis, except
    along z for the 14-cell half list, whose partners never lie below."""
    return [1, 1, 0 if shell else 1]


def brick_colours(nc: Sequence[int], bshape: Sequence[int], shell: bool = False) -> Tuple[List[int], int]:
    """Colour (wave index) of every brick of one replica, bricks numbered x
    fastest, and the number of colours."""
    nb = [len(brick_ranges(nc[d], bshape[d])) for d in range(3)]
    lo = below_layers(shell)
    seps = [axis_separation(nc[d], bshape[d], lo[d]) for d in range(3)]
    ws = waves(nb, seps)
    colour = [-1] * (nb[0] * nb[1] * nb[2])
    for w, cells in enumerate(ws):
        for (x, y, z) in cells:
            colour[x + nb[0] * (y + nb[1] * z)] = w
    return colour, len(ws)


# ---------------------------------------------------------------- dependences
def brick_write_cells(nc: Sequence[int], bshape: Sequence[int], b: int,
                      shell: bool = False) -> List[Tuple[int, int, int]]:
    """Cells (x, y, z) written by brick b (numbered x fastest) of a grid nc cut into bshape bricks."""
    nb = [len(brick_ranges(nc[d], bshape[d])) for d in range(3)]
    idx = (b % nb[0], (b // nb[0]) % nb[1], b // (nb[0] * nb[1]))
    lo = below_layers(shell)
    sets = []
    for d in range(3):
        o, e = brick_ranges(nc[d], bshape[d])[idx[d]]
        sets.append(sorted(write_set(o, e, nc[d], lo[d])))
    return [(x, y, z) for z in sets[2] for y in sets[1] for x in sets[0]]


def wave_order(colour: Sequence[int]) -> List[int]:
    """Tasks wave by wave, by index within a wave."""
    return sorted(range(len(colour)), key=lambda t: (colour[t], t))


def predecessors_forward(order: Sequence[int], cells) -> dict:
    """Forward method: {task: set of direct predecessors}."""
    last = {}
    pred = {}
    for t in order:
        pred[t] = set()
        for c in cells(t):
            if c in last:
                pred[t].add(last[c])
            last[c] = t
    return pred


def successors_backward(order: Sequence[int], cells) -> dict:
    """Backward method: {task: set of direct successors}."""
    nxt = {}
    succ = {}
    for t in reversed(order):
        succ[t] = set()
        for c in cells(t):
            if c in nxt:
                succ[t].add(nxt[c])
            nxt[c] = t
    return succ


def brick_task_graph(nc: Sequence[int], bshape: Sequence[int], shell: bool = False) -> Tuple[dict, List[int]]:
    """Successor sets of the bricks of one grid (backward method over the wave
    order of brick_colours) and that order."""
    colour, _ = brick_colours(nc, bshape, shell)
    order = wave_order(colour)
    succ = successors_backward(order, lambda t: brick_write_cells(nc, bshape, t, shell))
    return succ, order
