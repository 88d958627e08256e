// md_waves.h -- waves of non-overlapping brick tasks (Sec. II.B, appendix).
//
// The paper groups its cell tasks into waves: sets of tasks whose 3x3x3 cell
// neighbourhoods do not overlap, so a wave can run concurrently without any two
// tasks writing the same particle.  A wave is the Cartesian product of one
// index set per axis.  Along an axis of D task positions with minimum separation
// s (3 for cell tasks), the sets are the s residue classes when D is a multiple
// of s; otherwise (a periodic axis) the positions are visited in steps of s,
// cyclically, and a new set is opened whenever the next position lies closer
// than s to a member of the current one.  Axes are nested loops, x innermost;
// an inner loop is not reset when an outer one advances: its next pass starts
// with the set it ended on, completed along the same walk, and visits every
// position once more.
//
// Here the tasks are bricks of cells.  A brick writes its halo (its cells and
// one layer around them; with the 14-cell half list of Sec. II.D.3 no partner
// lies below an atom's cell, so along z only the layer above: the 3 x 3 x 2
// overlap); along an axis, two bricks s positions apart have
// disjoint write sets for s = 2 as soon as bricks are at least two cells wide,
// and for s = 3 in general; an axis where neither holds (a halo that covers the
// axis) puts every brick in a set of its own.  The separation is checked on the
// actual brick extents (the last brick of an axis may be shorter).
//
// The dependent schedule (task_graph below) replaces the barrier after each
// wave by per-task dependences derived from the same wave order.
//
// Host code only.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

namespace mdwaves {

inline int cyc(int a, int b, int D)
{
    int d = a - b;
    if (d < 0) d = -d;
    d %= D;
    return std::min(d, D - d);
}

// Successive passes of the index sets of one axis.
class Axis {
public:
    Axis(int D, int s) : D_(D), s_(s), residue_(D % s == 0) {}

    std::vector<std::vector<int>> pass()
    {
        std::vector<std::vector<int>> sets;
        if (residue_) {
            const int m = std::min(s_, D_);
            const int first = started_ ? last_class_ : 0;
            for (int t = 0; t < m; t++) {
                const int r = (first + t) % m;
                std::vector<int> cls;
                for (int x = r; x < D_; x += s_) cls.push_back(x);
                sets.push_back(cls);
            }
            last_class_ = (first + m - 1) % m;
        } else {
            int x = started_ ? last_set_.front() : 0;
            for (int t = 0; t < D_; t++, x = (x + s_) % D_) {
                bool far = !sets.empty();
                if (far)
                    for (int y : sets.back())
                        if (cyc(x, y, D_) < s_) {
                            far = false;
                            break;
                        }
                if (far) sets.back().push_back(x);
                else sets.push_back(std::vector<int>{x});
            }
            last_set_ = sets.back();
        }
        started_ = true;
        return sets;
    }

private:
    int D_, s_;
    bool residue_;
    bool started_ = false;
    int last_class_ = 0;
    std::vector<int> last_set_;
};

// Do the cyclic intervals [a, a + la) and [b, b + lb) of a ring of n cells meet?
inline bool rings_meet(int a, int la, int b, int lb, int n)
{
    const int ba = ((b - a) % n + n) % n, ab = ((a - b) % n + n) % n;
    return ba < la || ab < lb;
}

// Separation along one axis of nc cells cut into bricks of bd cells, each
// writing its cells, `below` layers under them (1, or 0 along z for the
// 14-cell half list) and one layer above.
inline int axis_separation(int nc, int bd, int below = 1)
{
    const int D = (nc + bd - 1) / bd;
    std::vector<int> o(D), len(D);
    for (int p = 0; p < D; p++) {
        o[p] = p * bd;
        const int e = std::min(bd, nc - o[p]);
        len[p] = std::min(e + 1 + below, nc);
    }
    for (int s = 2; s <= 3; s++) {
        bool ok = true;
        for (int p = 0; p < D && ok; p++)
            for (int q = p + 1; q < D && ok; q++)
                if (cyc(p, q, D) >= s && rings_meet(o[p] - below + nc, len[p], o[q] - below + nc, len[q], nc)) ok = false;
        if (ok) return s;
    }
    return D;
}

// Colour (wave) of each brick of a grid nb[0] x nb[1] x nb[2] (x fastest) with
// separations sep[3]; returns the number of colours.
inline int colour_bricks(const int32_t nb[3], const int sep[3], std::vector<int32_t> &colour)
{
    colour.assign((size_t)nb[0] * nb[1] * nb[2], -1);
    Axis ax(nb[0], sep[0]), ay(nb[1], sep[1]), az(nb[2], sep[2]);
    int w = 0;
    for (const auto &Z : az.pass())
        for (const auto &Y : ay.pass())
            for (const auto &X : ax.pass()) {
                for (int z : Z)
                    for (int y : Y)
                        for (int x : X) colour[(size_t)x + (size_t)nb[0] * ((size_t)y + (size_t)nb[1] * z)] = w;
                w++;
            }
    return w;
}

// Cells a brick writes along one axis: (o - below + t) mod nc,
// t = 0 .. min(e + 1 + below, nc) - 1 (the brick's cells, `below` layers under
// them and one above).
inline void axis_write_set(int o, int e, int nc, int below, std::vector<int> &out)
{
    out.clear();
    const int len = std::min(e + 1 + below, nc);
    for (int t = 0; t < len; t++) out.push_back(((o - below + t) % nc + nc) % nc);
}

// Dependences between tasks (Sec. II.B): a task waits only for the last earlier
// task, in wave order, that writes each of its cells; these direct predecessors
// order every pair of tasks that share a cell.  The successor lists come from
// the backward method: walk the tasks from the last to the first, keeping for
// every cell the next task that writes it; a task's successors are the
// distinct entries of its cells, after which the task becomes the next writer
// of each of them.
//
// order: the tasks in wave order; cells(t, out) fills the global cell ids that
// task t writes; n_cells: number of global cells; n_tasks: tasks are numbered
// 0 .. n_tasks - 1.  Output: succ_off (n_tasks + 1), succ (each list
// ascending), npred (predecessor count of each task).
template <typename Cells>
inline void task_graph(const std::vector<int32_t> &order, Cells cells, int64_t n_cells, int64_t n_tasks,
                       std::vector<int32_t> &succ_off, std::vector<int32_t> &succ,
                       std::vector<int32_t> &npred)
{
    std::vector<int32_t> next((size_t)n_cells, -1), seen((size_t)n_tasks, -1);
    std::vector<std::vector<int32_t>> lists((size_t)n_tasks);
    std::vector<int64_t> mine;
    for (size_t q = order.size(); q-- > 0;) {
        const int32_t t = order[q];
        mine.clear();
        cells(t, mine);
        std::vector<int32_t> &L = lists[(size_t)t];
        for (int64_t c : mine) {
            const int32_t u = next[(size_t)c];
            if (u >= 0 && seen[(size_t)u] != t) {
                seen[(size_t)u] = t;
                L.push_back(u);
            }
            next[(size_t)c] = t;
        }
        std::sort(L.begin(), L.end());
    }
    succ_off.assign((size_t)n_tasks + 1, 0);
    npred.assign((size_t)n_tasks, 0);
    for (int64_t t = 0; t < n_tasks; t++) {
        succ_off[(size_t)t + 1] = succ_off[(size_t)t] + (int32_t)lists[(size_t)t].size();
        for (int32_t u : lists[(size_t)t]) npred[(size_t)u]++;
    }
    succ.clear();
    succ.reserve((size_t)succ_off[(size_t)n_tasks]);
    for (int64_t t = 0; t < n_tasks; t++) succ.insert(succ.end(), lists[(size_t)t].begin(), lists[(size_t)t].end());
}

} // namespace mdwaves
