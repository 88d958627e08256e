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
// one layer around them); along an axis, two bricks s positions apart have
// disjoint write sets for s = 2 as soon as bricks are at least two cells wide,
// and for s = 3 in general; an axis where neither holds (a halo that covers the
// axis) puts every brick in a set of its own.  The separation is checked on the
// actual brick extents (the last brick of an axis may be shorter).
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

// Separation along one axis of nc cells cut into bricks of bd cells.
inline int axis_separation(int nc, int bd)
{
    const int D = (nc + bd - 1) / bd;
    std::vector<int> o(D), len(D);
    for (int p = 0; p < D; p++) {
        o[p] = p * bd;
        const int e = std::min(bd, nc - o[p]);
        len[p] = std::min(e + 2, nc);
    }
    for (int s = 2; s <= 3; s++) {
        bool ok = true;
        for (int p = 0; p < D && ok; p++)
            for (int q = p + 1; q < D && ok; q++)
                if (cyc(p, q, D) >= s && rings_meet(o[p] - 1 + nc, len[p], o[q] - 1 + nc, len[q], nc)) ok = false;
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

} // namespace mdwaves
