// md_list.hip -- Verlet neighbor lists built cell by cell (Sec. II.A).
//
// One wavefront per cell (a "cell task").  The distinct cells of the 3x3x3
// neighbourhood are found by 27 lanes, their atoms staged into the wave's LDS
// slice (in chunks if they do not fit), and every atom of the centre cell then
// tests all candidates, 64 lanes at a time:
//   d = x_i - x_j;  d > L/2 -> d - L,  d < -L/2 -> d + L;  r2 = (dx*dx + dy*dy) + dz*dz
// in binary64 with contraction off, kept iff r2 < (rc + skin)^2 (and, for the
// half list, j after i in the sorted order).  Hits are compacted with a ballot
// and a lane prefix count into the atom's own row, so each row has exactly one
// writer and no atomics are needed (each task owns its lists, Sec. II.C).  The
// image chosen by the minimum-image rule is stored with the entry.
#include "md_internal.h"

namespace {

constexpr int CAP = 384;   // staged candidates per wavefront (6 x 64)
constexpr int WPB = 4;     // wavefronts per workgroup

__global__ __launch_bounds__(256) void k_build_list(ListArgs a)
{
    if (*a.pred == 0) return;
    __shared__ double sx[WPB][CAP];
    __shared__ double sy[WPB][CAP];
    __shared__ double sz[WPB][CAP];
    __shared__ int32_t sj[WPB][CAP];

    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const ItemRange it = xcd_items(a.C, WPB, w);

    for (int64_t c = it.first; c < it.end; c += it.stride) {
        // replica of this cell (replica cell ranges are contiguous)
        int32_t r = 0;
        if (a.R > 1) {
            int32_t lo = 0, hi = a.R - 1;
            while (lo < hi) {
                int32_t mid = (lo + hi + 1) >> 1;
                if (a.reps[mid].cell_off <= c) lo = mid; else hi = mid - 1;
            }
            r = lo;
        }
        const RepDesc &rep = a.reps[r];
        const int32_t nx = rep.nc[0], ny = rep.nc[1], nz = rep.nc[2];
        const int64_t lc = c - rep.cell_off;
        const int32_t cx = (int32_t)(lc % nx);
        const int32_t cy = (int32_t)((lc / nx) % ny);
        const int32_t cz = (int32_t)(lc / ((int64_t)nx * ny));

        // distinct neighbourhood cells: lane s < 27 holds offset (s%3-1, s/3%3-1, s/9-1)
        int64_t nb = -1;
        if (lane < 27) {
            int32_t x = (cx + lane % 3 - 1 + nx) % nx;
            int32_t y = (cy + (lane / 3) % 3 - 1 + ny) % ny;
            int32_t z = (cz + lane / 9 - 1 + nz) % nz;
            nb = rep.cell_off + x + (int64_t)nx * (y + (int64_t)ny * z);
        }
        bool dup = false;
        for (int l = 0; l < 27; l++) {
            int64_t o = __shfl(nb, l, 64);
            dup |= (l < lane) && (o == nb);
        }
        int32_t beg = 0, num = 0;
        if (lane < 27 && !dup) {
            beg = a.start[nb];
            num = a.start[nb + 1] - beg;
        }
        int32_t inc = num;
        for (int o = 1; o < 64; o <<= 1) {
            int32_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        const int32_t off = inc - num;
        const int32_t total = __shfl(inc, 63, 64);

        const int32_t s0 = a.start[c], s1 = a.start[c + 1];
        const double Lx = rep.L[0], Ly = rep.L[1], Lz = rep.L[2];
        const double hx = rep.hL[0], hy = rep.hL[1], hz = rep.hL[2];

        for (int32_t base = 0; base < total; base += CAP) {
            const int32_t len = total - base < CAP ? total - base : CAP;
            // stage candidates [base, base + len) of the concatenated neighbourhood
            for (int s = 0; s < 27; s++) {
                const int32_t sb = __shfl(beg, s, 64);
                const int32_t sn = __shfl(num, s, 64);
                const int32_t so = __shfl(off, s, 64);
                if (so + sn <= base || so >= base + len) continue;
                for (int32_t k = lane; k < sn; k += 64) {
                    const int32_t slot = so + k - base;
                    if (slot >= 0 && slot < len) {
                        const double4 p = a.src[sb + k];
                        sx[w][slot] = p.x;
                        sy[w][slot] = p.y;
                        sz[w][slot] = p.z;
                        sj[w][slot] = sb + k;
                    }
                }
            }
            wave_sync();
            for (int32_t i = s0; i < s1; i++) {
                const double4 xi = a.src[i];
                int32_t ni = base == 0 ? 0 : a.cnt[i];
                for (int32_t k0 = 0; k0 < len; k0 += 64) {
                    const int32_t k = k0 + lane;
                    bool hit = false;
                    uint32_t entry = 0;
                    if (k < len) {
                        const int32_t j = sj[w][k];
                        double dx = xi.x - sx[w][k];
                        double dy = xi.y - sy[w][k];
                        double dz = xi.z - sz[w][k];
                        uint32_t code = 0;
                        if (dx > hx) { dx = dx - Lx; code |= 2u; }
                        else if (dx < -hx) { dx = dx + Lx; code |= 1u; }
                        if (dy > hy) { dy = dy - Ly; code |= 8u; }
                        else if (dy < -hy) { dy = dy + Ly; code |= 4u; }
                        if (dz > hz) { dz = dz - Lz; code |= 32u; }
                        else if (dz < -hz) { dz = dz + Lz; code |= 16u; }
                        const double r2 = (dx * dx + dy * dy) + dz * dz;
                        hit = (r2 < a.rl2) && (j != i) && (!a.half || j > i);
                        entry = (uint32_t)j | (code << MD_IDX_BITS);
                    }
                    const uint64_t mask = __ballot(hit);
                    const int32_t p = ni + (int32_t)lanes_below(mask);
                    if (hit && p < a.M) a.nbr[(int64_t)i * a.M + p] = entry;
                    ni += __popcll(mask);
                }
                // every lane stores the (uniform) count, so each lane re-reads its own
                // store when a later chunk continues this row
                a.cnt[i] = ni;
                if (lane == 0) {
                    if (base + CAP >= total) {
                        atomicMax(&a.ctl->max_cnt, ni);
                        if (ni > a.M && a.M > 0) atomicOr(&a.ctl->err, MD_FLAG_OVERFLOW);
                    }
                }
            }
            wave_sync();
        }
        // copy the freshly sorted state of this cell into the working buffers
        if (a.pos_dst != nullptr) {
            for (int32_t i = s0 + lane; i < s1; i += 64) {
                const double4 p = a.src[i];
                a.pos_dst[i] = p;
                a.xref[i] = p;
                a.id_dst[i] = a.id_src[i];
                if (a.vel_dst != nullptr) {
                    a.vel_dst[i] = a.vel_src[i];
                    a.vel_dst[a.n + i] = a.vel_src[a.n + i];
                    a.vel_dst[2 * a.n + i] = a.vel_src[2 * a.n + i];
                }
            }
        }
    }
}

} // namespace

void launch_build_list(hipStream_t s, int grid, const ListArgs &a)
{
    hipLaunchKernelGGL(k_build_list, dim3(grid), dim3(256), 0, s, a);
}
