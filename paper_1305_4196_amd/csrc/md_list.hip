// md_list.hip -- Verlet neighbor lists built cell by cell (Sec. II.A).
//
// One workgroup per cell (a "cell task", md_nbhd.h).  The neighbourhood's
// candidates (the atoms of the distinct cells of the 3x3x3 block) are staged in
// LDS once; candidates beyond the staged part are read from global memory.  The
// four wavefronts share the centre cell's atoms (atom s0 + w, s0 + w + 4, ...),
// and for each atom the 64 lanes test all candidates:
//   d = x_i - x_j;  d > L/2 -> d - L,  d < -L/2 -> d + L;  r2 = (dx*dx + dy*dy) + dz*dz
// in binary64 with contraction off, kept iff r2 < (rc + skin)^2 and j != i (and,
// for the half list, j after i in the sorted order).  Hits are compacted with a
// ballot and a lane prefix count into the atom's own row, so every row has
// exactly one writer and no atomics are needed (each task owns its lists,
// Sec. II.C).  An entry holds the candidate index and the image code.
//
// Interior cells: along an axis with at least 5 cells, no neighbour of a cell
// that is not on the box face can be more than 2 cell widths (< L/2) away, so
// the minimum-image branch never fires and is skipped -- the arithmetic (and so
// the pair set) is unchanged.
#include "md_nbhd.h"

namespace {

__global__ __launch_bounds__(256) void k_build_list(ListArgs a)
{
    if (*a.pred == 0) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t smax[4], stot[4];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const Stage st = stage_slice(lds_raw, 0, a.cap, 0);
    const ItemRange it = xcd_items(a.C, 1, 0);
    int32_t wave_max = 0, wave_tot = 0;

    for (int64_t c = it.first; c < it.end; c += it.stride) {
        const int32_t s0 = a.start[c], s1 = a.start[c + 1];
        if (s1 == s0) continue;
        const CellGeom g = cell_geom(a.reps, a.R, c);
        __syncthreads();
        if (w == 0) nbhd_setup(a.reps, g, a.start, *st.L);
        __syncthreads();
        task_stage(st, a.src, nullptr);
        __syncthreads();
        const int32_t total = st.L->soff[27];
        wave_tot = total > wave_tot ? total : wave_tot;

        const RepDesc &rep = a.reps[g.r];
        const double Lx = rep.L[0], Ly = rep.L[1], Lz = rep.L[2];
        const double hx = rep.hL[0], hy = rep.hL[1], hz = rep.hL[2];
        const bool wrapx = !(g.nx >= 5 && g.cx >= 1 && g.cx <= g.nx - 2);
        const bool wrapy = !(g.ny >= 5 && g.cy >= 1 && g.cy <= g.ny - 2);
        const bool wrapz = !(g.nz >= 5 && g.cz >= 1 && g.cz <= g.nz - 2);
        const int32_t gself0 = nbhd_centre(*st.L);
        const bool all_staged = total <= st.cap;

        for (int32_t i = s0 + w; i < s1; i += 4) {
            const double4 xi = a.src[i];
            const int32_t gself = gself0 + (i - s0);
            const int64_t row = i * (int64_t)a.M;
            int32_t ni = 0;
            STAGED_SPLIT(all_staged,
            for (int32_t k0 = 0; k0 < total; k0 += 64) {
                const int32_t k = k0 + lane;
                bool hit = false;
                uint32_t code = 0;
                if (k < total) {
                    double xj, yj, zj;
                    int32_t j;
                    candidate<STAGED>(st, k, a.src, xj, yj, zj, j);
                    double dx = xi.x - xj, dy = xi.y - yj, dz = xi.z - zj;
                    if (wrapx) {
                        if (dx > hx) { dx = dx - Lx; code |= 2u; }
                        else if (dx < -hx) { dx = dx + Lx; code |= 1u; }
                    }
                    if (wrapy) {
                        if (dy > hy) { dy = dy - Ly; code |= 8u; }
                        else if (dy < -hy) { dy = dy + Ly; code |= 4u; }
                    }
                    if (wrapz) {
                        if (dz > hz) { dz = dz - Lz; code |= 32u; }
                        else if (dz < -hz) { dz = dz + Lz; code |= 16u; }
                    }
                    const double r2 = (dx * dx + dy * dy) + dz * dz;
                    hit = (r2 < a.rl2) && (k != gself) && (!a.half || j > i);
                }
                const uint64_t mask = __ballot(hit);
                const int32_t p = ni + (int32_t)lanes_below(mask);
                if (hit && p < a.M) a.nbr[row + p] = (uint32_t)k | (code << MD_IDX_BITS);
                ni += __popcll(mask);
            }
            )
            if (lane == 0) a.cnt[i] = ni;
            wave_max = ni > wave_max ? ni : wave_max;
        }

        // copy the freshly sorted state of this cell into the working buffers
        if (a.pos_dst != nullptr) {
            for (int32_t i = s0 + threadIdx.x; i < s1; i += 256) {
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
    // one atomic per workgroup (a per-atom atomic on one word would serialise in L2)
    if (lane == 0) {
        smax[w] = wave_max;
        stot[w] = wave_tot;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = smax[0], t = stot[0];
        for (int k = 1; k < 4; k++) {
            m = smax[k] > m ? smax[k] : m;
            t = stot[k] > t ? stot[k] : t;
        }
        atomicMax(&a.ctl->max_cnt, m);
        atomicMax(&a.ctl->max_nbhd, t);
        if (m > a.M && a.M > 0) atomicOr(&a.ctl->err, MD_FLAG_OVERFLOW);
    }
}

} // namespace

void launch_build_list(hipStream_t s, int grid, const ListArgs &a)
{
    const size_t lds = nbhd_lds_bytes(a.cap, 0);
    allow_lds(k_build_list, lds);
    hipLaunchKernelGGL(k_build_list, dim3(grid), dim3(256), lds, s, a);
}
