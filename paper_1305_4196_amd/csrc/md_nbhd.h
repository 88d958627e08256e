// md_nbhd.h -- the neighbourhood of a cell task, shared by list, force and adjoint kernels.
//
// A cell task (Sec. II.A) is one workgroup working on one cell.  Its
// neighbourhood is the distinct cells of the 3x3x3 block around it, taken in
// the order (dz, dy, dx) = (-1..1)^3 with dx fastest and duplicates (grids of 2
// cells per axis) dropped at their first occurrence.  The atoms of these cells,
// concatenated in that order, are the task's candidates; candidate g lives in
// neighbourhood cell s with soff[s] <= g < soff[s+1], at sorted index
// sbeg[s] + g - soff[s].  List entries store g (low 26 bits) plus the image code
// (high 6 bits), so the force and adjoint tasks can stage the same candidates
// in LDS and read every neighbour from there.
//
// List layout: atom i (sorted order) owns the row nbr[i*M .. i*M + M) and uses
// its first cnt[i] entries; M is a multiple of 8, so rows start 16-byte aligned.
#pragma once

#include "md_internal.h"

struct NbhdLds {
    int32_t soff[28];   // exclusive prefix of the cell sizes; soff[27] = total
    int32_t sbeg[28];   // first sorted index of each neighbourhood cell
};

// allow a kernel to take `bytes` of dynamic LDS (once per size)
template <typename K>
inline void allow_lds(K kernel, size_t bytes)
{
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// bytes of LDS per cell task: staged x, y, z (binary64) and sorted index for
// `cap` candidates, `extra` more binary64 per candidate, and the offsets
__host__ __device__ inline size_t nbhd_lds_bytes(int cap, int extra)
{
    return (size_t)cap * (3 * sizeof(double) + sizeof(int32_t) + extra * sizeof(double)) + sizeof(NbhdLds);
}

#ifdef __HIPCC__

struct CellGeom {
    int32_t r;          // replica
    int32_t cx, cy, cz; // cell coordinates
    int32_t nx, ny, nz;
};

__device__ __forceinline__ CellGeom cell_geom(const RepDesc *reps, int32_t R, int64_t c)
{
    CellGeom g;
    int32_t r = 0;
    if (R > 1) {
        int32_t lo = 0, hi = R - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (reps[mid].cell_off <= c) lo = mid; else hi = mid - 1;
        }
        r = lo;
    }
    const RepDesc &rep = reps[r];
    g.r = r;
    g.nx = rep.nc[0];
    g.ny = rep.nc[1];
    g.nz = rep.nc[2];
    // a replica has fewer than 2^31 cells: 32-bit division suffices
    const uint32_t lc = (uint32_t)(c - rep.cell_off);
    const uint32_t q = lc / (uint32_t)g.nx;
    g.cx = (int32_t)(lc - q * (uint32_t)g.nx);
    g.cy = (int32_t)(q % (uint32_t)g.ny);
    g.cz = (int32_t)(q / (uint32_t)g.ny);
    return g;
}

// Fills L with the neighbourhood of cell c and returns the candidate count.
// Must be called by all 64 lanes of the wavefront.
__device__ __forceinline__ int32_t nbhd_setup(const RepDesc *reps, const CellGeom &g,
                                              const int32_t *start, NbhdLds &L)
{
    const int lane = threadIdx.x & 63;
    const int64_t coff = reps[g.r].cell_off;
    int64_t nb = -1;
    if (lane < 27) {
        const int32_t x = (g.cx + lane % 3 - 1 + g.nx) % g.nx;
        const int32_t y = (g.cy + (lane / 3) % 3 - 1 + g.ny) % g.ny;
        const int32_t z = (g.cz + lane / 9 - 1 + g.nz) % g.nz;
        nb = coff + x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
    }
    bool dup = false;
    for (int l = 0; l < 27; l++) {
        const int64_t o = __shfl(nb, l, 64);
        dup |= (l < lane) && (o == nb);
    }
    int32_t beg = 0, num = 0;
    if (lane < 27 && !dup) {
        beg = start[nb];
        num = start[nb + 1] - beg;
    }
    int32_t inc = num;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    const int32_t total = __shfl(inc, 63, 64);
    if (lane < 27) {
        L.soff[lane] = inc - num;
        L.sbeg[lane] = beg;
    }
    if (lane == 27) L.soff[27] = total;
    wave_sync();
    return total;
}

// sorted index of candidate g (binary search over the neighbourhood offsets)
__device__ __forceinline__ int32_t nbhd_index(const NbhdLds &L, int32_t g)
{
    int32_t lo = 0, hi = 26;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (L.soff[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return L.sbeg[lo] + (g - L.soff[lo]);
}

// candidate index of the centre cell's first atom (neighbourhood cell 13 is the
// centre and never a duplicate: every other offset has a non-zero component)
__device__ __forceinline__ int32_t nbhd_centre(const NbhdLds &L) { return L.soff[13]; }

// 1/x in binary64: hardware reciprocal refined by two Newton steps (within
// 1 ulp of the correctly rounded quotient, without the scaled-division sequence)
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ void apply_image_code(uint32_t e, double Lx, double Ly, double Lz,
                                                 double &dx, double &dy, double &dz)
{
    const uint32_t c = e >> MD_IDX_BITS;
    if (c & 1u) dx = dx + Lx;
    if (c & 2u) dx = dx - Lx;
    if (c & 4u) dy = dy + Ly;
    if (c & 8u) dy = dy - Ly;
    if (c & 16u) dz = dz + Lz;
    if (c & 32u) dz = dz - Lz;
}

// LDS slice of a cell task within a dynamically sized shared block.
struct Stage {
    double *x, *y, *z;
    int32_t *j;
    double *ex;         // extra per-candidate binary64 (may be null)
    NbhdLds *L;
    int cap;
};

__device__ __forceinline__ Stage stage_slice(void *base, int wave, int cap, int extra)
{
    char *p = (char *)base + nbhd_lds_bytes(cap, extra) * wave;
    Stage s;
    s.cap = cap;
    s.x = (double *)p;
    s.y = s.x + cap;
    s.z = s.y + cap;
    s.ex = extra ? s.z + cap : nullptr;
    s.j = (int32_t *)(s.z + cap + extra * cap);
    s.L = (NbhdLds *)(s.j + cap);
    return s;
}

// Position (and sorted index) of candidate g.  STAGED = true is the path of a
// cell whose whole neighbourhood fits the LDS slice: pure LDS reads.  The other
// path (neighbourhoods larger than the slice) falls back to global memory past
// the staged part.  The two are separate instantiations selected once per cell,
// so the common path never merges LDS and global addresses into flat loads.
template <bool STAGED>
__device__ __forceinline__ void candidate_pos(const Stage &s, int32_t g, const double4 *pos,
                                              double &x, double &y, double &z)
{
    if (STAGED || g < s.cap) {
        x = s.x[g];
        y = s.y[g];
        z = s.z[g];
    } else {
        const double4 p = pos[nbhd_index(*s.L, g)];
        x = p.x;
        y = p.y;
        z = p.z;
    }
}

template <bool STAGED>
__device__ __forceinline__ void candidate(const Stage &s, int32_t g, const double4 *pos, double &x,
                                          double &y, double &z, int32_t &j)
{
    if (STAGED || g < s.cap) {
        x = s.x[g];
        y = s.y[g];
        z = s.z[g];
        j = s.j[g];
    } else {
        j = nbhd_index(*s.L, g);
        const double4 p = pos[j];
        x = p.x;
        y = p.y;
        z = p.z;
    }
}

// runs the block once with STAGED = true or false (uniform per cell)
#define STAGED_SPLIT(ALL_STAGED, ...)                                                     \
    if (ALL_STAGED) {                                                                     \
        constexpr bool STAGED = true;                                                     \
        __VA_ARGS__                                                                       \
    } else {                                                                              \
        constexpr bool STAGED = false;                                                    \
        __VA_ARGS__                                                                       \
    }

// ---------------------------------------------------------------- cell-task loop
// A cell task is one 256-thread workgroup per cell (persistent grid, cells split
// in XCD-sized ranges).  Wave 0 sets up the neighbourhood, all threads stage its
// candidates (thread t < 243 copies atoms t%9, t%9+9, ... of neighbourhood cell
// t/9), and the cell's atoms are spread over the threads: `tpa` = floor(256/m)
// threads per atom (at most 64), each walking its share of the atom's row four
// entries at a time.  Per-thread partial sums are combined through LDS by the
// atom's first thread in thread order, so the result is deterministic.
constexpr int TASK_THREADS = 256;

struct TaskLds {
    NbhdLds L;
    int32_t total;
    int32_t pad;
};

// stage the candidates of the block's current cell (block-wide)
__device__ __forceinline__ void task_stage(const Stage &s, const double4 *pos, const double *extra)
{
    const int t = threadIdx.x;
    if (t < 243) {
        const int nb = t / 9;
        const int32_t o = s.L->soff[nb];
        const int32_t num = s.L->soff[nb + 1] - o;
        const int32_t beg = s.L->sbeg[nb];
        for (int32_t k = t % 9; k < num; k += 9) {
            const int32_t g = o + k;
            if (g >= s.cap) break;
            const double4 p = pos[beg + k];
            s.x[g] = p.x;
            s.y[g] = p.y;
            s.z[g] = p.z;
            s.j[g] = beg + k;
            if (extra != nullptr) s.ex[g] = extra[beg + k];
        }
    }
}

// Sums v over the `tpa` threads of each atom group through LDS (red: 256 doubles
// per component); the group's first thread receives the totals in thread order.
template <int NV>
__device__ __forceinline__ void task_group_sum(double (&v)[NV], int tpa, int am, double *red)
{
    const int t = threadIdx.x;
    if (tpa == 1) return;   // block-uniform
    for (int c = 0; c < NV; c++) {
        __syncthreads();
        red[t] = v[c];
        __syncthreads();
        if (tpa > 1 && t % tpa == 0 && t / tpa < am) {
            double acc = red[t];
            for (int k = 1; k < tpa; k++) acc += red[t + k];
            v[c] = acc;
        }
    }
}

#define CELL_TASK_BEGIN(EXTRA_STAGE)                                                      \
    const ItemRange it_ = xcd_items(a.C, 1, 0);                                           \
    for (int64_t c = it_.first; c < it_.end; c += it_.stride) {                           \
        const int32_t s0 = a.start[c], s1 = a.start[c + 1];                               \
        if (s1 == s0) continue;                                                           \
        const CellGeom g_ = cell_geom(a.reps, a.R, c);                                    \
        __syncthreads();                                                                  \
        if (threadIdx.x < 64) nbhd_setup(a.reps, g_, a.start, *st.L);                     \
        __syncthreads();                                                                  \
        task_stage(st, a.pos, EXTRA_STAGE);                                               \
        __syncthreads();                                                                  \
        const RepDesc &rep_ = a.reps[g_.r];                                               \
        const double Lx = rep_.L[0], Ly = rep_.L[1], Lz = rep_.L[2];                      \
        const bool all_staged = st.L->soff[27] <= st.cap;                                 \
        for (int32_t a0 = s0; a0 < s1; a0 += TASK_THREADS) {                              \
            const int am = s1 - a0 < TASK_THREADS ? s1 - a0 : TASK_THREADS;               \
            int tpa = TASK_THREADS / am;                                                  \
            tpa = tpa > 64 ? 64 : tpa;                                                    \
            const int grp = threadIdx.x / tpa, sub = threadIdx.x % tpa;                   \
            const bool valid = grp < am;                                                  \
            const int64_t i = a0 + grp;                                                   \
            const int32_t mm = valid ? (a.cnt[i] < a.M ? a.cnt[i] : a.M) : 0;             \
            const uint4 *row4 = reinterpret_cast<const uint4 *>(a.nbr + (valid ? i * (int64_t)a.M : 0)); \
            const int32_t nq = (mm + 3) >> 2;

#define CELL_TASK_END                                                                     \
        }                                                                                 \
    }

#endif
