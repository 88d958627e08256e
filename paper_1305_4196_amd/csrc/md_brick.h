// md_brick.h -- cell tasks blocked into bricks of cells (Sec. II.A, II.D.2).
//
// A task is one workgroup working on a brick of bx x by x bz cells (the blocking
// of Sec. II.D.2; its shape is a tuning parameter).  The brick's halo is the
// distinct cells of the (bx+2) x (by+2) x (bz+2) block around it: along an axis
// with origin o, extent e and n cells the halo coordinates are
//   (o - 1 + t) mod n,  t = 0 .. min(e + 2, n) - 1,
// which are distinct and, when e + 2 > n, cover the axis once.  The atoms of the
// halo cells, concatenated in halo order (x fastest), are the task's
// candidates; halo cell h holds candidates soff[h] .. soff[h+1]-1, the first of
// them at sorted index sbeg[h].  Every neighbour of every atom of the brick is
// a candidate, so the tasks stage the candidates in LDS once and read all
// neighbours from there.  A list entry holds the candidate index (low 26 bits)
// and the image code (high 6 bits) fixed when the list was built.
//
// Image of a halo cell: along an axis of n >= 4 cells whose halo does not wrap
// onto itself (e + 2 <= n), the layer below a brick at the low face is cell n-1
// seen through -L, the layer above one at the high face cell 0 seen through +L,
// and every other halo cell is seen directly.  A listed pair is closer than
// r_c + skin <= one cell width along each axis, while the cell image puts its
// atoms at most two cell widths (plus rounding) apart; a different image would
// move them by L >= 4 cell widths, so the list's minimum-image code of every
// entry equals the image of its candidate's halo cell.  Such bricks, when
// their whole halo fits the force and adjoint tasks' LDS stage (BR_SHIFT = 1),
// stage their candidates already shifted by the cell image, their list
// entries carry no code and the pair loops apply none; the others (an axis of
// fewer than 4 cells, a halo that covers its axis, or one only partly staged)
// keep the per-entry codes.  The stage capacity is fixed when the list is
// built (changing it drops the list), so the flag the list build records holds
// for every later task.  (The list build stages up to its own, possibly
// smaller, capacity; BR_SHIFT follows the tasks' stage.)
//
// Each lane owns one atom of its brick (lane t of a workgroup of T threads
// takes the brick's atoms t, t + T, ...; T is a multiple of 64 up to 512), so
// the atom's sums stay in registers and no atom is written by two lanes: the
// cell-task invariant of Sec. II.A by ownership.
//
// Brick record (int32, one per brick, written by the list build, read by the
// force and adjoint tasks so that they skip the setup):
//   [BR_TOTAL] candidates  [BR_ATOMS] atoms  [BR_REP] replica  [BR_H] halo cells
//   [BR_E] own cells  [BR_IMG] 1 if pairs need the per-entry image codes
//   [BR_SHIFT] 1 if the halo is staged through the cell images (entries carry no
//              code and use the narrow 16-bit layout)
//   [BR_FACE] 1 if some halo cell is seen through an image (the brick touches a
//              face of the box); staging through the images of a brick without
//              one is a plain copy
//   soff[Hm+1]  sbeg[Hm]  aoff[Em+1]  abeg[Em]  himg[Hm]
// (aoff/abeg: the same for the brick's own cells, in x-fastest order; himg:
// the image code of each halo cell, in the list-entry encoding.)
//
// List layout (interleaved rows): entry p of sorted atom i is word
//   ((i/64) * M/4 + p/4) * 256 + (i%64) * 4 + p%4
// so lane i reads its entries four at a time (one 16-byte load) and the 64
// atoms of a row group read 1 KiB contiguously.  M is a multiple of 8.  Atoms
// of BR_SHIFT bricks store 16-bit entries in the same rows, eight per 16-byte
// group (ell_half), and read half the bytes.
#pragma once

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>

#include "md_internal.h"
#include "md_reduce.h"

constexpr int TASK_MAX_THREADS = 512;

enum { BR_TOTAL = 0, BR_ATOMS = 1, BR_REP = 2, BR_H = 3, BR_E = 4, BR_IMG = 5, BR_SHIFT = 6, BR_FACE = 7, BR_HDR = 8 };

__host__ __device__ inline int32_t br_soff(const BrickDims &d) { (void)d; return BR_HDR; }
__host__ __device__ inline int32_t br_sbeg(const BrickDims &d) { return BR_HDR + d.Hm + 1; }
__host__ __device__ inline int32_t br_aoff(const BrickDims &d) { return BR_HDR + 2 * d.Hm + 1; }
__host__ __device__ inline int32_t br_abeg(const BrickDims &d) { return BR_HDR + 2 * d.Hm + d.Em + 2; }
__host__ __device__ inline int32_t br_himg(const BrickDims &d) { return BR_HDR + 2 * d.Hm + 2 * d.Em + 2; }
__host__ __device__ inline int32_t br_stride(int32_t Hm, int32_t Em)
{
    return (BR_HDR + 3 * Hm + 2 * Em + 2 + 3) / 4 * 4;
}

// word index of entry p of sorted atom i in the interleaved list
__host__ __device__ inline int64_t ell_word(int64_t i, int64_t p, int32_t M)
{
    return (((i >> 6) * (M >> 2) + (p >> 2)) << 8) + ((i & 63) << 2) + (p & 3);
}

// 16-bit index of entry p of sorted atom i in the narrow layout (bricks with
// BR_SHIFT = 1, whose entries are bare candidate indices below 65536): the same
// 16-byte groups hold eight entries, entry p at halfword
//   ((i/64) * M/4 + p/8) * 512 + (i%64) * 8 + p%8
// (the first M/8 groups of the atom's rows)
__host__ __device__ inline int64_t ell_half(int64_t i, int64_t p, int32_t M)
{
    return (((i >> 6) * (M >> 2) + (p >> 3)) << 9) + ((i & 63) << 3) + (p & 7);
}

// allow a kernel to take `bytes` of dynamic LDS (the attribute is set only when a
// kernel needs more than before, so launches recorded into a graph after a
// first eager call make no attribute calls)
inline void allow_lds_ptr(const void *kernel, size_t bytes)
{
    static std::mutex mu;
    static std::unordered_map<const void *, size_t> done;
    std::lock_guard<std::mutex> lock(mu);
    size_t &have = done[kernel];
    if (bytes <= have) return;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess)
        have = bytes;
}

template <typename K>
inline void allow_lds(K kernel, size_t bytes)
{
    allow_lds_ptr(reinterpret_cast<const void *>(kernel), bytes);
}

// At most as many workgroups as the device keeps resident at once (registers,
// LDS and wavefront slots all counted): a persistent brick-task grid with more
// would run its surplus after the first ones and double the tail of the static
// schedules.  Queried once per kernel, block size, LDS size and device.
inline int resident_grid_ptr(const void *kernel, int grid, int threads, size_t lds)
{
    static std::mutex mu;
    static std::map<std::tuple<const void *, int, size_t, int>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return grid;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(kernel, threads, lds, dev);
    auto it = cache.find(key);
    if (it == cache.end()) {
        int occ = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, lds) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || occ <= 0 ||
            ncu <= 0)
            return grid;
        it = cache.emplace(key, occ * ncu).first;
    }
    return std::max(1, std::min(grid, it->second));
}

template <typename K>
inline int resident_grid(K kernel, int grid, int threads, size_t lds)
{
    return resident_grid_ptr(reinterpret_cast<const void *>(kernel), grid, threads, lds);
}

// dynamic LDS of a task: staged (x, y, z) (binary64, interleaved) of `cap`
// candidates, `nextra` more binary64 per candidate, their sorted indices
// (optional), the brick record and the halo cell of each staged candidate
// (16 bits)
__host__ __device__ inline size_t stage_bytes(int cap, int nextra, bool with_j, int32_t stride)
{
    return (size_t)cap * ((3 + nextra) * sizeof(double) + (with_j ? sizeof(int32_t) : 0)) +
           (size_t)stride * sizeof(int32_t) + (((size_t)cap * sizeof(uint16_t) + 15) & ~(size_t)15);
}

#ifdef __HIPCC__

struct Stage {
    double *xyz;        // x, y, z of candidate g at xyz[3g .. 3g+2]
    double *ex;         // extra k of candidate g at ex[k * cap + g] (null if none)
    int32_t *j;         // sorted index of each candidate (null if not staged)
    int32_t *rec;       // brick record (then, in brick tasks, the halo cell of each staged candidate)
    int cap;
};

__device__ __forceinline__ Stage stage_slice(void *base, int cap, int nextra, bool with_j)
{
    Stage s;
    s.cap = cap;
    s.xyz = (double *)base;
    s.ex = nextra ? s.xyz + 3 * (size_t)cap : nullptr;
    int32_t *p = (int32_t *)(s.xyz + 3 * (size_t)cap + (size_t)nextra * cap);
    s.j = with_j ? p : nullptr;
    s.rec = with_j ? p + cap : p;
    return s;
}

// geometry of brick b (list build only; the other tasks read the record)
struct BrickGeom {
    int32_t r;
    int32_t o[3], e[3], hn[3], nc[3];
    int64_t cell_off;
};

__device__ __forceinline__ BrickGeom brick_geom(const RepDesc *reps, int32_t R, int64_t b)
{
    int32_t r = 0;
    if (R > 1) {
        int32_t lo = 0, hi = R - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (reps[mid].brick_off <= b) lo = mid; else hi = mid - 1;
        }
        r = lo;
    }
    const RepDesc &rep = reps[r];
    BrickGeom g;
    g.r = r;
    g.cell_off = rep.cell_off;
    // fewer than 2^31 bricks per replica: 32-bit division suffices
    uint32_t lb = (uint32_t)(b - rep.brick_off);
    uint32_t bi[3];
    bi[0] = lb % (uint32_t)rep.nb[0];
    lb /= (uint32_t)rep.nb[0];
    bi[1] = lb % (uint32_t)rep.nb[1];
    bi[2] = lb / (uint32_t)rep.nb[1];
    for (int d = 0; d < 3; d++) {
        g.nc[d] = rep.nc[d];
        g.o[d] = (int32_t)bi[d] * rep.bd[d];
        g.e[d] = min(rep.bd[d], rep.nc[d] - g.o[d]);
        g.hn[d] = min(g.e[d] + 2, rep.nc[d]);
    }
    return g;
}

// In-place exclusive scan of a[0..n) by one wavefront (all 64 lanes call it);
// a[n] receives the total.
__device__ __forceinline__ void wave_scan_lds(int32_t *a, int32_t n)
{
    const int lane = threadIdx.x & 63;
    const int32_t per = (n + 63) >> 6;
    const int32_t b = lane * per;
    const int32_t e = b + per < n ? b + per : n;
    int32_t s = 0;
    for (int32_t k = b; k < e; k++) s += a[k];
    int32_t inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    int32_t run = inc - s;
    for (int32_t k = b; k < e; k++) {
        const int32_t v = a[k];
        a[k] = run;
        run += v;
    }
    if (lane == 63) a[n] = inc;
    wave_sync();
}

// Builds the record of brick g in LDS (block-wide; ends with a barrier).
__device__ __forceinline__ void brick_setup(const Stage &s, const BrickDims &d, const BrickGeom &g,
                                            const int32_t *start, int32_t shift_cap)
{
    int32_t *rec = s.rec;
    int32_t *soff = rec + br_soff(d), *sbeg = rec + br_sbeg(d);
    int32_t *aoff = rec + br_aoff(d), *abeg = rec + br_abeg(d), *himg = rec + br_himg(d);
    const int32_t H = g.hn[0] * g.hn[1] * g.hn[2];
    const int32_t E = g.e[0] * g.e[1] * g.e[2];
    const int64_t nx = g.nc[0], nxy = (int64_t)g.nc[0] * g.nc[1];
    for (int32_t h = threadIdx.x; h < H; h += blockDim.x) {
        const int32_t px = h % g.hn[0], t = h / g.hn[0];
        const int32_t py = t % g.hn[1], pz = t / g.hn[1];
        const int32_t cx = (g.o[0] - 1 + px + g.nc[0]) % g.nc[0];
        const int32_t cy = (g.o[1] - 1 + py + g.nc[1]) % g.nc[1];
        const int32_t cz = (g.o[2] - 1 + pz + g.nc[2]) % g.nc[2];
        const int64_t cell = g.cell_off + cx + nx * cy + nxy * cz;
        const int32_t b0 = start[cell];
        soff[h] = start[cell + 1] - b0;
        sbeg[h] = b0;
        // image code (bit 0: d + L, bit 1: d - L per axis) of the halo cell
        const int32_t q[3] = {g.o[0] - 1 + px, g.o[1] - 1 + py, g.o[2] - 1 + pz};
        int32_t code = 0;
        for (int k = 0; k < 3; k++) {
            if (q[k] < 0) code |= 1 << (2 * k);
            else if (q[k] >= g.nc[k]) code |= 2 << (2 * k);
        }
        himg[h] = code;
    }
    for (int32_t e = threadIdx.x; e < E; e += blockDim.x) {
        const int32_t ex = e % g.e[0], t = e / g.e[0];
        const int32_t ey = t % g.e[1], ez = t / g.e[1];
        const int64_t cell = g.cell_off + (g.o[0] + ex) + nx * (g.o[1] + ey) + nxy * (g.o[2] + ez);
        const int32_t b0 = start[cell];
        aoff[e] = start[cell + 1] - b0;
        abeg[e] = b0;
    }
    __syncthreads();
    // (workgroups have at least two wavefronts)
    const int w = threadIdx.x >> 6;
    if (w == 0) wave_scan_lds(soff, H);
    if (w == 1) wave_scan_lds(aoff, E);
    __syncthreads();
    if (threadIdx.x == 0) {
        rec[BR_TOTAL] = soff[H];
        rec[BR_ATOMS] = aoff[E];
        rec[BR_REP] = g.r;
        rec[BR_H] = H;
        rec[BR_E] = E;
        bool img = false;
        for (int k = 0; k < 3; k++) img |= g.nc[k] < 4 || g.e[k] + 2 > g.nc[k];
        rec[BR_IMG] = img ? 1 : 0;
        rec[BR_SHIFT] = !img && soff[H] <= shift_cap && soff[H] <= 65536 ? 1 : 0;
        int32_t face = 0;
        for (int32_t h = 0; h < H; h++) face |= himg[h];
        rec[BR_FACE] = face != 0 ? 1 : 0;
    }
    __syncthreads();
}

// halo cell holding candidate k (largest h with soff[h] <= k)
__device__ __forceinline__ int32_t halo_cell(const Stage &s, int32_t k)
{
    const int32_t *soff = s.rec + BR_HDR;
    int32_t lo = 0, hi = s.rec[BR_H] - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (soff[mid] <= k) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t candidate_index(const Stage &s, const BrickDims &d, int32_t k)
{
    const int32_t h = halo_cell(s, k);
    return s.rec[br_sbeg(d) + h] + (k - s.rec[BR_HDR + h]);
}

// sorted index of the brick's atom la (la < atoms); *e receives its own cell
__device__ __forceinline__ int64_t brick_atom(const Stage &s, const BrickDims &d, int32_t la,
                                              int32_t *e = nullptr)
{
    const int32_t *aoff = s.rec + br_aoff(d);
    int32_t lo = 0, hi = s.rec[BR_E] - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (aoff[mid] <= la) lo = mid; else hi = mid - 1;
    }
    if (e != nullptr) *e = lo;
    return s.rec[br_abeg(d) + lo] + (la - aoff[lo]);
}

// the image shift of a list entry, as an addition: bit 0 adds L, bit 1
// subtracts it (d + 0 leaves every non-zero d unchanged)
__device__ __forceinline__ double image_shift(uint32_t code, uint32_t add_bit, double L)
{
    return (code & add_bit) ? L : ((code & (add_bit << 1)) ? -L : 0.0);
}

// p[j] for a sorted atom index j (below 2^26): a 32-bit unsigned byte offset,
// so that the gather takes one scalar base plus a vector offset
template <typename T>
__device__ __forceinline__ T at32(const T *p, int32_t j)
{
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) + (uint32_t)j * (uint32_t)sizeof(T));
}

// Copies the record of brick b into LDS and stages its first `cap` candidates
// (block-wide; ends with a barrier).  extra0/extra1 (may be null) are staged
// as extras 0 and 1; vec (may be null) as three more extras (its x, y, z)
// starting at extra vec_at.  A brick with BR_SHIFT = 1 has its candidates
// staged through their halo cell's image (x_j - shift, so that x_i - x_j' is
// the shifted difference); pairs of it take no image code.
__device__ __forceinline__ void brick_load(const Stage &s, const BrickDims &d, const int32_t *grec,
                                           const RepDesc *reps, const double4 *pos,
                                           const double *extra0, const double *extra1,
                                           const double4 *vec = nullptr, int vec_at = 0)
{
    for (int32_t t = threadIdx.x; t < d.stride; t += blockDim.x) s.rec[t] = grec[t];
    __syncthreads();
    const int32_t total = s.rec[BR_TOTAL];
    const int32_t lim = total < s.cap ? total : s.cap;
    // (a brick away from the box faces sees every halo cell directly)
    const bool shifted = s.rec[BR_SHIFT] != 0 && s.rec[BR_FACE] != 0;
    const RepDesc &rep = reps[s.rec[BR_REP]];
    const double Lx = rep.L[0], Ly = rep.L[1], Lz = rep.L[2];
    // the halo cell of every staged candidate, one cell per thread, so that
    // the staging below reads it instead of searching the cell offsets
    uint16_t *hc = (uint16_t *)(s.rec + d.stride);
    const int32_t H = s.rec[BR_H];
    for (int32_t h = threadIdx.x; h < H; h += blockDim.x) {
        const int32_t b0 = s.rec[BR_HDR + h], b1 = min(s.rec[BR_HDR + h + 1], lim);
        for (int32_t k = b0; k < b1; k++) hc[k] = (uint16_t)h;
    }
    __syncthreads();
    for (int32_t k = threadIdx.x; k < lim; k += blockDim.x) {
        const int32_t h = hc[k];
        const int32_t g = s.rec[br_sbeg(d) + h] + (k - s.rec[BR_HDR + h]);
        const double4 p = at32(pos, g);
        if (shifted) {
            const uint32_t c = (uint32_t)s.rec[br_himg(d) + h];
            s.xyz[3 * k] = p.x - image_shift(c, 1u, Lx);
            s.xyz[3 * k + 1] = p.y - image_shift(c, 4u, Ly);
            s.xyz[3 * k + 2] = p.z - image_shift(c, 16u, Lz);
        } else {
            s.xyz[3 * k] = p.x;
            s.xyz[3 * k + 1] = p.y;
            s.xyz[3 * k + 2] = p.z;
        }
        if (s.j != nullptr) s.j[k] = g;
        if (extra0 != nullptr) s.ex[k] = at32(extra0, g);
        if (extra1 != nullptr) s.ex[s.cap + k] = at32(extra1, g);
        if (vec != nullptr) {
            const double4 u = at32(vec, g);
            double *e = s.ex + (size_t)vec_at * s.cap + k;
            e[0] = u.x;
            e[s.cap] = u.y;
            e[2 * (size_t)s.cap] = u.z;
        }
    }
    __syncthreads();
}

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

// sqrt(x) in binary64 for a pair's squared distance (x positive and normal;
// x = 0, which only dummy slots see, gives NaN, which their masks discard):
// the hardware reciprocal square root y, then one coupled Newton step on
// g = x y and h = y / 2 and one residual correction of g (within about an
// ulp, without the scaling of the general square root for tiny, huge and
// special arguments)
__device__ __forceinline__ double sqrt_pair(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    return fma(d, h, g);
}

// Position of candidate k.  STAGED = true: the whole halo is in LDS (pure LDS
// reads); false: candidates past the staged part come from global memory.  The
// two are separate instantiations chosen once per brick, so the common path
// never merges LDS and global addresses into flat loads.
template <bool STAGED>
__device__ __forceinline__ void candidate_pos(const Stage &s, const BrickDims &d, int32_t k,
                                              const double4 *pos, double &x, double &y, double &z)
{
    if (STAGED || k < s.cap) {
        const double *q = s.xyz + 3 * k;
        x = q[0];
        y = q[1];
        z = q[2];
    } else {
        const double4 p = pos[candidate_index(s, d, k)];
        x = p.x;
        y = p.y;
        z = p.z;
    }
}

template <bool STAGED>
__device__ __forceinline__ int32_t candidate_j(const Stage &s, const BrickDims &d, int32_t k)
{
    if (STAGED || k < s.cap) return s.j[k];
    return candidate_index(s, d, k);
}

// Four list entries: the four positions first, then the four pairs.  Slots
// at or past `rem` are called with ok = false and candidate 0 (a valid dummy).
template <bool STAGED, bool IMG, typename Body>
__device__ __forceinline__ void walk_four(const Stage &s, const BrickDims &d, const double4 *pos,
                                          const uint32_t es[4], int32_t rem, const double4 &xi,
                                          double Lx, double Ly, double Lz, Body &body)
{
    double px[4], py[4], pz[4];
    _Pragma("unroll")
    for (int u = 0; u < 4; u++)
        candidate_pos<STAGED>(s, d, (int32_t)(IMG ? ((u < rem ? es[u] : 0u) & MD_IDX_MASK) : (u < rem ? es[u] : 0u)),
                              pos, px[u], py[u], pz[u]);
    _Pragma("unroll")
    for (int u = 0; u < 4; u++) {
        const bool ok = u < rem;
        const uint32_t en = ok ? es[u] : 0u;
        const int32_t k = (int32_t)(IMG ? en & MD_IDX_MASK : en);
        double dx = xi.x - px[u], dy = xi.y - py[u], dz = xi.z - pz[u];
        if (IMG) {
            const uint32_t c = en >> MD_IDX_BITS;
            dx = dx + image_shift(c, 1u, Lx);
            dy = dy + image_shift(c, 4u, Ly);
            dz = dz + image_shift(c, 16u, Lz);
        }
        // fused: one rounding fewer than the list build's r2 (whose pair
        // sets must equal the oracle's); here r2 only feeds the pair
        // arithmetic and a cutoff test
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        body(ok, k, dx, dy, dz, r2);
    }
}

// Walks the list of one atom one 16-byte group at a time, with the next two
// groups in flight, and calls body(ok, k, dx, dy, dz, r2) for every slot; slots
// past the list's end come with ok = false and a valid dummy candidate.  IMG =
// false (a brick staged through its cell images) reads the narrow layout:
// 16-bit entries, eight per group, half the bytes of the 32-bit one.
template <bool STAGED, bool IMG, bool UNROLL = false, typename Body>
__device__ __forceinline__ void walk_list(const Stage &s, const BrickDims &d, const double4 *pos,
                                          const uint32_t *nbr, int64_t i, int32_t M, int32_t mm,
                                          const double4 &xi, double Lx, double Ly, double Lz,
                                          Body &&body)
{
    const uint4 *row = reinterpret_cast<const uint4 *>(nbr) + (((i >> 6) * (int64_t)(M >> 2)) << 6) + (i & 63);
    constexpr int PER = IMG ? 4 : 8;
    const int32_t nq = (mm + PER - 1) / PER;
    uint4 n1 = make_uint4(0u, 0u, 0u, 0u), n2 = n1;
    if (nq > 0) n1 = row[0];
    if (nq > 1) n2 = row[64];
    for (int32_t q = 0; q < nq; q++) {
        const uint4 ev = n1;
        n1 = n2;
        if (q + 2 < nq) n2 = row[(int64_t)(q + 2) << 6];
        const int32_t rem = mm - PER * q;
        if (IMG) {
            const uint32_t es[4] = {ev.x, ev.y, ev.z, ev.w};
            walk_four<STAGED, IMG>(s, d, pos, es, rem, xi, Lx, Ly, Lz, body);
        } else if (UNROLL) {
            // both halves inlined: the second half's LDS reads may be issued
            // ahead of the first half's arithmetic (more registers live)
            const uint32_t lo[4] = {ev.x & 0xffffu, ev.x >> 16, ev.y & 0xffffu, ev.y >> 16};
            const uint32_t hi[4] = {ev.z & 0xffffu, ev.z >> 16, ev.w & 0xffffu, ev.w >> 16};
            walk_four<STAGED, IMG>(s, d, pos, lo, rem, xi, Lx, Ly, Lz, body);
            if (rem > 4) walk_four<STAGED, IMG>(s, d, pos, hi, rem - 4, xi, Lx, Ly, Lz, body);
        } else {
            // one copy of the pair code for both halves (as many registers
            // live as in the 32-bit walk)
            _Pragma("unroll 1")
            for (int h = 0; h < 2 && rem > 4 * h; h++) {
                const uint32_t w0 = h != 0 ? ev.z : ev.x, w1 = h != 0 ? ev.w : ev.y;
                const uint32_t es[4] = {w0 & 0xffffu, w0 >> 16, w1 & 0xffffu, w1 >> 16};
                walk_four<STAGED, IMG>(s, d, pos, es, rem - 4 * h, xi, Lx, Ly, Lz, body);
            }
        }
    }
}

// runs the block once per (STAGED, IMG) combination (both uniform per brick):
// IMG = false exactly for the bricks whose staging applied the cell images
// (BR_SHIFT = 1, which implies a wholly staged halo)
#define STAGE_IMG_SPLIT(ALL_STAGED, HAS_IMG, ...)                                         \
    if (ALL_STAGED) {                                                                     \
        constexpr bool STAGED = true;                                                     \
        if (HAS_IMG) {                                                                    \
            constexpr bool IMG = true;                                                    \
            __VA_ARGS__                                                                   \
        } else {                                                                          \
            constexpr bool IMG = false;                                                   \
            __VA_ARGS__                                                                   \
        }                                                                                 \
    } else {                                                                              \
        constexpr bool STAGED = false;                                                    \
        constexpr bool IMG = true;                                                        \
        __VA_ARGS__                                                                       \
    }

// ---------------------------------------------------------------- brick-task loop
// Next brick for this workgroup (-1 when none is left): the range of its XCD
// (workgroups are dispatched round-robin over the eight XCDs, so block b runs
// on XCD b % 8) first, so that an XCD's L2 works on one compact region, then
// the other ranges, so that dense regions of an inhomogeneous system are
// shared out.  Block-wide; starts and ends with a barrier.
__device__ __forceinline__ int64_t next_brick(TaskQueue *q, int64_t nb, int32_t *slot)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const int x = blockIdx.x & 7;
        const int64_t per = (nb + 7) >> 3;
        int64_t b = -1;
        for (int d = 0; d < 8 && b < 0; d++) {
            const int y = (x + d) & 7;
            const int64_t lo = y * per, hi = lo + per < nb ? lo + per : nb;
            if (lo >= hi) continue;
            const uint32_t seen = __hip_atomic_load(&q->next[32 * y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int64_t)seen >= hi - lo) continue;
            const uint32_t t = atomicAdd(&q->next[32 * y], 1u);
            if (lo + (int64_t)t < hi) b = lo + t;
        }
        *slot = (int32_t)b;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);
}

// End of a queue-driven force launch: the last workgroup resets the queue.
// No fence: every workgroup's last take has returned before it counts itself
// done, and the launch publishes nothing else through the queue.
__device__ __forceinline__ void queue_done(TaskQueue *q)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = atomicAdd(&q->done, 1u);
        if (prev == gridDim.x - 1) {
            for (int k = 0; k < 8; k++) __hip_atomic_store(&q->next[32 * k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&q->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// End of a queue-driven launch: returns true (in every thread) in the last
// workgroup to finish, which has reset the queue for the next launch.
__device__ __forceinline__ bool tasks_done(TaskQueue *q)
{
    __shared__ int last_;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&q->done, 1u);
        last_ = prev == gridDim.x - 1 ? 1 : 0;
        if (last_) {
            for (int k = 0; k < 8; k++) __hip_atomic_store(&q->next[32 * k], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&q->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (last_) __threadfence();
    return last_ != 0;
}

// first index b in [0, n] with w[b] >= t (w non-decreasing over [0, n], and
// w[n] >= t); called by all 64 lanes of a wavefront, which probe 64 points per
// round, so a prefix of up to 64^3 entries takes at most four dependent loads
__device__ __forceinline__ int64_t lower_bound_wave(const int64_t *w, int64_t n, int64_t t)
{
    const int lane = threadIdx.x & 63;
    int64_t lo = 0, hi = n;        // the answer lies in [lo, hi]
    while (hi - lo > 63) {
        const int64_t step = (hi - lo + 63) >> 6;
        const int64_t p = lo + (int64_t)(lane + 1) * step;      // lane 63 probes >= hi
        const bool ge = p >= hi || w[p] >= t;
        const int first = __ffsll((long long)__ballot(ge)) - 1;
        const int64_t nlo = first > 0 ? lo + (int64_t)first * step + 1 : lo;
        const int64_t nhi = lo + (int64_t)(first + 1) * step < hi ? lo + (int64_t)(first + 1) * step : hi;
        lo = nlo;
        hi = nhi;
    }
    const int64_t p = lo + lane;
    const bool ge = p >= hi || w[p] >= t;
    return lo + (__ffsll((long long)__ballot(ge)) - 1);
}

// This workgroup's bricks: the cost prefix (from the list build) is cut into
// eight parts of equal cost, one per XCD (block g runs on XCD g % 8), and the
// workgroups of an XCD take the bricks of its part in turn (slot s takes
// bricks first + s, first + s + G/8, ...), so the bricks in flight on an XCD
// at any time are neighbours that share their halos in its L2, and every XCD
// carries the same load even where the system is inhomogeneous.
struct BrickRange {
    int64_t first, end, stride;
};

__device__ __forceinline__ BrickRange balanced_bricks(const int64_t *w, int64_t nb)
{
    const int64_t G = gridDim.x;
    BrickRange r;
    if (G % 8 != 0) {
        r.first = blockIdx.x;
        r.end = nb;
        r.stride = G;
        return r;
    }
    const int64_t x = blockIdx.x & 7, W = w[nb];
    const int64_t lo = lower_bound_wave(w, nb, W * x / 8);
    r.end = x == 7 ? nb : lower_bound_wave(w, nb, W * (x + 1) / 8);
    r.first = lo + (blockIdx.x >> 3);
    r.stride = G >> 3;
    return r;
}

// Brick-task loop of the force and adjoint kernels: the workgroup walks its
// bricks -- its static cost-balanced ranges (balanced_bricks), or, with a.dyn,
// bricks taken one at a time from the queue (next_brick: its XCD's share
// first, then the others') -- loads each record and stages the halo, then its
// lanes take the brick's atoms (la = a0 + thread) in rounds of blockDim.x.
// Defines for the body: natoms, rep_r, Lx/Ly/Lz, all_staged, has_img, valid,
// la, i (sorted index), mm (list length, capped at M).
#define BRICK_TASK_BEGIN(ST, POS, EXTRA0, EXTRA1) BRICK_TASK_BEGIN_V(ST, POS, EXTRA0, EXTRA1, nullptr, 0)
#define BRICK_TASK_BEGIN_V(ST, POS, EXTRA0, EXTRA1, VEC, VEC_AT)                           \
    const bool dyn_ = a.dyn != 0;                                                         \
    const BrickRange br_ = dyn_ ? BrickRange{0, a.B, 1} : balanced_bricks(a.bwork, a.B);  \
    __shared__ int32_t qslot_;                                                            \
    for (int64_t b_ = dyn_ ? next_brick(a.ftq, a.B, &qslot_) : br_.first; b_ >= 0 && b_ < br_.end; \
         b_ = dyn_ ? next_brick(a.ftq, a.B, &qslot_) : b_ + br_.stride) {                 \
        const int32_t *grec_ = a.brec + b_ * (int64_t)a.bd.stride;                        \
        const int32_t natoms = __builtin_amdgcn_readfirstlane(grec_[BR_ATOMS]);           \
        if (natoms == 0) continue;                                                        \
        __syncthreads();                                                                  \
        brick_load(ST, a.bd, grec_, a.reps, POS, EXTRA0, EXTRA1, VEC, VEC_AT);            \
        const int32_t rep_r = ST.rec[BR_REP];                                             \
        const bool has_img = ST.rec[BR_SHIFT] == 0;                                       \
        const bool all_staged = ST.rec[BR_TOTAL] <= ST.cap;                               \
        const RepDesc &rep_ = a.reps[rep_r];                                              \
        const double Lx = rep_.L[0], Ly = rep_.L[1], Lz = rep_.L[2];                      \
        for (int32_t a0_ = 0; a0_ < natoms; a0_ += (int32_t)blockDim.x) {                 \
            const int32_t la = a0_ + (int32_t)threadIdx.x;                                \
            const bool valid = la < natoms;                                               \
            const int64_t i = valid ? brick_atom(ST, a.bd, la) : 0;                       \
            const int32_t mm = valid ? min(a.cnt[i], a.M) : 0;

#define BRICK_TASK_END                                                                    \
        }                                                                                 \
    }                                                                                     \
    if (dyn_) queue_done(a.ftq);

#endif
