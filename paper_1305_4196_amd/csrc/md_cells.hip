// md_cells.hip -- linked cells (Sec. II.A): wrap, bin, scan, stable sort by cell.
//
// The cell of an atom follows the pinned binning rule: wrap x -> x - L floor(x/L)
// (x >= L -> x - L, x < 0 -> 0), cell coordinate min(floor(x * n_c / L), n_c - 1),
// cell index x fastest.  Within a cell atoms are ordered by ascending user index,
// so the sorted order -- and every sum taken in it -- is deterministic.
//
// Kernels run on a fixed persistent grid with grid-stride loops (the count scan
// on one workgroup per chunk of cells).  Each takes a predicate word: inside the integration loop it is the device-side rebuild
// request, so an unneeded rebuild costs only an early exit and no host sync.
#include "md_internal.h"

namespace {

__device__ __forceinline__ double wrap1(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L) w = w - L;
    if (w < 0.0) w = 0.0;
    return w;
}

__device__ __forceinline__ int32_t cell_coord(double x, int32_t nc, double L)
{
    int32_t c = (int32_t)floor(x * (double)nc / L);
    if (c > nc - 1) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

__global__ void k_load_user(int64_t n, const double *__restrict__ pos_user,
                            const double *__restrict__ vel_user, double4 *__restrict__ pos,
                            double *__restrict__ vel, int32_t *__restrict__ id)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        pos[i] = make_double4(pos_user[i], pos_user[n + i], pos_user[2 * n + i], 0.0);
        if (vel_user != nullptr) {
            vel[i] = vel_user[i];
            vel[n + i] = vel_user[n + i];
            vel[2 * n + i] = vel_user[2 * n + i];
        }
        id[i] = (int32_t)i;
    }
}

// Atoms arrive in the previous cell order, so neighbouring lanes usually fall
// into the same cell: each run of equal cells among consecutive lanes of a
// wavefront takes its slots with one atomic add by the run's first lane.
//
// A non-finite position (a run that blew up, or bad input) raises
// MD_FLAG_NONFINITE and puts the atom in cell i mod (its replica's cells): such
// atoms stay spread over the cells instead of all falling into cell 0, where
// the list build would test each of them against all the others; their tests
// fail (NaN compares false), so they get no partners.
__global__ void k_bin(const int32_t *__restrict__ pred, int64_t n, const RepDesc *__restrict__ reps,
                      const int32_t *__restrict__ rep_of, double4 *__restrict__ pos,
                      int32_t *__restrict__ cell_of, int32_t *__restrict__ slot,
                      int32_t *__restrict__ count, int32_t *__restrict__ err)
{
    if (*pred == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < n;
        int32_t c = -1;
        if (valid) {
            const RepDesc &r = reps[rep_of[i]];
            const double4 q = pos[i];
            double4 p = q;
            p.x = wrap1(q.x, r.L[0]);
            p.y = wrap1(q.y, r.L[1]);
            p.z = wrap1(q.z, r.L[2]);
            // stored only where wrapping changed a bit (most atoms are inside the box)
            if (__double_as_longlong(p.x) != __double_as_longlong(q.x) ||
                __double_as_longlong(p.y) != __double_as_longlong(q.y) ||
                __double_as_longlong(p.z) != __double_as_longlong(q.z))
                pos[i] = p;
            if (isfinite(p.x) && isfinite(p.y) && isfinite(p.z)) {
                const int32_t cx = cell_coord(p.x, r.nc[0], r.L[0]);
                const int32_t cy = cell_coord(p.y, r.nc[1], r.L[1]);
                const int32_t cz = cell_coord(p.z, r.nc[2], r.L[2]);
                c = (int32_t)(r.cell_off + cx + (int64_t)r.nc[0] * (cy + (int64_t)r.nc[1] * cz));
            } else {
                atomicOr(err, MD_FLAG_NONFINITE);
                c = (int32_t)(r.cell_off + i % ((int64_t)r.nc[0] * r.nc[1] * r.nc[2]));
            }
            cell_of[i] = c;
        }
        const int32_t prev = __shfl_up(c, 1, 64);
        const bool head = valid && (lane == 0 || prev != c);
        const uint64_t heads = __ballot(head);
        const uint64_t live = __ballot(valid);
        // first lane of this lane's run, and the first lane after it
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        const int leader = 63 - __clzll(heads & upto);
        const uint64_t after = lane == 63 ? 0ull : (heads & ~upto);
        const int nlive = __popcll(live);
        int32_t b = 0;
        if (head) {
            const int next = after != 0 ? __ffsll((long long)after) - 1 : nlive;
            b = atomicAdd(&count[c], next - lane);
        }
        b = __shfl(b, leader, 64);
        if (valid) slot[i] = b + (lane - leader);
    }
}

// Exclusive scan of the cell counts.  The counts are left in place: k_sort_cells,
// which visits every cell, clears them for the next build.
constexpr int SCAN_CHUNK = 8192;           // cells per chunk: 8 per thread of 1024
constexpr int SCAN_MAX_CHUNKS = 64;        // chunks scanned by k_scan_chunks

// Sum over the workgroup of 1024 threads (every thread gets it).
__device__ __forceinline__ int32_t block_sum_1024(int32_t v, int32_t *wsum)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) wsum[wv] = v;
    __syncthreads();
    int32_t t = 0;
    for (int w = 0; w < 16; w++) t += wsum[w];
    return t;
}

// One chunk of SCAN_CHUNK cells from c0 on, given the sum of the counts before
// it: each thread takes 8 consecutive counts, the threads' totals are scanned
// across the workgroup; returns the chunk's total.
__device__ __forceinline__ int32_t scan_chunk(int64_t C, int64_t c0, int32_t carry,
                                              const int32_t *__restrict__ count,
                                              int32_t *__restrict__ start, int32_t *wsum)
{
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6;
    const int64_t k0 = c0 + 8 * (int64_t)t;
    int32_t v[8];
    if (k0 + 8 <= C) {
        const int4 a = reinterpret_cast<const int4 *>(count + k0)[0];
        const int4 b = reinterpret_cast<const int4 *>(count + k0)[1];
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
        for (int q = 0; q < 8; q++) v[q] = k0 + q < C ? count[k0 + q] : 0;
    }
    int32_t s = 0;
    for (int q = 0; q < 8; q++) s += v[q];
    int32_t inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < 16; w++) {
        const int32_t ws = wsum[w];
        before += w < wv ? ws : 0;
        total += ws;
    }
    int32_t run = carry + before + inc - s;
    int32_t o[8];
    for (int q = 0; q < 8; q++) {
        o[q] = run;
        run += v[q];
    }
    if (k0 + 8 <= C) {
        reinterpret_cast<int4 *>(start + k0)[0] = make_int4(o[0], o[1], o[2], o[3]);
        reinterpret_cast<int4 *>(start + k0)[1] = make_int4(o[4], o[5], o[6], o[7]);
    } else {
        for (int q = 0; q < 8; q++)
            if (k0 + q < C) start[k0 + q] = o[q];
    }
    return total;
}

// Up to SCAN_MAX_CHUNKS chunks, one workgroup each: a workgroup first sums the
// counts of every chunk before its own (read from L2; no workgroup waits for
// another), so the chunks are scanned in parallel rather than one after the
// other by one CU, whose bandwidth to L2 bounds a single-workgroup scan.
__global__ __launch_bounds__(1024) void k_scan_chunks(const int32_t *__restrict__ pred, int64_t C,
                                                      const int32_t *__restrict__ count,
                                                      int32_t *__restrict__ start, DevCtl *ctl)
{
    if (*pred == 0) return;
    __shared__ int32_t wsum[16];
    const int64_t c0 = (int64_t)blockIdx.x * SCAN_CHUNK;
    int32_t part = 0;
    for (int64_t k = 4 * (int64_t)threadIdx.x; k < c0; k += 4 * 1024) {
        const int4 a = *reinterpret_cast<const int4 *>(count + k);
        part += (a.x + a.y) + (a.z + a.w);
    }
    const int32_t carry = block_sum_1024(part, wsum);
    const int32_t total = scan_chunk(C, c0, carry, count, start, wsum);
    if (threadIdx.x == 0) {
        if (blockIdx.x == gridDim.x - 1) start[C] = carry + total;
        if (blockIdx.x == 0) ctl->nrebuild += 1;
    }
}

// More chunks: one workgroup takes them in order, a carry linking them.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ pred, int64_t C,
                                               const int32_t *__restrict__ count,
                                               int32_t *__restrict__ start, DevCtl *ctl)
{
    if (*pred == 0) return;
    __shared__ int32_t wsum[16];
    int32_t carry = 0;
    for (int64_t c0 = 0; c0 < C; c0 += SCAN_CHUNK) carry += scan_chunk(C, c0, carry, count, start, wsum);
    if (threadIdx.x == 0) {
        start[C] = carry;
        ctl->nrebuild += 1;
    }
}

__global__ void k_scatter(const int32_t *__restrict__ pred, int64_t n,
                          const int32_t *__restrict__ cell_of, const int32_t *__restrict__ slot,
                          const int32_t *__restrict__ start, int32_t *__restrict__ perm)
{
    if (*pred == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        perm[start[cell_of[i]] + slot[i]] = (int32_t)i;
}

// Moves atom `old` of a cell to its slot d (positions, velocities, id).
__device__ __forceinline__ void move_atom(int32_t old, int64_t d, int32_t key, const double4 *__restrict__ pos,
                                          const double *__restrict__ vel, int64_t n,
                                          double4 *__restrict__ pos_out, double *__restrict__ vel_out,
                                          int32_t *__restrict__ id_out)
{
    pos_out[d] = pos[old];
    if (vel != nullptr) {
        vel_out[d] = vel[old];
        vel_out[n + d] = vel[n + old];
        vel_out[2 * n + d] = vel[2 * n + old];
    }
    id_out[d] = key;
}

// Cells of at most G atoms, 64 / G of them at once: lane g0 + l (g0 the first
// lane of its group of G) holds atom l of its cell (start s, m atoms), whose
// rank is the number of the cell's atoms with a smaller user index; mmax is
// the largest m of the wavefront's cells (lanes past their cell hold the
// largest key, which counts for no atom).
__device__ __forceinline__ void sort_groups(int G, int32_t s, int32_t m, int32_t mmax,
                                            const int32_t *__restrict__ perm, const int32_t *__restrict__ id,
                                            const double4 *__restrict__ pos, const double *__restrict__ vel,
                                            int64_t n, double4 *__restrict__ pos_out, double *__restrict__ vel_out,
                                            int32_t *__restrict__ id_out)
{
    const int lane = threadIdx.x & 63;
    const int g0 = lane & ~(G - 1), l = lane & (G - 1);
    int32_t old = 0, key = 0x7fffffff;
    if (l < m) {
        old = perm[s + l];
        key = id[old];
    }
    int32_t rank = 0;
    for (int q = 0; q < mmax; q++) {
        const int32_t kq = __shfl(key, g0 + q, 64);
        rank += kq < key ? 1 : 0;
    }
    if (l < m) move_atom(old, (int64_t)s + rank, key, pos, vel, n, pos_out, vel_out, id_out);
}

// A cell of more than 64 atoms, 64 at a time (ranks counted over the whole cell).
__device__ __forceinline__ void sort_large(int32_t s, int32_t m, const int32_t *__restrict__ perm,
                                           const int32_t *__restrict__ id, const double4 *__restrict__ pos,
                                           const double *__restrict__ vel, int64_t n,
                                           double4 *__restrict__ pos_out, double *__restrict__ vel_out,
                                           int32_t *__restrict__ id_out)
{
    const int lane = threadIdx.x & 63;
    for (int32_t b = 0; b < m; b += 64) {
        const int32_t k = b + lane;
        int32_t old = 0, key = 0;
        if (k < m) {
            old = perm[s + k];
            key = id[old];
        }
        int32_t rank = 0;
        for (int32_t l = 0; l < m; l++) rank += id[perm[s + l]] < key ? 1 : 0;
        if (k < m) move_atom(old, (int64_t)s + rank, key, pos, vel, n, pos_out, vel_out, id_out);
    }
}

// Ranks each cell's atoms by user index and moves them (positions, velocities,
// ids) to their final slots in the output buffers, and clears the cell counts
// for the next build.  A wavefront takes four consecutive cells at a time:
// all four together in groups of 16 lanes when none holds more than 16 atoms,
// else each pair together in groups of 32 when both fit, else one cell at a
// time (the chain of dependent loads per cell, not the lanes, sets the time).
__global__ __launch_bounds__(256) void k_sort_cells(
    const int32_t *__restrict__ pred, int64_t C, const int32_t *__restrict__ start,
    int32_t *__restrict__ count,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ id,
    const double4 *__restrict__ pos, const double *__restrict__ vel, int64_t n,
    double4 *__restrict__ pos_out, double *__restrict__ vel_out, int32_t *__restrict__ id_out)
{
    if (*pred == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c0 = 4 * wave; c0 < C; c0 += 4 * nwaves) {
        const int32_t nc = (int32_t)(C - c0 < 4 ? C - c0 : 4);
        // starts of the (up to) four cells and the end of the last, lanes 0..nc
        const int32_t st = lane <= nc ? start[c0 + lane] : 0;
        if (lane < nc) count[c0 + lane] = 0;
        int32_t sk[4], mk[4];
        for (int k = 0; k < 4; k++) {
            sk[k] = __shfl(st, k, 64);
            mk[k] = k < nc ? __shfl(st, k + 1, 64) - sk[k] : 0;
        }
        const int32_t m01 = max(mk[0], mk[1]), m23 = max(mk[2], mk[3]);
        if (max(m01, m23) <= 16) {
            const int k = lane >> 4;
            const int32_t s = k == 0 ? sk[0] : (k == 1 ? sk[1] : (k == 2 ? sk[2] : sk[3]));
            const int32_t m = k == 0 ? mk[0] : (k == 1 ? mk[1] : (k == 2 ? mk[2] : mk[3]));
            sort_groups(16, s, m, max(m01, m23), perm, id, pos, vel, n, pos_out, vel_out, id_out);
            continue;
        }
        for (int p = 0; p < 2; p++) {
            const int32_t sa = sk[2 * p], ma = mk[2 * p], sb = sk[2 * p + 1], mb = mk[2 * p + 1];
            if (max(ma, mb) <= 32) {
                const bool hi = lane >= 32;
                sort_groups(32, hi ? sb : sa, hi ? mb : ma, max(ma, mb), perm, id, pos, vel, n, pos_out,
                            vel_out, id_out);
                continue;
            }
            for (int h = 0; h < 2; h++) {
                const int32_t s = h ? sb : sa, m = h ? mb : ma;
                if (m <= 64) sort_groups(64, s, m, m, perm, id, pos, vel, n, pos_out, vel_out, id_out);
                else sort_large(s, m, perm, id, pos, vel, n, pos_out, vel_out, id_out);
            }
        }
    }
}

__global__ void k_copy_back(const int32_t *__restrict__ pred, int64_t n,
                            const double4 *__restrict__ pos_t, const double *__restrict__ vel_t,
                            const int32_t *__restrict__ id_t, double4 *__restrict__ pos,
                            double *__restrict__ vel, int32_t *__restrict__ id,
                            double4 *__restrict__ xref)
{
    if (*pred == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double4 p = pos_t[i];
        pos[i] = p;
        xref[i] = p;
        if (vel != nullptr) {
            vel[i] = vel_t[i];
            vel[n + i] = vel_t[n + i];
            vel[2 * n + i] = vel_t[2 * n + i];
        }
        id[i] = id_t[i];
    }
}

} // namespace

void launch_load_user(hipStream_t s, int grid, int64_t n, const double *pos_user,
                      const double *vel_user, double4 *pos, double *vel, int32_t *id)
{
    hipLaunchKernelGGL(k_load_user, dim3(grid), dim3(256), 0, s, n, pos_user, vel_user, pos, vel, id);
}

void launch_bin(hipStream_t s, int grid, const int32_t *pred, int64_t n, int32_t R,
                const RepDesc *reps, const int32_t *rep_of, double4 *pos, int32_t *cell_of,
                int32_t *slot, int32_t *count, int32_t *err)
{
    (void)R;
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(256), 0, s, pred, n, reps, rep_of, pos, cell_of,
                       slot, count, err);
}

void launch_scan(hipStream_t s, const int32_t *pred, int64_t C, int32_t *count, int32_t *start,
                 DevCtl *ctl)
{
    const int64_t chunks = (C + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (chunks <= SCAN_MAX_CHUNKS)
        hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)chunks), dim3(1024), 0, s, pred, C, count, start, ctl);
    else
        hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, pred, C, count, start, ctl);
}

void launch_scatter(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                    const int32_t *cell_of, const int32_t *slot, const int32_t *start,
                    int32_t *perm)
{
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, s, pred, n, cell_of, slot, start, perm);
}

void launch_sort_cells(hipStream_t s, int grid, const int32_t *pred, int64_t C,
                       const int32_t *start, int32_t *count, const int32_t *perm, const int32_t *id,
                       const double4 *pos, const double *vel, int64_t n, double4 *pos_out,
                       double *vel_out, int32_t *id_out)
{
    hipLaunchKernelGGL(k_sort_cells, dim3(grid), dim3(256), 0, s, pred, C, start, count, perm, id, pos,
                       vel, n, pos_out, vel_out, id_out);
}

void launch_copy_back(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                      const double4 *pos_t, const double *vel_t, const int32_t *id_t,
                      double4 *pos, double *vel, int32_t *id, double4 *xref)
{
    hipLaunchKernelGGL(k_copy_back, dim3(grid), dim3(256), 0, s, pred, n, pos_t, vel_t, id_t, pos,
                       vel, id, xref);
}
