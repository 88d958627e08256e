// md_cells.hip -- linked cells (Sec. II.A): wrap, bin, scan, stable sort by cell.
//
// The cell of an atom follows the pinned binning rule: wrap x -> x - L floor(x/L)
// (x >= L -> x - L, x < 0 -> 0), cell coordinate min(floor(x * n_c / L), n_c - 1),
// cell index x fastest.  Within a cell atoms are ordered by ascending user index,
// so the sorted order -- and every sum taken in it -- is deterministic.
//
// Kernels run on a fixed persistent grid with grid-stride loops.  Each takes a
// predicate word: inside the integration loop it is the device-side rebuild
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

__global__ void k_bin(const int32_t *__restrict__ pred, int64_t n, const RepDesc *__restrict__ reps,
                      const int32_t *__restrict__ rep_of, double4 *__restrict__ pos,
                      int32_t *__restrict__ cell_of, int32_t *__restrict__ slot,
                      int32_t *__restrict__ count)
{
    if (*pred == 0) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const RepDesc &r = reps[rep_of[i]];
        double4 p = pos[i];
        p.x = wrap1(p.x, r.L[0]);
        p.y = wrap1(p.y, r.L[1]);
        p.z = wrap1(p.z, r.L[2]);
        pos[i] = p;
        int32_t cx = cell_coord(p.x, r.nc[0], r.L[0]);
        int32_t cy = cell_coord(p.y, r.nc[1], r.L[1]);
        int32_t cz = cell_coord(p.z, r.nc[2], r.L[2]);
        int64_t c = r.cell_off + cx + (int64_t)r.nc[0] * (cy + (int64_t)r.nc[1] * cz);
        cell_of[i] = (int32_t)c;
        slot[i] = atomicAdd(&count[c], 1);
    }
}

// Exclusive scan of the cell counts by one workgroup of 1024 threads; each
// thread owns a contiguous chunk.  The counts are cleared for the next build.
__global__ __launch_bounds__(1024) void k_scan(const int32_t *__restrict__ pred, int64_t C,
                                               int32_t *__restrict__ count,
                                               int32_t *__restrict__ start, DevCtl *ctl)
{
    if (*pred == 0) return;
    __shared__ int32_t wsum[16];
    __shared__ int32_t wmax[16];
    const int t = threadIdx.x;
    const int64_t chunk = (C + 1023) / 1024;
    const int64_t lo = t * chunk < C ? t * chunk : C;
    const int64_t hi = lo + chunk < C ? lo + chunk : C;
    int32_t s = 0, mx = 0;
    for (int64_t k = lo; k < hi; k++) {
        int32_t v = count[k];
        s += v;
        mx = v > mx ? v : mx;
    }
    // inclusive scan within the wave, then across the 16 waves
    const int lane = t & 63, wv = t >> 6;
    int32_t inc = s;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    for (int o = 32; o > 0; o >>= 1) {
        int32_t y = __shfl_xor(mx, o, 64);
        mx = y > mx ? y : mx;
    }
    if (lane == 63) wsum[wv] = inc;
    if (lane == 0) wmax[wv] = mx;
    __syncthreads();
    if (t == 0) {
        int32_t run = 0, m = 0;
        for (int w = 0; w < 16; w++) {
            int32_t v = wsum[w];
            wsum[w] = run;
            run += v;
            m = wmax[w] > m ? wmax[w] : m;
        }
        start[C] = run;
        ctl->max_cell = m;
        ctl->nrebuild += 1;
    }
    __syncthreads();
    int32_t run = wsum[wv] + inc - s;
    for (int64_t k = lo; k < hi; k++) {
        int32_t v = count[k];
        start[k] = run;
        run += v;
        count[k] = 0;
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

// One wavefront per cell: rank the cell's atoms by user index and move them
// (positions, velocities, ids) to their final slots in the output buffers.
__global__ __launch_bounds__(256) void k_sort_cells(
    const int32_t *__restrict__ pred, int64_t C, const int32_t *__restrict__ start,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ id,
    const double4 *__restrict__ pos, const double *__restrict__ vel, int64_t n,
    double4 *__restrict__ pos_out, double *__restrict__ vel_out, int32_t *__restrict__ id_out)
{
    if (*pred == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t c = wave; c < C; c += nwaves) {
        const int32_t s = start[c];
        const int32_t m = start[c + 1] - s;
        if (m <= 64) {
            int32_t old = 0, key = 0x7fffffff;
            if (lane < m) {
                old = perm[s + lane];
                key = id[old];
            }
            int32_t rank = 0;
            for (int l = 0; l < m; l++) {
                int32_t kl = __shfl(key, l, 64);
                rank += kl < key ? 1 : 0;
            }
            if (lane < m) {
                const int64_t d = s + rank;
                pos_out[d] = pos[old];
                if (vel != nullptr) {
                    vel_out[d] = vel[old];
                    vel_out[n + d] = vel[n + old];
                    vel_out[2 * n + d] = vel[2 * n + old];
                }
                id_out[d] = key;
            }
        } else {
            for (int32_t b = 0; b < m; b += 64) {
                const int32_t k = b + lane;
                int32_t old = 0, key = 0;
                if (k < m) {
                    old = perm[s + k];
                    key = id[old];
                }
                int32_t rank = 0;
                for (int32_t l = 0; l < m; l++) rank += id[perm[s + l]] < key ? 1 : 0;
                if (k < m) {
                    const int64_t d = s + rank;
                    pos_out[d] = pos[old];
                    if (vel != nullptr) {
                        vel_out[d] = vel[old];
                        vel_out[n + d] = vel[n + old];
                        vel_out[2 * n + d] = vel[2 * n + old];
                    }
                    id_out[d] = key;
                }
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
                int32_t *slot, int32_t *count)
{
    (void)R;
    hipLaunchKernelGGL(k_bin, dim3(grid), dim3(256), 0, s, pred, n, reps, rep_of, pos, cell_of,
                       slot, count);
}

void launch_scan(hipStream_t s, const int32_t *pred, int64_t C, int32_t *count, int32_t *start,
                 DevCtl *ctl)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, pred, C, count, start, ctl);
}

void launch_scatter(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                    const int32_t *cell_of, const int32_t *slot, const int32_t *start,
                    int32_t *perm)
{
    hipLaunchKernelGGL(k_scatter, dim3(grid), dim3(256), 0, s, pred, n, cell_of, slot, start, perm);
}

void launch_sort_cells(hipStream_t s, int grid, const int32_t *pred, int64_t C,
                       const int32_t *start, const int32_t *perm, const int32_t *id,
                       const double4 *pos, const double *vel, int64_t n, double4 *pos_out,
                       double *vel_out, int32_t *id_out)
{
    hipLaunchKernelGGL(k_sort_cells, dim3(grid), dim3(256), 0, s, pred, C, start, perm, id, pos,
                       vel, n, pos_out, vel_out, id_out);
}

void launch_copy_back(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                      const double4 *pos_t, const double *vel_t, const int32_t *id_t,
                      double4 *pos, double *vel, int32_t *id, double4 *xref)
{
    hipLaunchKernelGGL(k_copy_back, dim3(grid), dim3(256), 0, s, pred, n, pos_t, vel_t, id_t, pos,
                       vel, id, xref);
}
