// md_api.hip -- host side of the C ABI declared in include/md.h.
//
// The context owns all workspace; every entry point validates its arguments on
// the host, then enqueues kernels on the caller's stream.  Inside md_verlet_step
// the rebuild decision is taken on the device (a predicate word per step parity),
// so a run of n steps is one stream of launches with no host round trip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "md_brick.h"
#include "md_waves.h"

// Device memory of md_compute_forces_noalloc: every scratch buffer its kernels
// use (sorted forces, block partials, counters, brick queue, EAM densities and
// tables, per-atom energies) is carved out of this array, so the call allocates
// nothing.  Each device the library runs on holds one copy until the process
// ends; its address on a device comes from hipGetSymbolAddress (the array's name
// in host code is a host-side stand-in, never a device address).
#define MD_NOALLOC_BYTES (48ull << 20)
static __device__ __align__(256) unsigned char scratch[MD_NOALLOC_BYTES];

namespace {

__global__ void k_set_ctl(DevCtl *ctl, int reset_rebuild, int reset_count)
{
    if (threadIdx.x == 0) {
        if (reset_rebuild) {
            ctl->rebuild[0] = 0;
            ctl->rebuild[1] = 0;
        }
        if (reset_count) ctl->nrebuild = 0;
    }
}

__global__ void k_copy_int(const int32_t *src, int32_t *dst)
{
    if (threadIdx.x == 0) *dst = *src;
}

__global__ void k_pos_from_user(int64_t n, const RepDesc *__restrict__ reps,
                                const int32_t *__restrict__ rep_of, const int32_t *__restrict__ id,
                                const double *__restrict__ user, const double4 *__restrict__ xref,
                                double4 *__restrict__ pos)
{
    // positions continued from the build-time reference by the minimum image,
    // so that the image fixed with each list entry stays valid
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const RepDesc &r = reps[rep_of[i]];
        const int64_t u = id[i];
        const double4 x0 = xref[i];
        double d[3] = {user[u] - x0.x, user[n + u] - x0.y, user[2 * n + u] - x0.z};
        for (int c = 0; c < 3; c++) {
            if (d[c] > r.hL[c]) d[c] = d[c] - r.L[c];
            else if (d[c] < -r.hL[c]) d[c] = d[c] + r.L[c];
        }
        pos[i] = make_double4(x0.x + d[0], x0.y + d[1], x0.z + d[2], 0.0);
    }
}

template <typename T>
bool dalloc(T **p, size_t count)
{
    if (*p != nullptr) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    return hipMalloc((void **)p, sizeof(T) * count) == hipSuccess;
}

template <typename T>
void dfree(T *&p)
{
    if (p != nullptr) (void)hipFree(p);
    p = nullptr;
}

} // namespace

struct md_ctx {
    int device = 0;
    int64_t n = 0;
    int32_t R = 0;
    std::vector<int64_t> off;
    int n_cu = 256;
    int lds_max = 65536;   // LDS bytes a workgroup may use
    int wgpc = 8;      // most brick-task workgroups per CU
    std::string err;
    hipStream_t last = nullptr;

    // geometry
    bool have_cells = false;
    double rc = 0.0, skin = 0.0, rl = 0.0;
    std::vector<double> boxes;
    std::vector<RepDesc> reps_h;
    RepDesc *reps = nullptr;
    int64_t C = 0, C_alloc = 0;
    int32_t *rep_of = nullptr;

    // bricks of cells (one task each)
    int32_t bshape[3] = {0, 0, 0};   // requested brick shape (0: chosen from the cell occupancy)
    int32_t threads_req = 0;          // requested threads per task (0: chosen with the shape)
    int32_t threads = 256;            // threads per brick task
    bool bricks_valid = false;
    int64_t B = 0, brec_alloc = 0;
    BrickDims bd{0, 0, 0};
    int32_t *brec = nullptr;
    int32_t *bcost = nullptr;         // [B] brick costs of the last list build
    int64_t *bwork = nullptr;         // [B+1] their prefix
    int64_t bcost_alloc = 0;
    TaskQueue *tq = nullptr;
    // brick schedule of the force and adjoint kernels: static cost-balanced
    // ranges, or the queue (systems with empty regions, where the static
    // ranges leave workgroups idle); sched_mode 0 picks from `sparse`
    TaskQueue *ftq = nullptr;
    int32_t sched_mode = 0;
    int32_t gwin_limit = -1;   // most table intervals the EAM adjoint sums in LDS (-1: as many as fit)
    int32_t stage_u = 0;       // adjoint kernels stage partner cotangents in LDS when they fit (key 9)
    bool sparse = false;
    // waves of bricks with disjoint write sets (MD_LIST_WAVES)
    bool waves_valid = false;
    int32_t ncol = 0;
    std::vector<int64_t> wave_off;        // [ncol+1] offsets into wave_br
    std::vector<int32_t> brick_colour;    // [B] colour of each brick (host copy)
    int32_t *wave_br = nullptr;           // [B] bricks ordered by colour, then index
    int64_t wave_alloc = 0;
    std::vector<int32_t> wave_order;      // host copy of wave_br
    // the same tasks in dependence order (MD_LIST_DEPS): the task graph of the wave order
    bool deps_valid = false;
    std::vector<int32_t> dag_off_h, dag_succ_h, dag_npred_h;
    int32_t *dag_off = nullptr, *dag_succ = nullptr, *dag_npred = nullptr, *dag_init = nullptr;
    int32_t *dag_ref = nullptr, *dag_queue = nullptr;
    int64_t dag_alloc_t = 0, dag_alloc_e = 0;
    int32_t dag_roots = 0;
    int64_t wait_us = 2000000;            // longest wait for a queue slot (microseconds)
    // half lists over 14 of the 27 cells (built full, then filtered) and the
    // 3 x 3 x 2 task overlap they allow
    bool shell = false;
    bool eam_seen = false;               // an EAM potential was used with this context
    int64_t wall_khz = 100000;            // device wall clock (kHz)

    // atoms (cell-sorted)
    double4 *pos[2] = {nullptr, nullptr};
    double4 *pos_t = nullptr, *xref = nullptr;
    double *vel = nullptr, *vel_t = nullptr, *force = nullptr;
    int32_t *id = nullptr, *id_t = nullptr;
    int32_t *cell_of = nullptr, *slot = nullptr, *perm = nullptr;
    int32_t *count = nullptr, *start = nullptr;
    int cur = 0;

    // list
    bool have_list = false;
    int list_kind = MD_LIST_FULL;
    int32_t cap = 256;       // candidates staged in LDS per brick task
    int32_t cap_list = 256;  // candidates the list build stages (<= cap: its static LDS is larger)
    bool cap_user = false;
    int32_t M = 0;
    int64_t need_M = 0;
    uint32_t *nbr = nullptr;
    int32_t *cnt = nullptr;

    // scratch
    double *partial = nullptr;      // [maxgrid][4] x 4 sites
    double *eatom = nullptr, *watom = nullptr;
    double *rho = nullptr, *fp = nullptr, *fpp = nullptr, *rdot = nullptr;
    double *u_s = nullptr, *gx_s = nullptr;
    double *zeros_R = nullptr;
    double *tab64 = nullptr;
    float *tab32 = nullptr;
    int64_t tab_cap = 0;
    DevCtl *ctl = nullptr;
    int32_t *one = nullptr;
    unsigned char *scratch_dev = nullptr;   // this device's copy of `scratch`

    // event timing (md_profile)
    bool prof = false;
    bool prof_launches = false;   // event pairs around every force and list launch too
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_force, ev_list;
    // kind of each force launch: 0 F(x0) of md_verlet_step's setup (or a
    // md_compute_forces call), 1 a step that records no energies, 2 a recorded step
    std::vector<int8_t> ev_force_kind;
    int8_t force_kind = 0;
    // md_verlet_step: its setup (load, sort, list, F(x0)) and its step loop
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_setup, ev_loop;
    int64_t prof_steps = 0;
    double detail[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipEvent_t next_event()
    {
        if (ev_used == ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }

    int max_grid() const { return n_cu * 16; }
    int grid_atoms(int64_t per_block) const
    {
        int64_t g = (n + per_block - 1) / per_block;
        int64_t cap = (int64_t)n_cu * 8;
        return (int)std::max<int64_t>(1, std::min(g, cap));
    }
    int grid_cells(int cells_per_block, int per_cu) const
    {
        int64_t g = (C + cells_per_block - 1) / cells_per_block;
        int64_t capg = (int64_t)n_cu * per_cu;
        return (int)std::max<int64_t>(1, std::min(g, capg));
    }
    // persistent grid of brick tasks (one 256-thread workgroup per brick): as
    // many workgroups per CU as the LDS allows (160 KiB per CU), at most wgpc
    // workgroups of a brick-task grid whose workgroups take lds_block bytes of LDS
    int grid_with(size_t lds_block) const
    {
        const size_t per_block = lds_block + 512;
        int per_cu = (int)std::min<size_t>((size_t)wgpc, std::max<size_t>(1, (160 * 1024) / per_block));
        per_cu = std::max(1, std::min(per_cu, 32 / (threads / 64)));
        const int64_t g = std::min<int64_t>(B, (int64_t)n_cu * per_cu);
        return (int)std::max<int64_t>(1, g);
    }
    // the mixed density pass also holds its binary32 table in LDS when it fits
    bool density_table_in_lds(bool mixed, const md_potential *p) const
    {
        return mixed && stage_bytes(cap, 0, false, bd.stride) + (size_t)(p->rho.n_knots - 1) * 16 + 256 <= (size_t)lds_max;
    }
    int grid_density(bool mixed, const md_potential *p) const
    {
        return grid_with(stage_bytes(cap, 0, false, bd.stride) +
                         (density_table_in_lds(mixed, p) ? (size_t)(p->rho.n_knots - 1) * 16 : 0));
    }
    // the list build's grid: its own stage plus its static LDS
    int grid_list(int half) const
    {
        const size_t per_block = stage_bytes(cap_list, 0, half != 0, bd.stride) + list_static_lds(half) + 512;
        int per_cu = (int)std::min<size_t>((size_t)wgpc, std::max<size_t>(1, (160 * 1024) / per_block));
        per_cu = std::max(1, std::min(per_cu, 32 / (threads / 64)));
        const int64_t g = std::min<int64_t>(B, (int64_t)n_cu * per_cu);
        return (int)std::max<int64_t>(1, g);
    }
    int grid_tasks(int nextra, bool with_j) const
    {
        const size_t per_block = stage_bytes(cap, nextra, with_j, bd.stride) + 512;
        int per_cu = (int)std::min<size_t>((size_t)wgpc, std::max<size_t>(1, (160 * 1024) / per_block));
        per_cu = std::max(1, std::min(per_cu, 32 / (threads / 64)));   // at most 32 wavefronts per CU
        const int64_t g = std::min<int64_t>(B, (int64_t)n_cu * per_cu);
        return (int)std::max<int64_t>(1, g);
    }
    // list rows are allocated in groups of 64 atoms
    int64_t n64() const { return (n + 63) / 64 * 64; }
};

namespace {

int fail(md_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

int check_hip(md_ctx *c, const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, MD_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
    return MD_OK;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// cell grid of every replica; returns MD_OK, MD_ERR_ARG or MD_ERR_BOX
int plan_cells(md_ctx *c, const double *boxes, double rc, double skin, hipStream_t s)
{
    if (!(isfinite(rc) && rc > 0.0)) return fail(c, MD_ERR_ARG, "rc must be finite and > 0");
    if (!(isfinite(skin) && skin >= 0.0)) return fail(c, MD_ERR_ARG, "skin must be finite and >= 0");
    const double rl = rc + skin;
    for (int32_t r = 0; r < c->R; r++)
        for (int d = 0; d < 3; d++) {
            const double L = boxes[3 * r + d];
            if (!finite_pos(L)) return fail(c, MD_ERR_ARG, "box edges must be finite and > 0");
            if (!(L >= 2.0 * rl)) return fail(c, MD_ERR_BOX, "box edge shorter than 2 (rc + skin)");
        }
    bool same = c->have_cells && c->rc == rc && c->skin == skin &&
                std::equal(c->boxes.begin(), c->boxes.end(), boxes);
    if (same) return MD_OK;
    c->reps_h.assign(c->R, RepDesc{});
    int64_t cells = 0;
    for (int32_t r = 0; r < c->R; r++) {
        RepDesc &d = c->reps_h[r];
        for (int k = 0; k < 3; k++) {
            d.L[k] = boxes[3 * r + k];
            d.hL[k] = 0.5 * d.L[k];
            d.nc[k] = (int32_t)floor(d.L[k] / rl);
            if (d.nc[k] < 1) d.nc[k] = 1;
        }
        d.cell_off = cells;
        d.atom_off = c->off[r];
        d.atom_end = c->off[r + 1];
        cells += (int64_t)d.nc[0] * d.nc[1] * d.nc[2];
    }
    if (cells >= (1ll << 31) - 1) return fail(c, MD_ERR_ARG, "too many cells");
    if (cells > c->C_alloc) {
        if (!dalloc(&c->count, cells) || !dalloc(&c->start, cells + 1))
            return fail(c, MD_ERR_HIP, "cell arrays: out of device memory");
        if (hipMemsetAsync(c->count, 0, sizeof(int32_t) * cells, s) != hipSuccess)
            return fail(c, MD_ERR_HIP, "cell arrays: memset");
        c->C_alloc = cells;
    }
    c->C = cells;
    c->bricks_valid = false;
    if (hipMemcpyAsync(c->reps, c->reps_h.data(), sizeof(RepDesc) * c->R, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "replica descriptors: copy");
    c->rc = rc;
    c->skin = skin;
    c->rl = rl;
    c->boxes.assign(boxes, boxes + 3 * c->R);
    return MD_OK;
}

// bin -> scan -> scatter -> per-cell sort of pos[cur] (and vel, id) into the *_t buffers
void sort_into_tmp(md_ctx *c, const int32_t *pred, bool with_vel, hipStream_t s)
{
    const int ga = c->grid_atoms(256);
    launch_bin(s, ga, pred, c->n, c->R, c->reps, c->rep_of, c->pos[c->cur], c->cell_of, c->slot,
               c->count, &c->ctl->err);
    launch_scan(s, pred, c->C, c->count, c->start, c->ctl);
    launch_scatter(s, ga, pred, c->n, c->cell_of, c->slot, c->start, c->perm);
    launch_sort_cells(s, c->grid_cells(4, 8), pred, c->C, c->start, c->count, c->perm, c->id, c->pos[c->cur],
                      with_vel ? c->vel : nullptr, c->n, c->pos_t, with_vel ? c->vel_t : nullptr,
                      c->id_t);
}

ListArgs list_args(md_ctx *c, const int32_t *pred, const double4 *src, int half)
{
    ListArgs a{};
    a.pred = pred;
    a.B = c->B;
    a.R = c->R;
    a.reps = c->reps;
    a.start = c->start;
    a.brec = c->brec;
    a.bd = c->bd;
    a.tq = c->tq;
    a.bcost = c->bcost;
    a.bwork = c->bwork;
    a.src = src;
    a.n = c->n;
    a.nbr = c->nbr;
    a.cnt = c->cnt;
    a.M = c->M;
    a.rl2 = c->rl * c->rl;
    a.half = half;
    a.cap = c->cap_list;
    a.shift_cap = c->cap;
    a.ctl = c->ctl;
    return a;
}

// largest LDS stage (candidates, a multiple of 64) a brick task may use with
// one extra binary64 array per candidate within the per-workgroup LDS limit
int64_t cap_limit(const md_ctx *c)
{
    const int64_t room = c->lds_max - 4096 - 4 * (int64_t)c->bd.stride;
    return std::max<int64_t>(64, room / (int64_t)(4 * sizeof(double) + sizeof(uint16_t)) / 64 * 64);
}

// Brick shape and workgroup size from the mean occupancy `occ` of the
// non-empty cells: every shape of 1..4 cells per axis and every workgroup of
// 128..512 threads is scored by the lanes that hold an atom (mean atoms per
// brick over the threads of the rounds a brick of mean + 2 sqrt(mean) atoms
// takes), the wavefronts per CU that the
// LDS stage allows (saturating at 16) and the halo candidates staged per atom.
void choose_shape(md_ctx *c, double occ, int32_t out[4])
{
    double best = -1.0;
    for (int bz = 1; bz <= 4; bz++)
        for (int by = 1; by <= 4; by++)
            for (int bx = 1; bx <= 4; bx++)
                for (int T = 128; T <= TASK_MAX_THREADS; T += 64) {
                    const double cells = bx * by * bz, halo = (bx + 2) * (by + 2) * (bz + 2);
                    const double atoms = occ * cells;
                    // rounds of T lanes for a brick two standard deviations above the mean
                    const double rounds = std::ceil((atoms + 2.0 * std::sqrt(atoms)) / T);
                    const double eff = atoms / (rounds * T);
                    const double lds = 24.0 * 1.1 * occ * halo + 4.0 * br_stride((int32_t)halo, (int32_t)cells) + 512;
                    const double blocks = std::min<double>(c->wgpc, std::floor(160.0 * 1024 / lds));
                    if (blocks < 1 || lds > c->lds_max) continue;
                    const double waves = std::min(16.0, std::min(32.0, blocks * T / 64));
                    const double score = eff * (waves / 16.0) * (1.0 - 0.01 * halo / cells);
                    if (score > best + 1e-9) {
                        best = score;
                        out[0] = bx;
                        out[1] = by;
                        out[2] = bz;
                        out[3] = T;
                    }
                }
    if (best < 0) out[0] = out[1] = out[2] = 1, out[3] = 256;
}

// Bricks of every replica (shape clipped to the grid), record sizes, record buffer.
int plan_bricks(md_ctx *c, hipStream_t s)
{
    int32_t shape[4] = {c->bshape[0], c->bshape[1], c->bshape[2], c->threads_req > 0 ? c->threads_req : 256};
    std::vector<int32_t> cs(c->C + 1);
    if (hipMemcpyAsync(cs.data(), c->start, sizeof(int32_t) * (c->C + 1), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "brick plan: cell readback");
    int64_t ne = 0;
    for (int64_t k = 0; k < c->C; k++) ne += cs[k + 1] > cs[k];
    // more than 5 % empty cells: a system with voids or vacuum
    c->sparse = (double)ne < 0.95 * (double)c->C;
    if (shape[0] == 0) {
        choose_shape(c, (double)c->n / (double)std::max<int64_t>(1, ne), shape);
        if (c->threads_req > 0) shape[3] = c->threads_req;
    }
    c->threads = shape[3];
    int64_t bricks = 0;
    int32_t Hm = 1, Em = 1;
    for (int32_t r = 0; r < c->R; r++) {
        RepDesc &d = c->reps_h[r];
        int32_t H = 1, E = 1;
        for (int k = 0; k < 3; k++) {
            d.bd[k] = std::min(shape[k], d.nc[k]);
            d.nb[k] = (d.nc[k] + d.bd[k] - 1) / d.bd[k];
            H *= std::min(d.bd[k] + 2, d.nc[k]);
            E *= d.bd[k];
        }
        d.brick_off = bricks;
        bricks += (int64_t)d.nb[0] * d.nb[1] * d.nb[2];
        Hm = std::max(Hm, H);
        Em = std::max(Em, E);
    }
    c->bd.Hm = Hm;
    c->bd.Em = Em;
    c->bd.stride = br_stride(Hm, Em);
    const int64_t words = bricks * (int64_t)c->bd.stride;
    if (words > c->brec_alloc) {
        if (!dalloc(&c->brec, words)) return fail(c, MD_ERR_HIP, "brick records: out of device memory");
        c->brec_alloc = words;
    }
    if (bricks > c->bcost_alloc) {
        if (!dalloc(&c->bcost, bricks) || !dalloc(&c->bwork, bricks + 1))
            return fail(c, MD_ERR_HIP, "brick costs: out of device memory");
        c->bcost_alloc = bricks;
    }
    c->B = bricks;
    if (hipMemcpyAsync(c->reps, c->reps_h.data(), sizeof(RepDesc) * c->R, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "replica descriptors: copy");
    c->bricks_valid = true;
    c->waves_valid = false;
    c->deps_valid = false;
    return MD_OK;
}

// layers under a brick that its tasks write along axis k: none along z for the
// 14-cell half list, whose partners never lie below an atom's cell
int below_layers(const md_ctx *c, int k) { return k == 2 && c->shell ? 0 : 1; }

// Colours the bricks of every replica (md_waves.h); colour k of all replicas
// runs in one launch (replicas never interact).
int plan_waves(md_ctx *c, hipStream_t s)
{
    if (c->waves_valid) return MD_OK;
    c->brick_colour.assign((size_t)c->B, 0);
    int32_t ncol = 0;
    for (int32_t r = 0; r < c->R; r++) {
        const RepDesc &d = c->reps_h[r];
        int sep[3];
        for (int k = 0; k < 3; k++) sep[k] = mdwaves::axis_separation(d.nc[k], d.bd[k], below_layers(c, k));
        std::vector<int32_t> col;
        ncol = std::max(ncol, (int32_t)mdwaves::colour_bricks(d.nb, sep, col));
        std::copy(col.begin(), col.end(), c->brick_colour.begin() + d.brick_off);
    }
    std::vector<int64_t> cnt((size_t)ncol + 1, 0);
    for (int64_t b = 0; b < c->B; b++) cnt[(size_t)c->brick_colour[b] + 1]++;
    for (int32_t k = 0; k < ncol; k++) cnt[(size_t)k + 1] += cnt[k];
    std::vector<int32_t> order((size_t)c->B);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t b = 0; b < c->B; b++) order[(size_t)fill[c->brick_colour[b]]++] = (int32_t)b;
    if (c->B > c->wave_alloc) {
        if (!dalloc(&c->wave_br, c->B)) return fail(c, MD_ERR_HIP, "waves: out of device memory");
        c->wave_alloc = c->B;
    }
    if (hipMemcpyAsync(c->wave_br, order.data(), sizeof(int32_t) * c->B, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "waves: copy");
    c->ncol = ncol;
    c->wave_off = cnt;
    c->wave_order = order;
    c->waves_valid = true;
    c->deps_valid = false;
    return MD_OK;
}

// Task graph of the wave order (md_waves.h, backward method) for the
// dependent schedule; a brick's write set is its halo cells.
int plan_deps(md_ctx *c, hipStream_t s)
{
    int rc = plan_waves(c, s);
    if (rc != MD_OK) return rc;
    if (c->deps_valid) return MD_OK;
    const int64_t T = c->B;
    int64_t cells_total = 0;
    for (int32_t r = 0; r < c->R; r++) {
        const RepDesc &d = c->reps_h[r];
        cells_total = std::max<int64_t>(cells_total, d.cell_off + (int64_t)d.nc[0] * d.nc[1] * d.nc[2]);
    }
    std::vector<int> ax[3];
    auto cells = [&](int32_t b, std::vector<int64_t> &out) {
        int32_t r = 0;
        while (r + 1 < c->R && c->reps_h[r + 1].brick_off <= b) r++;
        const RepDesc &d = c->reps_h[r];
        int64_t lb = b - d.brick_off;
        const int bi[3] = {(int)(lb % d.nb[0]), (int)(lb / d.nb[0] % d.nb[1]), (int)(lb / ((int64_t)d.nb[0] * d.nb[1]))};
        for (int k = 0; k < 3; k++) {
            const int o = bi[k] * d.bd[k];
            mdwaves::axis_write_set(o, std::min(d.bd[k], d.nc[k] - o), d.nc[k], below_layers(c, k), ax[k]);
        }
        for (int z : ax[2])
            for (int y : ax[1])
                for (int x : ax[0]) out.push_back(d.cell_off + x + (int64_t)d.nc[0] * (y + (int64_t)d.nc[1] * z));
    };
    mdwaves::task_graph(c->wave_order, cells, cells_total, T, c->dag_off_h, c->dag_succ_h, c->dag_npred_h);
    std::vector<int32_t> init((size_t)T, -1);
    int32_t nroots = 0;
    for (int32_t t : c->wave_order)
        if (c->dag_npred_h[(size_t)t] == 0) init[(size_t)nroots++] = t;
    const int64_t E = (int64_t)c->dag_succ_h.size();
    bool ok = true;
    if (T > c->dag_alloc_t) {
        ok &= dalloc(&c->dag_off, (size_t)T + 1) && dalloc(&c->dag_npred, (size_t)T) && dalloc(&c->dag_init, (size_t)T) &&
              dalloc(&c->dag_ref, (size_t)T) && dalloc(&c->dag_queue, (size_t)T);
        c->dag_alloc_t = ok ? T : 0;
    }
    if (ok && E > c->dag_alloc_e) {
        ok &= dalloc(&c->dag_succ, (size_t)E);
        c->dag_alloc_e = ok ? E : 0;
    }
    if (!ok) return fail(c, MD_ERR_HIP, "dependent schedule: out of device memory");
    if (hipMemcpyAsync(c->dag_off, c->dag_off_h.data(), sizeof(int32_t) * (T + 1), hipMemcpyHostToDevice, s) != hipSuccess ||
        (E > 0 && hipMemcpyAsync(c->dag_succ, c->dag_succ_h.data(), sizeof(int32_t) * E, hipMemcpyHostToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(c->dag_npred, c->dag_npred_h.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(c->dag_init, init.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "dependent schedule: copy");
    c->dag_roots = nroots;
    c->deps_valid = true;
    return MD_OK;
}

// The wave kernel stages three more binary64 values (partner force sums) and
// the sorted index per candidate: a chosen stage shrinks to fit, a stage set
// by the caller that does not fit is an error.  Runs before the list build,
// whose records depend on the stage capacity.
int fit_wave_stage(md_ctx *c)
{
    // 256 bytes stay free for the kernels' static LDS
    const int64_t room = (int64_t)c->lds_max - 256;
    if ((int64_t)stage_bytes(c->cap, 3, true, c->bd.stride) <= room) return MD_OK;
    if (c->cap_user) return fail(c, MD_ERR_ARG, "wave-scheduled list: the LDS stage set with md_set_tuning is too large");
    const int64_t fit = (room - 16 - 4 * (int64_t)c->bd.stride) / (6 * 8 + 4 + 2) / 64 * 64;
    if (fit < 64) return fail(c, MD_ERR_STATE, "wave-scheduled list: brick record leaves no LDS stage");
    c->cap = (int32_t)fit;
    c->cap_list = std::min(c->cap_list, c->cap);
    return MD_OK;
}

// the wave launches of one force evaluation (forces accumulate into c->force,
// which the caller has cleared)
void launch_waves(md_ctx *c, hipStream_t s, bool mixed, ForceArgs a)
{
    if (c->list_kind == MD_LIST_DEPS) {
        DepArgs d{};
        d.off = c->dag_off;
        d.succ = c->dag_succ;
        d.ref = c->dag_ref;
        d.queue = c->dag_queue;
        d.sched = c->ctl->sched;
        d.T = (int32_t)c->B;
        d.limit = (uint64_t)(c->wait_us * c->wall_khz / 1000);
        launch_lj_deps(s, c->grid_tasks(3, true), c->threads, mixed, a, d, c->dag_npred, c->dag_init, c->dag_roots);
        return;
    }
    for (int32_t k = 0; k < c->ncol; k++) {
        const int64_t nb = c->wave_off[(size_t)k + 1] - c->wave_off[k];
        if (nb == 0) continue;
        a.wbr = c->wave_br + c->wave_off[k];
        a.nwb = (int32_t)nb;
        launch_lj_wave(s, (int)std::min<int64_t>(nb, c->max_grid()), c->threads, mixed, a);
    }
}

// first build: count pass, then size the lists (1.25 x the longest + margin)
// and the LDS stage (the largest halo seen + 5 %)
// per_cand: LDS bytes per staged candidate of the kernels that will use the
// list (xyz, the halo-cell table, extras, sorted indices); callers that do not
// know the potential pass the largest layout of the potentials the context has
// seen (LJ with sorted indices: 30; EAM, one extra value: 34)
inline int stage_bytes_any(const md_ctx *c) { return 3 * 8 + 2 + (c->eam_seen ? 8 : 4); }

int size_list(md_ctx *c, const double4 *src, int half, hipStream_t s, int per_cand)
{
    if (!c->bricks_valid) {
        int rc = plan_bricks(c, s);
        if (rc != MD_OK) return rc;
    }
    if (!c->cap_user) c->cap = c->cap_list = (int32_t)std::min<int64_t>(cap_limit(c), 2048);
    ListArgs a = list_args(c, c->one, src, half);
    a.M = 0;
    a.nbr = nullptr;
    const int32_t zero3[3] = {0, 0, 0};
    if (hipMemcpyAsync(&c->ctl->max_cnt, &zero3[0], sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(&c->ctl->max_nbhd, &zero3[1], sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(&c->ctl->max_brick, &zero3[2], sizeof(int32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "list sizing: reset");
    launch_build_list(s, c->grid_list(half), c->threads, a);
    int32_t mx = 0, nbhd = 0;
    if (hipMemcpyAsync(&mx, &c->ctl->max_cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&nbhd, &c->ctl->max_nbhd, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(c, MD_ERR_HIP, "list sizing: readback");
    // LDS stage: the largest halo seen plus 5 %, in multiples of 64, within
    // half a CU's LDS for the kernels' layout (larger halos read their last
    // candidates from global memory).  Without EAM, the stage then grows to
    // the largest that leaves as many workgroups resident per CU: halos that
    // grow as the system evolves (a free cluster contracting to its
    // equilibrium density) stay wholly staged, and their bricks keep the
    // 16-bit entries, at no cost in occupancy.  (The mixed EAM density pass
    // adds its table to the stage, so EAM stages keep the smallest size.)
    // The list build, whose static LDS is larger, grows its own stage under
    // the same rule; a halo that fits the force tasks' stage but not the list
    // build's is listed with some candidates read from global memory.
    if (!c->cap_user) {
        // (1 KB kept free for the allocation granularity)
        const int64_t cu = 160 * 1024, fixed = 512 + 1024 + 4 * (int64_t)c->bd.stride;
        const int64_t waves = 32 / (c->threads / 64);
        const int64_t want = ((int64_t)(1.05 * nbhd) + 63) / 64 * 64;
        auto grown = [&](int64_t bytes, int64_t extra) {
            const int64_t lim = std::min<int64_t>(cap_limit(c), (cu / 2 - fixed - extra) / bytes / 64 * 64);
            int64_t cap = std::max<int64_t>(64, std::min<int64_t>(lim, want));
            if (!c->eam_seen) {
                const int64_t per_cu = std::max<int64_t>(
                    1, std::min<int64_t>({(int64_t)c->wgpc, waves, cu / (cap * bytes + fixed + extra)}));
                cap = std::max<int64_t>(cap, std::min<int64_t>(lim, (cu / per_cu - fixed - extra) / bytes / 64 * 64));
            }
            return std::max<int64_t>(64, cap);
        };
        c->cap = (int32_t)grown(per_cand, 0);
        c->cap_list = (int32_t)std::min<int64_t>(
            c->cap, grown(3 * 8 + 2 + (half ? 4 : 0), (int64_t)list_static_lds(half)));
    }
    // rows: kept if they are already allocated and no overflow asked for more
    if (c->M > 0 && c->need_M <= c->M) return MD_OK;
    int64_t want = std::max<int64_t>({(int64_t)ceil(1.25 * mx), (int64_t)mx + 16, c->need_M, 16});
    want = (want + 7) / 8 * 8;
    if (want * c->n64() > (1ll << 40)) return fail(c, MD_ERR_ARG, "neighbour list too large");
    if (!dalloc(&c->nbr, (size_t)(want * c->n64()))) return fail(c, MD_ERR_HIP, "list: out of device memory");
    c->M = (int32_t)want;
    c->need_M = 0;
    return MD_OK;
}

int ensure_list_capacity(md_ctx *c, const double4 *src, int half, hipStream_t s, int per_cand = 0)
{
    if (per_cand == 0) per_cand = stage_bytes_any(c);
    if (!c->bricks_valid || c->M == 0 || c->need_M > c->M) return size_list(c, src, half, s, per_cand);
    return MD_OK;
}

// The list builder's pair rule for a list kind: the sorted-order half list is
// built directly; the 14-cell half list is built full and then filtered.
int builder_half(const md_ctx *c, int half) { return half && !c->shell ? 1 : 0; }

// one list build (la made with builder_half), and the filter of the 14-cell half list
void build_list(md_ctx *c, hipStream_t s, int half, const ListArgs &la)
{
    launch_build_list(s, c->grid_list(la.half), c->threads, la);
    if (half && c->shell) launch_shell_filter(s, c->grid_tasks(0, false), c->threads, la);
}

ForceArgs force_args(md_ctx *c, const md_potential *p)
{
    ForceArgs a{};
    a.lds_tab = p->kind == MD_POT_EAM && c->density_table_in_lds(true, p) ? 1 : 0;
    a.ftq = c->ftq;
    a.dyn = c->sched_mode == 2 || (c->sched_mode == 0 && c->sparse) ? 1 : 0;
    a.n = c->n;
    a.R = c->R;
    a.reps = c->reps;
    a.rep0 = c->reps_h[0];
    a.rep_of = c->rep_of;
    a.pos = c->pos[c->cur];
    a.pos_next = c->pos[1 - c->cur];
    a.xref = c->xref;
    a.vel = c->vel;
    a.force = c->force;
    a.nbr = c->nbr;
    a.cnt = c->cnt;
    a.M = c->M;
    a.B = c->B;
    a.brec = c->brec;
    a.bd = c->bd;
    a.bwork = c->bwork;
    a.cap = c->cap;
    a.rc2 = p->rc * p->rc;
    a.lj = p->lj_params;
    a.rho = c->rho;
    a.fp = c->fp;
    a.partial = c->partial;
    a.ctl = c->ctl;
    a.mass = 1.0;
    if (p->kind == MD_POT_EAM) {
        const md_spline *sp[3] = {&p->phi, &p->rho, &p->embed};
        int64_t o = 0;
        for (int k = 0; k < 3; k++) {
            a.tab[k] = c->tab64 + o;
            a.tabf[k] = c->tab32 + o;
            a.nk[k] = sp[k]->n_knots;
            a.x0[k] = sp[k]->x0;
            a.inv_h[k] = 1.0 / sp[k]->h;
            o += 4 * (int64_t)(sp[k]->n_knots - 1);
        }
        a.rphi2 = p->rc_phi * p->rc_phi;
        a.rrho2 = p->rc_rho * p->rc_rho;
    }
    return a;
}

// The device address of `scratch` on device dev, looked up once per device
// (with that device current) and kept.
std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_dev;

int scratch_address(int dev, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it == g_scratch_dev.end()) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return MD_ERR_HIP;
        it = g_scratch_dev.emplace(dev, static_cast<unsigned char *>(p)).first;
    }
    *out = it->second;
    return MD_OK;
}

int check_pot(md_ctx *c, const md_potential *p)
{
    if (p == nullptr) return fail(c, MD_ERR_ARG, "potential is null");
    if (!(isfinite(p->rc) && p->rc > 0.0)) return fail(c, MD_ERR_ARG, "potential rc must be > 0");
    if (p->rc != c->rc) return fail(c, MD_ERR_STATE, "potential rc differs from the rc of md_build_cells");
    if (p->kind == MD_POT_LJ) {
        if (p->lj_params == nullptr) return fail(c, MD_ERR_ARG, "LJ parameters are null");
        return MD_OK;
    }
    if (p->kind != MD_POT_EAM) return fail(c, MD_ERR_ARG, "unknown potential kind");
    c->eam_seen = true;     // later list sizings leave room for the EAM layout
    const md_spline *sp[3] = {&p->phi, &p->rho, &p->embed};
    for (int k = 0; k < 3; k++) {
        if (sp[k]->coef == nullptr || sp[k]->n_knots < 2 || !finite_pos(sp[k]->h) || !isfinite(sp[k]->x0))
            return fail(c, MD_ERR_ARG, "EAM table: need coef, n_knots >= 2, finite h > 0");
    }
    if (!finite_pos(p->rc_phi) || !finite_pos(p->rc_rho) || std::max(p->rc_phi, p->rc_rho) != p->rc)
        return fail(c, MD_ERR_ARG, "EAM cutoffs: rc must equal max(rc_phi, rc_rho)");
    return MD_OK;
}

// copy (and convert) the EAM tables into aligned context buffers
int stage_tables(md_ctx *c, const md_potential *p, hipStream_t s)
{
    if (p->kind != MD_POT_EAM) return MD_OK;
    const md_spline *sp[3] = {&p->phi, &p->rho, &p->embed};
    int64_t total = 0;
    for (int k = 0; k < 3; k++) total += 4 * (int64_t)(sp[k]->n_knots - 1);
    if (total > c->tab_cap) {
        if (!dalloc(&c->tab64, total) || !dalloc(&c->tab32, total))
            return fail(c, MD_ERR_HIP, "tables: out of device memory");
        c->tab_cap = total;
    }
    int64_t o = 0;
    for (int k = 0; k < 3; k++) {
        const int64_t m = 4 * (int64_t)(sp[k]->n_knots - 1);
        if (hipMemcpyAsync(c->tab64 + o, sp[k]->coef, sizeof(double) * m, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            return fail(c, MD_ERR_HIP, "tables: copy");
        o += m;
    }
    launch_tables_f32(s, c->tab64, c->tab32, total);
    return MD_OK;
}

// records an event pair around launch() when profiling is on
template <typename F>
void timed(md_ctx *c, hipStream_t s, std::vector<std::pair<hipEvent_t, hipEvent_t>> &log, F launch)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (c->prof && c->prof_launches) {
        a = c->next_event();
        b = c->next_event();
        if (a && b) (void)hipEventRecord(a, s);
    }
    launch();
    if (c->prof && c->prof_launches && a && b) {
        (void)hipEventRecord(b, s);
        log.emplace_back(a, b);
        if (&log == &c->ev_force) c->ev_force_kind.push_back(c->force_kind);
    }
}

// records one event when profiling is on (null otherwise)
hipEvent_t mark(md_ctx *c, hipStream_t s)
{
    if (!c->prof) return nullptr;
    hipEvent_t e = c->next_event();
    if (e) (void)hipEventRecord(e, s);
    return e;
}

} // namespace

extern "C" {

int md_create(md_ctx **out, int64_t n, int32_t R, const int64_t *off)
{
    if (out == nullptr) return MD_ERR_ARG;
    *out = nullptr;
    if (n <= 0 || n > MD_MAX_ATOMS || R <= 0 || off == nullptr) return MD_ERR_ARG;
    if (off[0] != 0 || off[R] != n) return MD_ERR_ARG;
    for (int32_t r = 0; r < R; r++)
        if (off[r + 1] <= off[r]) return MD_ERR_ARG;
    md_ctx *c = new md_ctx();
    c->n = n;
    c->R = R;
    c->off.assign(off, off + R + 1);
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return MD_ERR_HIP;
    }
    if (scratch_address(c->device, &c->scratch_dev) != MD_OK) {
        delete c;
        return MD_ERR_HIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        ncu > 0)
        c->n_cu = ncu;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) == hipSuccess &&
        lds > 0)
        c->lds_max = lds;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
        c->wall_khz = khz;
    bool ok = true;
    ok &= dalloc(&c->pos[0], n) && dalloc(&c->pos[1], n) && dalloc(&c->pos_t, n) && dalloc(&c->xref, n);
    ok &= dalloc(&c->vel, 3 * n) && dalloc(&c->vel_t, 3 * n) && dalloc(&c->force, 3 * n);
    ok &= dalloc(&c->id, n) && dalloc(&c->id_t, n) && dalloc(&c->cell_of, n) && dalloc(&c->slot, n) &&
          dalloc(&c->perm, n) && dalloc(&c->cnt, n) && dalloc(&c->rep_of, n);
    ok &= dalloc(&c->eatom, n) && dalloc(&c->watom, n) && dalloc(&c->rho, n) && dalloc(&c->fp, n) &&
          dalloc(&c->fpp, n) && dalloc(&c->rdot, n);
    ok &= dalloc(&c->u_s, 4 * n) && dalloc(&c->gx_s, 3 * n);
    ok &= dalloc(&c->partial, (size_t)c->max_grid() * 4 * 4) && dalloc(&c->zeros_R, R);
    ok &= dalloc(&c->reps, R) && dalloc(&c->ctl, 1) && dalloc(&c->one, 1) && dalloc(&c->tq, 1) && dalloc(&c->ftq, 1);
    if (!ok) {
        md_destroy(c);
        return MD_ERR_HIP;
    }
    std::vector<int32_t> rep(n);
    for (int32_t r = 0; r < R; r++)
        for (int64_t i = off[r]; i < off[r + 1]; i++) rep[i] = r;
    const int32_t one = 1;
    DevCtl z{};
    TaskQueue zq{};
    std::vector<double> zr(R, 0.0);
    ok = hipMemcpy(c->rep_of, rep.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->one, &one, sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->ctl, &z, sizeof(DevCtl), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->tq, &zq, sizeof(TaskQueue), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->ftq, &zq, sizeof(TaskQueue), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(c->zeros_R, zr.data(), sizeof(double) * R, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        md_destroy(c);
        return MD_ERR_HIP;
    }
    *out = c;
    return MD_OK;
}

void md_destroy(md_ctx *c)
{
    if (c == nullptr) return;
    (void)hipDeviceSynchronize();
    dfree(c->pos[0]); dfree(c->pos[1]); dfree(c->pos_t); dfree(c->xref);
    dfree(c->vel); dfree(c->vel_t); dfree(c->force);
    dfree(c->id); dfree(c->id_t); dfree(c->cell_of); dfree(c->slot); dfree(c->perm);
    dfree(c->count); dfree(c->start); dfree(c->nbr); dfree(c->cnt); dfree(c->rep_of); dfree(c->brec); dfree(c->bcost); dfree(c->bwork); dfree(c->tq); dfree(c->ftq); dfree(c->wave_br);
    dfree(c->dag_off); dfree(c->dag_succ); dfree(c->dag_npred); dfree(c->dag_init); dfree(c->dag_ref); dfree(c->dag_queue);
    dfree(c->eatom); dfree(c->watom); dfree(c->rho); dfree(c->fp); dfree(c->fpp); dfree(c->rdot);
    dfree(c->u_s); dfree(c->gx_s); dfree(c->partial); dfree(c->zeros_R);
    dfree(c->tab64); dfree(c->tab32); dfree(c->reps); dfree(c->ctl); dfree(c->one);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    delete c;
}

int md_build_cells(md_ctx *c, const double *pos, const double *boxes, double rc, double skin,
                   void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (pos == nullptr || boxes == nullptr) return fail(c, MD_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    int rcode = plan_cells(c, boxes, rc, skin, s);
    if (rcode != MD_OK) return rcode;
    launch_load_user(s, c->grid_atoms(256), c->n, pos, nullptr, c->pos[c->cur], c->vel, c->id);
    sort_into_tmp(c, c->one, false, s);
    launch_copy_back(s, c->grid_atoms(256), c->one, c->n, c->pos_t, nullptr, c->id_t,
                     c->pos[c->cur], nullptr, c->id, c->xref);
    c->have_cells = true;
    c->have_list = false;
    return check_hip(c, "md_build_cells");
}

int md_build_neighbor_list(md_ctx *c, int32_t kind, void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (kind != MD_LIST_FULL && kind != MD_LIST_HALF && kind != MD_LIST_WAVES && kind != MD_LIST_DEPS)
        return fail(c, MD_ERR_ARG, "unknown list kind");
    if (!c->have_cells) return fail(c, MD_ERR_STATE, "md_build_cells first");
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    const int half = kind != MD_LIST_FULL;
    int rcode = ensure_list_capacity(c, c->pos[c->cur], builder_half(c, half), s);
    if (rcode != MD_OK) return rcode;
    if (kind == MD_LIST_WAVES && ((rcode = fit_wave_stage(c)) != MD_OK || (rcode = plan_waves(c, s)) != MD_OK))
        return rcode;
    if (kind == MD_LIST_DEPS && ((rcode = fit_wave_stage(c)) != MD_OK || (rcode = plan_deps(c, s)) != MD_OK))
        return rcode;
    build_list(c, s, half, list_args(c, c->one, c->pos[c->cur], builder_half(c, half)));
    c->have_list = true;
    c->list_kind = kind;
    return check_hip(c, "md_build_neighbor_list");
}

int md_compute_forces(md_ctx *c, const md_potential *p, int32_t precision, double *forces,
                      double *energy, double *virial, void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (forces == nullptr) return fail(c, MD_ERR_ARG, "forces is null");
    if (precision != MD_FP64 && precision != MD_MIXED) return fail(c, MD_ERR_ARG, "unknown precision");
    if (!c->have_list) return fail(c, MD_ERR_STATE, "md_build_neighbor_list first");
    int rcode = check_pot(c, p);
    if (rcode != MD_OK) return rcode;
    if (c->list_kind == MD_LIST_HALF && (p->kind != MD_POT_LJ || c->R > 1))
        return fail(c, MD_ERR_STATE, "the half list serves LJ on one replica; build a full list");
    const bool scheduled = c->list_kind == MD_LIST_WAVES || c->list_kind == MD_LIST_DEPS;
    if (scheduled && p->kind != MD_POT_LJ)
        return fail(c, MD_ERR_STATE, "the scheduled half lists serve LJ; build a full list");
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    if ((rcode = stage_tables(c, p, s)) != MD_OK) return rcode;
    const bool mixed = precision == MD_MIXED;
    ForceArgs a = force_args(c, p);
    a.mode = 0;
    if (scheduled) {
        // per-atom energies summed per replica in a fixed order
        if (energy != nullptr || virial != nullptr) {
            a.eatom = c->eatom;
            a.watom = c->watom;
        }
        launch_zero(s, c->grid_atoms(256), c->force, 3 * c->n);
        launch_waves(c, s, mixed, a);
        if (energy != nullptr || virial != nullptr)
            launch_replica_sums(s, c->R, c->reps, c->eatom, c->watom, energy, virial);
        launch_to_user(s, c->grid_atoms(256), c->n, c->id, c->force, forces);
        return check_hip(c, "md_compute_forces");
    }
    if (c->R == 1) {
        a.outE = energy;
        a.outW = virial;
    } else if (energy != nullptr || virial != nullptr) {
        a.eatom = c->eatom;
        a.watom = c->watom;
    }
    const int gf = c->grid_tasks(0, false), gh = c->grid_tasks(0, true), gf1 = c->grid_tasks(1, false);
    if (p->kind == MD_POT_LJ && c->list_kind == MD_LIST_HALF) {
        launch_zero(s, c->grid_atoms(256), c->force, 3 * c->n);
        launch_lj_half(s, gh, c->threads, mixed, a);
    } else if (p->kind == MD_POT_LJ) {
        launch_lj_full(s, gf, c->threads, mixed, a);
    } else {
        launch_eam_density(s, c->grid_density(mixed, p), c->threads, mixed, a);
        launch_eam_force(s, gf1, c->threads, mixed, a);
    }
    if (c->R > 1 && (energy != nullptr || virial != nullptr))
        launch_replica_sums(s, c->R, c->reps, c->eatom, c->watom, energy, virial);
    launch_to_user(s, c->grid_atoms(256), c->n, c->id, c->force, forces);
    return check_hip(c, "md_compute_forces");
}

int md_compute_forces_noalloc(md_ctx *c, const md_potential *p, int32_t precision, double *forces,
                              double *energy, double *virial, void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (forces == nullptr) return fail(c, MD_ERR_ARG, "forces is null");
    if (precision != MD_FP64 && precision != MD_MIXED) return fail(c, MD_ERR_ARG, "unknown precision");
    if (!c->have_list) return fail(c, MD_ERR_STATE, "md_build_neighbor_list first");
    if (c->list_kind != MD_LIST_FULL) return fail(c, MD_ERR_STATE, "md_compute_forces_noalloc needs a full list");
    int rcode = check_pot(c, p);
    if (rcode != MD_OK) return rcode;
    if (c->scratch_dev == nullptr) return fail(c, MD_ERR_STATE, "no scratch address for this device");
    const bool eam = p->kind == MD_POT_EAM;
    const bool per_atom = c->R > 1 && (energy != nullptr || virial != nullptr);
    int64_t ntab = 0;
    if (eam) {
        const md_spline *sp[3] = {&p->phi, &p->rho, &p->embed};
        for (int k = 0; k < 3; k++) ntab += 4 * (int64_t)(sp[k]->n_knots - 1);
    }
    // carve the scratch: [brick queue | partials | forces | rho, F' | tables | per-atom E, W]
    auto up = [](uint64_t b) { return (b + 255) & ~(uint64_t)255; };
    const uint64_t n = (uint64_t)c->n;
    uint64_t o_queue = 0;
    uint64_t o_part = up(o_queue + sizeof(TaskQueue));
    uint64_t o_force = up(o_part + (uint64_t)c->max_grid() * 4 * sizeof(double));
    uint64_t o_rho = up(o_force + 3 * n * sizeof(double));
    uint64_t o_fp = up(o_rho + (eam ? n * sizeof(double) : 0));
    uint64_t o_t64 = up(o_fp + (eam ? n * sizeof(double) : 0));
    uint64_t o_t32 = up(o_t64 + (uint64_t)ntab * sizeof(double));
    uint64_t o_e = up(o_t32 + (uint64_t)ntab * sizeof(float));
    uint64_t o_w = up(o_e + (per_atom ? n * sizeof(double) : 0));
    const uint64_t need = up(o_w + (per_atom ? n * sizeof(double) : 0));
    if (need > MD_NOALLOC_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg, "md_compute_forces_noalloc: this system needs %llu bytes of scratch, "
                 "the library holds %llu", (unsigned long long)need, (unsigned long long)MD_NOALLOC_BYTES);
        return fail(c, MD_ERR_ARG, msg);
    }
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    unsigned char *base = c->scratch_dev;
    // the queue must start at zero (a fill kernel, no memset node)
    launch_zero(s, 1, reinterpret_cast<double *>(base), (int64_t)(o_part / sizeof(double)));
    const bool mixed = precision == MD_MIXED;
    ForceArgs a = force_args(c, p);
    a.mode = 0;
    a.ftq = reinterpret_cast<TaskQueue *>(base + o_queue);
    a.partial = reinterpret_cast<double *>(base + o_part);
    a.force = reinterpret_cast<double *>(base + o_force);
    if (eam) {
        a.rho = reinterpret_cast<double *>(base + o_rho);
        a.fp = reinterpret_cast<double *>(base + o_fp);
        double *t64 = reinterpret_cast<double *>(base + o_t64);
        float *t32 = reinterpret_cast<float *>(base + o_t32);
        const md_spline *sp[3] = {&p->phi, &p->rho, &p->embed};
        int64_t o = 0;
        for (int k = 0; k < 3; k++) {
            const int64_t m = 4 * (int64_t)(sp[k]->n_knots - 1);
            if (hipMemcpyAsync(t64 + o, sp[k]->coef, sizeof(double) * m, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return fail(c, MD_ERR_HIP, "tables: copy");
            a.tab[k] = t64 + o;
            a.tabf[k] = t32 + o;
            o += m;
        }
        launch_tables_f32(s, t64, t32, ntab);
    }
    if (c->R == 1) {
        a.outE = energy;
        a.outW = virial;
    } else if (per_atom) {
        a.eatom = reinterpret_cast<double *>(base + o_e);
        a.watom = reinterpret_cast<double *>(base + o_w);
    }
    if (p->kind == MD_POT_LJ) {
        launch_lj_full(s, c->grid_tasks(0, false), c->threads, mixed, a);
    } else {
        launch_eam_density(s, c->grid_density(mixed, p), c->threads, mixed, a);
        launch_eam_force(s, c->grid_tasks(1, false), c->threads, mixed, a);
    }
    if (per_atom) launch_replica_sums(s, c->R, c->reps, a.eatom, a.watom, energy, virial);
    launch_to_user(s, c->grid_atoms(256), c->n, c->id, a.force, forces);
    return check_hip(c, "md_compute_forces_noalloc");
}

int md_verlet_step(md_ctx *c, const md_potential *p, int32_t precision, int32_t kind, double *pos,
                   double *vel, double *forces, double dt, double mass, int32_t n_steps,
                   double *hist, int32_t hist_every, int32_t *rebuilds, void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (pos == nullptr || vel == nullptr || forces == nullptr) return fail(c, MD_ERR_ARG, "null argument");
    if (n_steps < 1 || !finite_pos(dt) || !finite_pos(mass)) return fail(c, MD_ERR_ARG, "need n_steps >= 1, dt > 0, mass > 0");
    if (hist != nullptr && hist_every < 1) return fail(c, MD_ERR_ARG, "hist_every must be >= 1");
    if (precision != MD_FP64 && precision != MD_MIXED) return fail(c, MD_ERR_ARG, "unknown precision");
    if (kind != MD_LIST_FULL && kind != MD_LIST_HALF && kind != MD_LIST_WAVES && kind != MD_LIST_DEPS)
        return fail(c, MD_ERR_ARG, "unknown list kind");
    if (!c->have_cells) return fail(c, MD_ERR_STATE, "md_build_cells first (sets boxes, rc, skin)");
    int rcode = check_pot(c, p);
    if (rcode != MD_OK) return rcode;
    if (kind != MD_LIST_FULL && p->kind != MD_POT_LJ) return fail(c, MD_ERR_STATE, "the half lists serve LJ only");
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    if ((rcode = stage_tables(c, p, s)) != MD_OK) return rcode;
    const bool mixed = precision == MD_MIXED;
    const int half = kind != MD_LIST_FULL;
    const bool waves = kind == MD_LIST_WAVES || kind == MD_LIST_DEPS;
    const int ga = c->grid_atoms(256);

    // initial state: user order -> sorted, cells and list from scratch
    hipEvent_t ev_begin = mark(c, s);
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, c->ctl, 1, 1);
    launch_load_user(s, ga, c->n, pos, vel, c->pos[c->cur], c->vel, c->id);
    sort_into_tmp(c, c->one, true, s);
    // the potential is known here: the stage is sized for its kernels' layout
    const int per_cand = 3 * 8 + 2 + (p->kind == MD_POT_EAM ? 8 : 0) + (half ? 4 : 0);
    if ((rcode = ensure_list_capacity(c, c->pos_t, builder_half(c, half), s, per_cand)) != MD_OK) return rcode;
    if (waves && ((rcode = fit_wave_stage(c)) != MD_OK ||
                  (rcode = kind == MD_LIST_DEPS ? plan_deps(c, s) : plan_waves(c, s)) != MD_OK))
        return rcode;
    {
        ListArgs la = list_args(c, c->one, c->pos_t, builder_half(c, half));
        la.vel_src = c->vel_t;
        la.id_src = c->id_t;
        la.pos_dst = c->pos[c->cur];
        la.vel_dst = c->vel;
        la.id_dst = c->id;
        la.xref = c->xref;
        build_list(c, s, half, la);
    }
    c->have_list = true;
    c->list_kind = kind;
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, c->ctl, 0, 1);   // count in-run rebuilds only

    const int gf = c->grid_tasks(0, false), gh = c->grid_tasks(0, true), gf1 = c->grid_tasks(1, false);
    auto forces_and_step = [&](int mode, int32_t *clear, int32_t *set, double *h) {
        ForceArgs a = force_args(c, p);
        a.mode = mode;
        a.cdt = 0.5 * dt / mass;
        a.dt = dt;
        a.mass = mass;
        a.thr2 = (0.5 * c->skin) * (0.5 * c->skin);
        a.flag_clear = clear;
        a.flag_set = set;
        if (h != nullptr) {
            a.outE = h;
            a.outK = h + 1;
            a.outW = h + 2;
        }
        if (waves) {
            // the wave launches, the energies of a recorded step from the
            // per-atom sums, then the velocity-Verlet pass
            ForceArgs f = a;
            f.mode = 0;
            f.force = c->force;
            f.outE = f.outK = f.outW = nullptr;
            f.flag_clear = nullptr;
            f.flag_set = nullptr;
            const bool en = mode >= 2 && a.outE != nullptr;
            f.eatom = en ? c->eatom : nullptr;
            f.watom = en ? c->watom : nullptr;
            ForceArgs g = a;
            g.outE = nullptr;
            g.outW = nullptr;
            g.outK = mode >= 2 ? a.outK : nullptr;
            g.partial = c->partial + (size_t)c->max_grid() * 8;
            timed(c, s, c->ev_force, [&] {
                launch_waves(c, s, mixed, f);
                if (en)
                    launch_atom_sums(s, c->grid_atoms(1024), c->n, c->eatom, c->watom, a.outE, a.outW,
                                     c->partial);
                launch_integrate(s, ga, g);
            });
        } else if (p->kind == MD_POT_LJ && half) {
            ForceArgs f = a;
            f.mode = 0;
            f.force = c->force;
            f.outK = nullptr;
            f.flag_clear = nullptr;
            f.flag_set = nullptr;
            f.outE = mode >= 2 ? a.outE : nullptr;
            f.outW = mode >= 2 ? a.outW : nullptr;
            f.partial = c->partial + (size_t)c->max_grid() * 4;
            ForceArgs g = a;
            g.outE = nullptr;
            g.outW = nullptr;
            g.outK = mode >= 2 ? a.outK : nullptr;
            g.partial = c->partial + (size_t)c->max_grid() * 8;
            timed(c, s, c->ev_force, [&] {
                launch_lj_half(s, gh, c->threads, mixed, f);
                launch_integrate(s, ga, g);
            });
        } else if (p->kind == MD_POT_LJ) {
            if (mode == 1) a.outE = a.outK = a.outW = nullptr;
            timed(c, s, c->ev_force, [&] { launch_lj_full(s, gf, c->threads, mixed, a); });
        } else {
            if (mode == 1) a.outE = a.outK = a.outW = nullptr;
            timed(c, s, c->ev_force, [&] {
                launch_eam_density(s, c->grid_density(mixed, p), c->threads, mixed, a);
                launch_eam_force(s, gf1, c->threads, mixed, a);
            });
        }
    };

    if (half) launch_zero(s, ga, c->force, 3 * c->n);
    // F(x0), first half kick and drift; requests a rebuild for step 1 if needed
    c->force_kind = 0;
    forces_and_step(1, &c->ctl->rebuild[0], &c->ctl->rebuild[1], nullptr);
    c->cur = 1 - c->cur;
    hipEvent_t ev_loop0 = mark(c, s);
    for (int32_t st = 1; st <= n_steps; st++) {
        int32_t *pred = &c->ctl->rebuild[st & 1];
        sort_into_tmp(c, pred, true, s);
        ListArgs la = list_args(c, pred, c->pos_t, builder_half(c, half));
        la.vel_src = c->vel_t;
        la.id_src = c->id_t;
        la.pos_dst = c->pos[c->cur];
        la.vel_dst = c->vel;
        la.id_dst = c->id;
        la.xref = c->xref;
        timed(c, s, c->ev_list, [&] { build_list(c, s, half, la); });
        const int mode = st < n_steps ? 2 : 3;
        // energies of every hist_every-th step and of the last one
        const bool rec = hist != nullptr && (st % hist_every == 0 || st == n_steps);
        c->force_kind = rec ? 2 : 1;
        forces_and_step(mode, pred, &c->ctl->rebuild[(st + 1) & 1],
                        rec ? hist + 3 * (int64_t)((st + hist_every - 1) / hist_every - 1) : nullptr);
        if (mode == 2) c->cur = 1 - c->cur;
    }
    hipEvent_t ev_loop1 = mark(c, s);
    c->force_kind = 0;
    if (ev_begin && ev_loop0 && ev_loop1) {
        c->ev_setup.emplace_back(ev_begin, ev_loop0);
        c->ev_loop.emplace_back(ev_loop0, ev_loop1);
        c->prof_steps += n_steps;
    }
    launch_pos_to_user(s, ga, c->n, c->R, c->reps, c->rep_of, c->id, c->pos[c->cur], pos);
    launch_to_user(s, ga, c->n, c->id, c->vel, vel);
    launch_to_user(s, ga, c->n, c->id, c->force, forces);
    if (rebuilds != nullptr) hipLaunchKernelGGL(k_copy_int, dim3(1), dim3(64), 0, s, &c->ctl->nrebuild, rebuilds);
    return check_hip(c, "md_verlet_step");
}

int md_force_vjp(md_ctx *c, const md_potential *p, int32_t precision, const double *pos,
                 const double *u, const double *vE, double *g_pos, double *g_params, void *stream)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (u == nullptr) return fail(c, MD_ERR_ARG, "u_forces is null");
    if (precision != MD_FP64 && precision != MD_MIXED) return fail(c, MD_ERR_ARG, "unknown precision");
    if (!c->have_list) return fail(c, MD_ERR_STATE, "md_build_neighbor_list first");
    if (c->list_kind != MD_LIST_FULL) return fail(c, MD_ERR_STATE, "the adjoint needs a full list");
    int rcode = check_pot(c, p);
    if (rcode != MD_OK) return rcode;
    hipStream_t s = (hipStream_t)stream;
    c->last = s;
    if ((rcode = stage_tables(c, p, s)) != MD_OK) return rcode;
    const int ga = c->grid_atoms(256);
    if (pos != nullptr)
        hipLaunchKernelGGL(k_pos_from_user, dim3(ga), dim3(256), 0, s, c->n, c->reps, c->rep_of, c->id,
                           pos, c->xref, c->pos[c->cur]);
    launch_from_user(s, ga, c->n, c->id, u, reinterpret_cast<double4 *>(c->u_s));
    VjpArgs v{};
    v.f = force_args(c, p);
    v.u = reinterpret_cast<const double4 *>(c->u_s);
    v.vE = vE != nullptr ? vE : c->zeros_R;
    v.gx = c->gx_s;
    v.gpart = c->partial + (size_t)c->max_grid() * 12;
    v.rdot = c->rdot;
    v.fpp = c->fpp;
    v.stage_u = c->stage_u;
    const int gh = c->grid_tasks(0, true);
    if (p->kind == MD_POT_LJ) {
        v.gout = g_params;
        launch_lj_vjp(s, gh, c->threads, v, c->lds_max);
    } else {
        v.gtab = g_params;
        if (g_params != nullptr) {
            int64_t total = 4 * (int64_t)(p->phi.n_knots - 1) + 4 * (int64_t)(p->rho.n_knots - 1) +
                            4 * (int64_t)(p->embed.n_knots - 1);
            launch_zero(s, 64, g_params, total);
        }
        launch_eam_vjp_a(s, gh, c->threads, v, c->lds_max);
        launch_eam_vjp_b(s, gh, c->threads, v, c->lds_max, c->gwin_limit);
        if (g_params != nullptr) launch_eam_vjp_embed(s, ga, v, c->lds_max, c->gwin_limit);
    }
    if (g_pos != nullptr) launch_to_user(s, ga, c->n, c->id, c->gx_s, g_pos);
    return check_hip(c, "md_force_vjp");
}

int md_get_status(md_ctx *c, int32_t *flags, int64_t *required)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
    DevCtl h{};
    if (hipMemcpy(&h, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, MD_ERR_HIP, "status readback");
    if (h.err & MD_FLAG_OVERFLOW) c->need_M = std::max<int64_t>(c->need_M, (int64_t)ceil(1.25 * h.max_cnt));
    if (flags) *flags = h.err;
    if (required) *required = std::max<int64_t>(c->M, c->need_M);
    if (h.err != 0) {
        int32_t zero = 0;
        if (hipMemcpy(&c->ctl->err, &zero, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)
            return fail(c, MD_ERR_HIP, "status clear");
    }
    if (h.err & MD_FLAG_OVERFLOW) return fail(c, MD_ERR_CAPACITY, "neighbour list overflow");
    if (h.err & MD_FLAG_NONFINITE) return fail(c, MD_ERR_NONFINITE, "non-finite force");
    if (h.err & MD_FLAG_SCHEDULE) return fail(c, MD_ERR_TIMEOUT, "dependent schedule: a wait ran past its limit");
    return MD_OK;
}

int64_t md_get_neighbor_list(md_ctx *c, int64_t *start, int32_t *nbr, int64_t capacity)
{
    if (c == nullptr || start == nullptr) return MD_ERR_ARG;
    if (!c->have_list) return fail(c, MD_ERR_STATE, "no list");
    if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
    const int64_t n = c->n;
    const int32_t stride = c->bd.stride;
    std::vector<int32_t> cnt(n), id(n), rec((size_t)(c->B * stride));
    std::vector<uint32_t> words((size_t)(c->n64() * c->M));
    if (hipMemcpy(cnt.data(), c->cnt, sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(id.data(), c->id, sizeof(int32_t) * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(rec.data(), c->brec, sizeof(int32_t) * rec.size(), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(words.data(), c->nbr, sizeof(uint32_t) * words.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, MD_ERR_HIP, "list readback");
    std::vector<int64_t> len(n, 0);
    for (int64_t i = 0; i < n; i++) len[id[i]] = std::min<int64_t>(cnt[i], c->M);
    start[0] = 0;
    for (int64_t u = 0; u < n; u++) start[u + 1] = start[u] + len[u];
    const int64_t total = start[n];
    if (nbr == nullptr || total > capacity) return total;
    // every atom belongs to exactly one brick; its entries index that brick's halo
    for (int64_t b = 0; b < c->B; b++) {
        const int32_t *r = &rec[(size_t)(b * stride)];
        const int32_t H = r[BR_H], E = r[BR_E];
        const int32_t *soff = r + br_soff(c->bd), *sbeg = r + br_sbeg(c->bd);
        const int32_t *aoff = r + br_aoff(c->bd), *abeg = r + br_abeg(c->bd);
        const bool narrow = r[BR_SHIFT] != 0;
        const uint16_t *half = reinterpret_cast<const uint16_t *>(words.data());
        for (int32_t e = 0; e < E; e++)
            for (int32_t a = aoff[e]; a < aoff[e + 1]; a++) {
                const int64_t i = abeg[e] + (a - aoff[e]);
                const int64_t u = id[i];
                for (int64_t p = 0; p < len[u]; p++) {
                    const int32_t k = narrow ? (int32_t)half[(size_t)ell_half(i, p, c->M)]
                                             : (int32_t)(words[(size_t)ell_word(i, p, c->M)] & MD_IDX_MASK);
                    int32_t h = H - 1;
                    while (h > 0 && soff[h] > k) h--;
                    nbr[start[u] + p] = id[sbeg[h] + (k - soff[h])];
                }
            }
    }
    return total;
}

int md_get_cells(md_ctx *c, int32_t *cell_start, int32_t *order, int64_t *ncells)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (!c->have_cells) return fail(c, MD_ERR_STATE, "no cells");
    if (ncells) *ncells = c->C;
    if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
    if (cell_start && hipMemcpy(cell_start, c->start, sizeof(int32_t) * (c->C + 1), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, MD_ERR_HIP, "cells readback");
    if (order && hipMemcpy(order, c->id, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(c, MD_ERR_HIP, "order readback");
    return MD_OK;
}

int md_set_tuning(md_ctx *c, int32_t key, int32_t value)
{
    if (c == nullptr) return MD_ERR_ARG;
    // the largest record a brick of at most 64 cells can need
    const int64_t cap_max = (c->lds_max - 4096 - 4 * (int64_t)br_stride(512, 64)) / (int64_t)(4 * sizeof(double) + sizeof(uint16_t));
    if (key == 0 && value >= 64 && value <= 4096 && value % 64 == 0 && value <= cap_max) {
        // the list's entry format depends on which halos fit the stage
        c->cap = c->cap_list = value;
        c->cap_user = true;
        c->have_list = false;
        return MD_OK;
    }
    if (key == 1 && value >= 1 && value <= 8) {
        c->wgpc = value;
        return MD_OK;
    }
    if (key == 2 && value >= 1 && value <= 4096) {
        // fixed per-atom list capacity (tests of the overflow path force a small one)
        if (hipDeviceSynchronize() != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
        const int32_t m = (value + 7) / 8 * 8;
        if (!dalloc(&c->nbr, (size_t)m * (size_t)c->n64())) return fail(c, MD_ERR_HIP, "list: out of device memory");
        c->M = m;
        c->need_M = 0;
        c->have_list = false;
        return MD_OK;
    }
    if (key == 3) {
        const int32_t bx = value & 255, by = (value >> 8) & 255, bz = (value >> 16) & 255;
        if (value == 0) {
            c->bshape[0] = c->bshape[1] = c->bshape[2] = 0;
        } else {
            if (bx < 1 || by < 1 || bz < 1 || bx > 8 || by > 8 || bz > 8 || (value >> 24) != 0 ||
                bx * by * bz > 64 || (bx + 2) * (by + 2) * (bz + 2) > 512)
                return fail(c, MD_ERR_ARG, "tuning: brick shape needs 1..8 cells per axis, at most 64 cells");
            c->bshape[0] = bx;
            c->bshape[1] = by;
            c->bshape[2] = bz;
        }
        c->bricks_valid = false;
        c->have_list = false;
        return MD_OK;
    }
    if (key == 4 && (value == 0 || (value >= 128 && value <= TASK_MAX_THREADS && value % 64 == 0))) {
        c->threads_req = value;
        c->bricks_valid = false;
        c->have_list = false;
        return MD_OK;
    }
    if (key == 5 && value >= 0) {
        c->wait_us = value;
        return MD_OK;
    }
    if (key == 7 && value >= 0 && value <= 2) {
        c->sched_mode = value;
        return MD_OK;
    }
    if (key == 8 && value >= -1) {
        c->gwin_limit = value;
        return MD_OK;
    }
    if (key == 9 && (value == 0 || value == 1)) {
        c->stage_u = value;
        return MD_OK;
    }
    if (key == 6 && (value == 0 || value == 1)) {
        c->shell = value == 1;
        c->have_list = false;
        c->waves_valid = false;
        c->deps_valid = false;
        return MD_OK;
    }
    return fail(c, MD_ERR_ARG, "tuning: key 0 in 64..4096 (multiple of 64, within the LDS), key 1 in 1..8, key 2 in 1..4096, "
                               "key 3 a brick shape, key 4 threads per task (0 or 128..512, multiple of 64), "
                               "key 5 a wait limit >= 0 (microseconds), key 6 the half-list rule (0 or 1), "
                               "key 7 the brick schedule (0 auto, 1 static ranges, 2 queue), "
                               "key 8 the EAM adjoint's LDS intervals (>= -1), "
                               "key 9 adjoint partner values staged in LDS (0 or 1)");
}

int md_query(md_ctx *c, int32_t key, int64_t *value)
{
    if (c == nullptr || value == nullptr) return MD_ERR_ARG;
    switch (key) {
    case 0: *value = c->cap; return MD_OK;
    case 1: *value = c->wgpc; return MD_OK;
    case 2: *value = c->M; return MD_OK;
    case 3:
        *value = c->bricks_valid ? (int64_t)c->reps_h[0].bd[0] | (int64_t)c->reps_h[0].bd[1] << 8 |
                                       (int64_t)c->reps_h[0].bd[2] << 16
                                 : 0;
        return MD_OK;
    case 4: *value = c->threads; return MD_OK;
    case 5: *value = c->B; return MD_OK;
    case 6:
    case 7: {
        if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
        DevCtl h{};
        if (hipMemcpy(&h, c->ctl, sizeof(DevCtl), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, MD_ERR_HIP, "status readback");
        *value = key == 6 ? h.max_nbhd : h.max_brick;
        return MD_OK;
    }
    case 8: *value = c->lds_max; return MD_OK;
    case 9: *value = c->bricks_valid ? c->grid_tasks(0, false) : 0; return MD_OK;
    case 10: {
        if (!c->have_list) return fail(c, MD_ERR_STATE, "no list");
        if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
        std::vector<int32_t> cnt(c->n);
        if (hipMemcpy(cnt.data(), c->cnt, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, MD_ERR_HIP, "list length readback");
        int64_t t = 0;
        for (int32_t v : cnt) t += std::min(v, c->M);
        *value = t;
        return MD_OK;
    }
    case 11: *value = c->waves_valid ? c->ncol : 0; return MD_OK;
    case 12: *value = c->deps_valid ? (int64_t)c->dag_succ_h.size() : 0; return MD_OK;
    case 13: *value = c->shell ? 1 : 0; return MD_OK;
    case 14: *value = c->sched_mode == 2 || (c->sched_mode == 0 && c->sparse) ? 2 : 1; return MD_OK;
    case 15: {
        // entries of atoms in bricks whose list uses the 16-bit layout
        if (!c->have_list) return fail(c, MD_ERR_STATE, "no list");
        if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
        const int32_t stride = c->bd.stride;
        std::vector<int32_t> cnt(c->n), rec((size_t)(c->B * stride));
        if (hipMemcpy(cnt.data(), c->cnt, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(rec.data(), c->brec, sizeof(int32_t) * rec.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(c, MD_ERR_HIP, "list readback");
        int64_t t = 0;
        for (int64_t b = 0; b < c->B; b++) {
            const int32_t *r = &rec[(size_t)(b * stride)];
            if (r[BR_SHIFT] == 0) continue;
            const int32_t *aoff = r + br_aoff(c->bd), *abeg = r + br_abeg(c->bd);
            for (int32_t e = 0; e < r[BR_E]; e++)
                for (int32_t a = 0; a < aoff[e + 1] - aoff[e]; a++) t += std::min(cnt[(size_t)(abeg[e] + a)], c->M);
        }
        *value = t;
        return MD_OK;
    }
    case 16: *value = (int64_t)MD_NOALLOC_BYTES; return MD_OK;
    case 17: *value = c->cap_list; return MD_OK;
    default: return fail(c, MD_ERR_ARG, "query: key 0..17");
    }
}

int md_get_waves(md_ctx *c, int32_t *colour, int64_t capacity, int64_t *n_bricks)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (!c->waves_valid) return fail(c, MD_ERR_STATE, "no wave schedule (build an MD_LIST_WAVES or MD_LIST_DEPS list)");
    if (n_bricks != nullptr) *n_bricks = c->B;
    if (colour != nullptr) {
        if (capacity < c->B) return fail(c, MD_ERR_ARG, "colour array too small");
        std::copy(c->brick_colour.begin(), c->brick_colour.end(), colour);
    }
    return c->ncol;
}

int64_t md_get_task_graph(md_ctx *c, int32_t *succ_off, int32_t *succ, int64_t capacity)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (!c->deps_valid) return fail(c, MD_ERR_STATE, "no dependent schedule (build an MD_LIST_DEPS list)");
    const int64_t E = (int64_t)c->dag_succ_h.size();
    if (succ_off != nullptr) std::copy(c->dag_off_h.begin(), c->dag_off_h.end(), succ_off);
    if (succ != nullptr) {
        if (capacity < E) return fail(c, MD_ERR_ARG, "successor array too small");
        std::copy(c->dag_succ_h.begin(), c->dag_succ_h.end(), succ);
    }
    return E;
}

int md_profile(md_ctx *c, int32_t enable, double *force_ms, int64_t *force_n, double *list_ms,
               int64_t *list_n)
{
    if (c == nullptr) return MD_ERR_ARG;
    if (enable) {
        if (hipStreamSynchronize(c->last) != hipSuccess)
            return fail(c, MD_ERR_HIP, "synchronise");
        c->ev_force.clear();
        c->ev_force_kind.clear();
        c->ev_list.clear();
        c->ev_setup.clear();
        c->ev_loop.clear();
        c->prof_steps = 0;
        c->ev_used = 0;
        c->prof = true;
        c->prof_launches = enable != 2;
        return MD_OK;
    }
    c->prof = false;
    if (hipStreamSynchronize(c->last) != hipSuccess) return fail(c, MD_ERR_HIP, "synchronise");
    auto total = [](const std::vector<std::pair<hipEvent_t, hipEvent_t>> &v, double &ms) {
        ms = 0.0;
        for (auto &p : v) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, p.first, p.second) != hipSuccess) return false;
            ms += (double)t;
        }
        return true;
    };
    double fm = 0.0, lm = 0.0, sm = 0.0, pm = 0.0;
    if (!total(c->ev_force, fm) || !total(c->ev_list, lm) || !total(c->ev_setup, sm) || !total(c->ev_loop, pm))
        return fail(c, MD_ERR_HIP, "event timing");
    // force launches by kind
    double km[3] = {0.0, 0.0, 0.0};
    int64_t kn[3] = {0, 0, 0};
    for (size_t k = 0; k < c->ev_force.size(); k++) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, c->ev_force[k].first, c->ev_force[k].second) != hipSuccess)
            return fail(c, MD_ERR_HIP, "event timing");
        const int kind = k < c->ev_force_kind.size() ? c->ev_force_kind[k] : 0;
        km[kind] += (double)t;
        kn[kind] += 1;
    }
    c->detail[0] = pm;
    c->detail[1] = (double)c->prof_steps;
    c->detail[2] = sm;
    c->detail[3] = km[1];
    c->detail[4] = (double)kn[1];
    c->detail[5] = km[2];
    c->detail[6] = (double)kn[2];
    c->detail[7] = km[0];
    if (force_ms) *force_ms = fm;
    if (force_n) *force_n = (int64_t)c->ev_force.size();
    if (list_ms) *list_ms = lm;
    if (list_n) *list_n = (int64_t)c->ev_list.size();
    c->ev_force.clear();
    c->ev_force_kind.clear();
    c->ev_list.clear();
    c->ev_setup.clear();
    c->ev_loop.clear();
    c->prof_steps = 0;
    c->ev_used = 0;
    return MD_OK;
}

int md_profile_detail(md_ctx *c, double *out, int32_t n_out)
{
    if (c == nullptr || out == nullptr || n_out < 0) return MD_ERR_ARG;
    for (int32_t k = 0; k < n_out && k < 8; k++) out[k] = c->detail[k];
    return MD_OK;
}

const char *md_last_error(md_ctx *c)
{
    return c == nullptr ? "null context" : c->err.c_str();
}

} // extern "C"
