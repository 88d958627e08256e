// md_force.hip -- LJ and FS-EAM forces over Verlet lists, fused with velocity Verlet.
//
// Work decomposition: brick tasks (md_brick.h).  One lane owns one atom of its
// brick, walks the atom's list four entries at a time and reads every neighbour
// from the brick's halo staged in LDS; the atom's sums stay in the lane's
// registers.  With the full list every pair appears in both lists and each
// atom's force is written only by its own lane, so no particle is updated by
// two workers at once -- the invariant the cell-task schedule of Sec. II.A/II.B
// exists to guarantee, here obtained by ownership instead of by a dependent
// schedule.  The half-list kernel is the Newton-3 alternative (Sec. II.D.3) with
// binary64 atomics on the partner atom.
//
// The pair loop has no data-dependent branches: slots past the end of a list
// and pairs beyond the cutoff are computed and then masked, and the image shift
// is an addition of +-L or 0 (instantiated only for bricks that touch a box
// face).
//
// Precision (MIXED = false: all binary64):
//   displacement, image shift, r2 and the r2 < rc^2 test are always binary64;
//   with MIXED the pair scalar (LJ 24 eps (2 q12 - q6)/r2 and V; EAM table
//   polynomials) is evaluated in binary32, then projected and accumulated in
//   binary64.  The list build forms r2 operation by operation, as the
//   exhaustive definition does, so lists are exact; here r2 is formed with
//   fused multiply-adds and, in bricks staged through their cell images, from
//   the partner's pre-shifted position, so the cutoff test of a force call can
//   decide differently from the exhaustive one for a pair whose r2 lies within
//   a few roundings of rc^2 (either decision is a valid result; every other
//   pair is decided the same way).
//
// Integration (mode): once the atom's force is known, its lane applies the
// velocity-Verlet pieces of this atom (the per-particle loop of Sec. II.A) --
// the closing half kick of the current step, the kinetic energy, the opening
// half kick and drift of the next -- and flags a rebuild when the displacement
// since the last build exceeds skin/2.  Drifted positions go to a second buffer
// because other tasks still gather the current ones.
#include <math.h>

#include "md_brick.h"
#include "md_reduce.h"

namespace {

__device__ __forceinline__ int seg(double u, int nk)
{
    int k = (int)floor(u);
    k = k > nk - 2 ? nk - 2 : k;
    return k < 0 ? 0 : k;
}

// value and d/du of a binary64 table row at u = (x - x0)/h
__device__ __forceinline__ void spl64(const double *tab, double u, int nk, double &f, double &fu)
{
    const int k = seg(u, nk);
    const double t = u - (double)k;
    // (a 32-bit unsigned byte offset: one scalar base plus a vector offset)
    const double4 c = *reinterpret_cast<const double4 *>(reinterpret_cast<const char *>(tab) + (uint32_t)k * 32u);
    f = c.x + t * (c.y + t * (c.z + t * c.w));
    fu = c.y + t * (2.0 * c.z + 3.0 * t * c.w);
}

// the same in binary32 throughout (the mixed path's pair tables): truncation
// picks the same segment as floor once clamped to [0, nk-2]
__device__ __forceinline__ void spl32f(const float *tab, float u, int nk, float &f, float &fu)
{
    // (u clamped to [0, nk-2] by one median-of-three, then truncated)
    const int k = (int)__builtin_amdgcn_fmed3f(u, 0.0f, (float)(nk - 2));
    const float t = u - (float)k;
    const float4 c = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(tab) + (uint32_t)k * 16u);
    f = c.x + t * (c.y + t * (c.z + t * c.w));
    fu = c.y + t * (2.0f * c.z + 3.0f * t * c.w);
}

// embedding function F(rho), F'(rho), binary64, linear beyond the last knot
__device__ __forceinline__ void embed64(const ForceArgs &a, double rho, double &F, double &Fp)
{
    const int nk = a.nk[2];
    const double u = (rho - a.x0[2]) * a.inv_h[2];
    const double4 *rows = reinterpret_cast<const double4 *>(a.tab[2]);
    if (u > (double)(nk - 1)) {
        const double4 c = rows[nk - 2];
        const double fend = ((c.x + c.y) + c.z) + c.w;
        const double sl = (c.y + 2.0 * c.z) + 3.0 * c.w;
        F = fend + sl * (u - (double)(nk - 1));
        Fp = sl * a.inv_h[2];
        return;
    }
    double fu;
    spl64(a.tab[2], u, nk, F, fu);
    Fp = fu * a.inv_h[2];
}

// Per-atom epilogue, run by the atom's lane.
__device__ __forceinline__ void finish_atom(const ForceArgs &a, int64_t i, const double4 &xi,
                                            double fx, double fy, double fz, double e, double w,
                                            double &accE, double &accW, double &accK,
                                            bool write_f = true)
{
    const int64_t n = a.n;
    if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicOr(&a.ctl->err, MD_FLAG_NONFINITE);
    if (a.mode == 0) {
        if (write_f && a.force != nullptr) {
            a.force[i] = fx;
            a.force[n + i] = fy;
            a.force[2 * n + i] = fz;
        }
        if (a.eatom != nullptr) {
            a.eatom[i] = e;
            a.watom[i] = w;
        }
        accE += e;
        accW += w;
        return;
    }
    const double c = a.cdt;
    double vx = a.vel[i], vy = a.vel[n + i], vz = a.vel[2 * n + i];
    if (a.mode >= 2) {
        vx = vx + c * fx;
        vy = vy + c * fy;
        vz = vz + c * fz;
        accK += (vx * vx + vy * vy) + vz * vz;
        accE += e;
        accW += w;
    }
    if (a.mode <= 2) {
        vx = vx + c * fx;
        vy = vy + c * fy;
        vz = vz + c * fz;
        const double4 xn = make_double4(xi.x + a.dt * vx, xi.y + a.dt * vy, xi.z + a.dt * vz, 0.0);
        a.pos_next[i] = xn;
        const double4 xr = a.xref[i];
        const double dx = xn.x - xr.x, dy = xn.y - xr.y, dz = xn.z - xr.z;
        if ((dx * dx + dy * dy) + dz * dz > a.thr2) *a.flag_set = 1;
    }
    a.vel[i] = vx;
    a.vel[n + i] = vy;
    a.vel[2 * n + i] = vz;
    if (a.mode == 3 && write_f && a.force != nullptr) {
        a.force[i] = fx;
        a.force[n + i] = fy;
        a.force[2 * n + i] = fz;
    }
}

// workgroup sums of E, W and 2 KE, then the launch totals in workgroup order
// (the bricks of a workgroup are fixed by the cost prefix, so the totals are
// bitwise repeatable for a given list and grid)
__device__ __forceinline__ void finish_block(const ForceArgs &a, double accE, double accW,
                                             double accK, double *lds)
{
    if (a.outE == nullptr && a.outK == nullptr && a.outW == nullptr) return;
    double v[4] = {accE, accW, accK, 0.0};
    mdred::block_to_partial4(v, a.partial, lds);
}

// ---------------------------------------------------------------- LJ pair scalar
// f_s = 24 eps (2 q12 - q6) / r2 and V = 4 eps (q12 - q6), q6 = (sigma^2/r2)^3.
// Outside the cutoff (or for an empty slot) 1/r2 is replaced by 0, which makes
// both exactly zero without further selects.  V only if EN (the force does not
// depend on it).
template <bool MIXED, bool EN = true>
__device__ __forceinline__ void lj_pair(bool in, double r2, double s2, double e4, double e24, float s2f,
                                        float e4f, float e24f, double &fs, double &V)
{
    if (MIXED) {
        const float ir2 = in ? __builtin_amdgcn_rcpf((float)r2) : 0.0f;
        const float q2 = s2f * ir2;
        const float q6 = q2 * q2 * q2;
        const float q12 = q6 * q6;
        fs = (double)(e24f * __builtin_fmaf(2.0f, q12, -q6) * ir2);
        V = EN ? (double)(e4f * (q12 - q6)) : 0.0;
    } else {
        const double ir2 = in ? rcp64(r2) : 0.0;
        const double q2 = s2 * ir2;
        const double q6 = q2 * q2 * q2;
        const double q12 = q6 * q6;
        fs = e24 * (2.0 * q12 - q6) * ir2;
        V = e4 * (q12 - q6);
    }
}

// The LJ pair without its energy scale: fs / (24 eps) and V / (4 eps), for
// sums that take the scale once per atom.
template <bool MIXED, bool EN = true>
__device__ __forceinline__ void lj_pair_unit(bool in, double r2, double s2, float s2f, double &fs, double &V)
{
    if (MIXED) {
        const float ir2 = in ? __builtin_amdgcn_rcpf((float)r2) : 0.0f;
        const float q2 = s2f * ir2;
        const float q6 = q2 * q2 * q2;
        const float q12 = q6 * q6;
        fs = (double)(__builtin_fmaf(2.0f, q12, -q6) * ir2);
        V = EN ? (double)(q12 - q6) : 0.0;
    } else {
        const double ir2 = in ? rcp64(r2) : 0.0;
        const double q2 = s2 * ir2;
        const double q6 = q2 * q2 * q2;
        const double q12 = q6 * q6;
        fs = (2.0 * q12 - q6) * ir2;
        V = q12 - q6;
    }
}

// ---------------------------------------------------------------- LJ, full list
// EN: the launch returns energy or virial (steps that record no energy skip
// their per-pair terms).  An atom's sums are taken without the energy scale,
// which multiplies them once at the end (24 eps for force and virial, 4 eps
// for the energy).
template <bool MIXED, bool EN>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_lj_full(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    const Stage st = stage_slice(lds_raw, a.cap, 0, false);
    if (a.flag_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.flag_clear = 0;
    const double eps = a.lj[0], sig = a.lj[1];
    const double s2 = sig * sig, e4 = 4.0 * eps, e24 = 24.0 * eps;
    const float s2f = (float)s2;
    const double rc2 = a.rc2;
    double accE = 0.0, accW = 0.0, accK = 0.0;
    BRICK_TASK_BEGIN(st, a.pos, nullptr, nullptr)
        double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, w = 0.0;
        const double4 xi = a.pos[i];
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG, true>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t, double dx, double dy, double dz, double r2) {
                    double fs, V;
                    lj_pair_unit<MIXED, EN>(ok && r2 < rc2, r2, s2, s2f, fs, V);
                    fx = fma(fs, dx, fx);
                    fy = fma(fs, dy, fy);
                    fz = fma(fs, dz, fz);
                    if (EN) {
                        e += V;
                        w += fs * r2;
                    }
                });
        )
        if (valid)
            finish_atom(a, i, xi, e24 * fx, e24 * fy, e24 * fz, (0.5 * e4) * e, (0.5 * e24) * w, accE, accW, accK);
    BRICK_TASK_END
    finish_block(a, accE, accW, accK, lds);
}

// ---------------------------------------------------------------- LJ, half list + atomics
template <bool MIXED>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_lj_half(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    const Stage st = stage_slice(lds_raw, a.cap, 0, true);
    const double eps = a.lj[0], sig = a.lj[1];
    const double s2 = sig * sig, e4 = 4.0 * eps, e24 = 24.0 * eps;
    const float s2f = (float)s2, e4f = (float)e4, e24f = (float)e24;
    const double rc2 = a.rc2;
    const int64_t n = a.n;
    double accE = 0.0, accW = 0.0;
    BRICK_TASK_BEGIN(st, a.pos, nullptr, nullptr)
        double fx = 0.0, fy = 0.0, fz = 0.0;
        const double4 xi = a.pos[i];
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    const bool in = ok && r2 < rc2;
                    double fs, V;
                    lj_pair<MIXED>(in, r2, s2, e4, e24, s2f, e4f, e24f, fs, V);
                    const double px = fs * dx, py = fs * dy, pz = fs * dz;
                    fx += px;
                    fy += py;
                    fz += pz;
                    if (in) {
                        const int32_t j = candidate_j<STAGED>(st, a.bd, k);
                        atomicAdd(&a.force[j], -px);
                        atomicAdd(&a.force[n + j], -py);
                        atomicAdd(&a.force[2 * n + j], -pz);
                    }
                    accE += V;
                    accW += fs * r2;
                });
        )
        if (valid) {
            atomicAdd(&a.force[i], fx);
            atomicAdd(&a.force[n + i], fy);
            atomicAdd(&a.force[2 * n + i], fz);
        }
    BRICK_TASK_END
    finish_block(a, accE, accW, 0.0, lds);
}

// One half-list brick task: stages the halo with a sorted index and three
// binary64 partner-force sums per candidate, walks the brick's lists (own force
// in registers, -f of each pair added to the partner's LDS sums with binary64
// LDS atomics between the lanes of the workgroup), then adds every non-zero
// sum to its atom's force in HBM with plain loads and stores.  Correct only while no
// other task that writes the same atoms runs at the same time (the callers'
// schedules guarantee it).  Candidates past the LDS stage take global atomics.
// Energy and virial are per atom (the pairs an atom holds).  Begins with a
// barrier, so consecutive calls may reuse the stage.
template <bool MIXED>
__device__ __forceinline__ void lj_half_task(const ForceArgs &a, const Stage &st, int64_t b)
{
    const double eps = a.lj[0], sig = a.lj[1];
    const double s2 = sig * sig, e4 = 4.0 * eps, e24 = 24.0 * eps;
    const float s2f = (float)s2, e4f = (float)e4, e24f = (float)e24;
    const double rc2 = a.rc2;
    const int64_t n = a.n;
    const int32_t cap = a.cap;
    double *sx = st.ex, *sy = st.ex + cap, *sz = st.ex + 2 * (size_t)cap;
    const int32_t *grec = a.brec + b * (int64_t)a.bd.stride;
    const int32_t natoms = __builtin_amdgcn_readfirstlane(grec[BR_ATOMS]);
    if (natoms == 0) return;
    __syncthreads();
    brick_load(st, a.bd, grec, a.reps, a.pos, nullptr, nullptr);
    const int32_t total = st.rec[BR_TOTAL];
    const int32_t lim = total < cap ? total : cap;
    for (int32_t k = threadIdx.x; k < lim; k += blockDim.x) {
        sx[k] = 0.0;
        sy[k] = 0.0;
        sz[k] = 0.0;
    }
    __syncthreads();
    const bool all_staged = total <= cap;
    const bool has_img = st.rec[BR_SHIFT] == 0;
    const RepDesc &rep = a.reps[st.rec[BR_REP]];
    const double Lx = rep.L[0], Ly = rep.L[1], Lz = rep.L[2];
    const BrickGeom g = brick_geom(a.reps, a.R, b);
    const int32_t *soff = st.rec + br_soff(a.bd), *aoff = st.rec + br_aoff(a.bd);
    auto add_to = [&](int32_t k, double fx, double fy, double fz) {
        if (k < cap) {
            atomicAdd(&sx[k], fx);
            atomicAdd(&sy[k], fy);
            atomicAdd(&sz[k], fz);
        } else {
            const int32_t j = candidate_index(st, a.bd, k);
            atomicAdd(&a.force[j], fx);
            atomicAdd(&a.force[n + j], fy);
            atomicAdd(&a.force[2 * n + j], fz);
        }
    };
    for (int32_t a0 = 0; a0 < natoms; a0 += (int32_t)blockDim.x) {
        const int32_t la = a0 + (int32_t)threadIdx.x;
        const bool valid = la < natoms;
        int32_t e = 0;
        const int64_t i = valid ? brick_atom(st, a.bd, la, &e) : 0;
        const int32_t mm = valid ? min(a.cnt[i], a.M) : 0;
        double fx = 0.0, fy = 0.0, fz = 0.0, en = 0.0, w = 0.0;
        const double4 xi = a.pos[i];
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    const bool in = ok && r2 < rc2;
                    double fs, V;
                    lj_pair<MIXED>(in, r2, s2, e4, e24, s2f, e4f, e24f, fs, V);
                    const double px = fs * dx, py = fs * dy, pz = fs * dz;
                    fx += px;
                    fy += py;
                    fz += pz;
                    if (in) add_to(k, -px, -py, -pz);
                    en += V;
                    w += fs * r2;
                });
        )
        if (valid) {
            // the atom's own candidate slot: its cell's first candidate plus its rank in the cell
            const int32_t lc0 = e % g.e[0], lc1 = (e / g.e[0]) % g.e[1], lc2 = e / (g.e[0] * g.e[1]);
            const int32_t hown = (lc0 + 1) % g.nc[0] + g.hn[0] * ((lc1 + 1) % g.nc[1] + g.hn[1] * ((lc2 + 1) % g.nc[2]));
            add_to(soff[hown] + (la - aoff[e]), fx, fy, fz);
            if (a.eatom != nullptr) {
                a.eatom[i] = en;
                a.watom[i] = w;
            }
        }
    }
    __syncthreads();
    // only atoms the task changed are stored: a halo atom that is no partner of
    // the brick's atoms (the layer below, with the 14-cell half list) may be
    // written by a task running at the same time
    for (int32_t k = threadIdx.x; k < lim; k += blockDim.x) {
        const double fx = sx[k], fy = sy[k], fz = sz[k];
        if (fx == 0.0 && fy == 0.0 && fz == 0.0) continue;
        const int32_t j = st.j[k];
        a.force[j] += fx;
        a.force[n + j] += fy;
        a.force[2 * n + j] += fz;
    }
}

// ---------------------------------------------------------------- LJ, half list in waves
// One launch per wave of bricks whose write sets (own cells plus one layer)
// are disjoint (the appendix's construction on the brick grid): no two tasks
// of a launch write the same atom.
template <bool MIXED>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_lj_wave(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Stage st = stage_slice(lds_raw, a.cap, 3, true);    // extras: partner sums x, y, z
    for (int32_t t = blockIdx.x; t < a.nwb; t += gridDim.x) lj_half_task<MIXED>(a, st, a.wbr[t]);
}

// ---------------------------------------------------------------- LJ, half list in dependence order
// The tasks of all waves in one persistent launch (Sec. II.B's dependent
// schedule): a task starts once its direct predecessors (the last earlier
// writer of each of its cells, in wave order) have finished.  Ready tasks go
// through a queue of n_tasks slots: workgroups take slots in order
// (d.sched[0]) and wait until the slot is filled; a finished task decrements
// its successors' counts and appends each that reaches zero (d.sched[1]).  The
// tasks with no predecessor are in the queue at the start.  Since the graph is
// acyclic and every taken slot belongs to a running workgroup, every slot is
// filled while tasks keep finishing; a wait longer than d.limit wall-clock
// ticks (a broken graph) raises MD_FLAG_SCHEDULE and the abort word, and every
// workgroup then leaves.  A task's plain stores reach other XCDs through an
// agent-scope release before its successors are counted down, and the task
// that takes a slot performs an agent-scope acquire before it reads them.
// Thread 0: takes the next queue slot and waits (bounded) until a task is in
// it; returns the task, or -1 when the queue is used up, the abort word is set
// or the wait ran past the limit (which sets the flag and the abort word).
__device__ __forceinline__ int32_t take_task(const ForceArgs &a, const DepArgs &d)
{
    const int32_t q = __hip_atomic_fetch_add(&d.sched[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (q >= d.T) return -1;
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const int32_t t = __hip_atomic_load(&d.queue[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (t >= 0) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return t;
        }
        if (__hip_atomic_load(&d.sched[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return -1;
        if ((uint64_t)wall_clock64() - t0 > d.limit) {
            atomicOr(&a.ctl->err, MD_FLAG_SCHEDULE);
            __hip_atomic_store(&d.sched[2], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return -1;
        }
        __builtin_amdgcn_s_sleep(16);
    }
}

// Thread 0, after task t (every wavefront's stores of the task have
// completed): one agent-scope release writes the task's stores back from this
// XCD's L2, then the successors are counted down and each that reaches zero is
// appended to the queue.  Every predecessor of a task has written its stores
// back before its own count-down, so the task that takes the slot finds all of
// them in memory after its acquire; the slot itself needs no further release.
__device__ __forceinline__ void finish_task(const DepArgs &d, int32_t t)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    for (int32_t e = d.off[t]; e < d.off[t + 1]; e++) {
        const int32_t u = d.succ[e];
        if (__hip_atomic_fetch_add(&d.ref[u], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1) {
            const int32_t slot = __hip_atomic_fetch_add(&d.sched[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // a task reaches zero once, so at most T - roots slots are filled
            if (slot < d.T) __hip_atomic_store(&d.queue[slot], u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// The loop is kept uniform for the compiler: thread 0 does all of the queue
// work between two barriers and the task index reaches the other lanes
// through LDS and readfirstlane, so the loop branch is scalar (a branch the
// compiler must treat as divergent lets it split the loop per lane and run
// the next barrier without thread 0).
template <bool MIXED>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_lj_deps(ForceArgs a, DepArgs d)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_task;
    const Stage st = stage_slice(lds_raw, a.cap, 3, true);
    if (threadIdx.x == 0) s_task = take_task(a, d);
    __syncthreads();
    int32_t t = __builtin_amdgcn_readfirstlane(s_task);
    while (t >= 0) {
        lj_half_task<MIXED>(a, st, t);
        // every wavefront waits until its stores have reached the L2, so that
        // thread 0's write-back covers the whole task
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            finish_task(d, t);
            s_task = take_task(a, d);
        }
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_task);
    }
}

// Working state of a dependent-schedule launch: reference counts from the
// predecessor counts, the queue holding the tasks without predecessors (in
// wave order) and empty slots, both slot counters and the abort word cleared.
__global__ __launch_bounds__(256) void k_deps_init(int32_t T, const int32_t *__restrict__ npred,
                                                   const int32_t *__restrict__ init_q, int32_t nroots,
                                                   int32_t *ref, int32_t *queue, int32_t *sched)
{
    for (int32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < T; t += gridDim.x * blockDim.x) {
        ref[t] = npred[t];
        queue[t] = init_q[t];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sched[0] = 0;
        sched[1] = nroots;
        sched[2] = 0;
        sched[3] = 0;
    }
}

// E and W summed over all atoms: per-workgroup partials over fixed strided
// ranges (added in workgroup order by k_sum_partials; fixed grid, so the sums
// are bitwise repeatable)
__global__ __launch_bounds__(256) void k_atom_sums(int64_t n, const double *__restrict__ eatom,
                                                   const double *__restrict__ watom, double *partial)
{
    __shared__ double lds[4 * 256 / 64];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        v[0] += eatom[i];
        v[1] += watom[i];
    }
    mdred::block_to_partial4(v, partial, lds);
}

// The totals of a launch's per-workgroup partials (g workgroups), added in
// workgroup order by one workgroup of the producing launch's size: o[c] =
// scale[c] * total c where o[c] is given.
__global__ __launch_bounds__(1024) void k_sum_partials(const double *__restrict__ partial, int32_t g, SumOut o)
{
    __shared__ double lds[4 * 1024 / 64];
    double v[4];
    mdred::sum_partials4(partial, g, v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; c++)
            if (o.out[c] != nullptr) *o.out[c] = o.scale[c] * v[c];
}

// velocity-Verlet pieces for forces already in a.force (half-list path); the
// consumed forces are cleared for the next atomic accumulation
__global__ __launch_bounds__(256) void k_integrate(ForceArgs a)
{
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    if (a.flag_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.flag_clear = 0;
    const int64_t n = a.n;
    double accE = 0.0, accW = 0.0, accK = 0.0;
    const int64_t ntiles = (n + 255) / 256;
    const ItemRange it = xcd_items(ntiles, 1, 0);
    for (int64_t t = it.first; t < it.end; t += it.stride) {
        const int64_t i = t * 256 + threadIdx.x;
        if (i >= n) continue;
        const double fx = a.force[i], fy = a.force[n + i], fz = a.force[2 * n + i];
        const double4 xi = a.pos[i];
        finish_atom(a, i, xi, fx, fy, fz, 0.0, 0.0, accE, accW, accK, false);
        if (a.mode != 3) {
            a.force[i] = 0.0;
            a.force[n + i] = 0.0;
            a.force[2 * n + i] = 0.0;
        }
    }
    double v[4] = {0.0, 0.0, accK, 0.0};
    if (a.outK == nullptr) return;
    mdred::block_to_partial4(v, a.partial, lds);
}

// ---------------------------------------------------------------- EAM pass 1: density
template <bool MIXED>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_eam_density(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Stage st = stage_slice(lds_raw, a.cap, 0, false);
    const int nk = a.nk[1];
    const double x0 = a.x0[1], ih = a.inv_h[1], rrho2 = a.rrho2;
    const float x0f = (float)x0, ihf = (float)ih;
    // the mixed path reads its binary32 density table from LDS when it fits
    // beside the stage (a.lds_tab), else from global memory
    float4 *ltab = reinterpret_cast<float4 *>(lds_raw + stage_bytes(a.cap, 0, false, a.bd.stride));
    const bool lt = MIXED && a.lds_tab != 0;
    if (lt) {
        const float4 *g = reinterpret_cast<const float4 *>(a.tabf[1]);
        for (int32_t t = threadIdx.x; t < nk - 1; t += blockDim.x) ltab[t] = g[t];
        __syncthreads();
    }
    BRICK_TASK_BEGIN(st, a.pos, nullptr, nullptr)
        double rho = 0.0;
        const double4 xi = a.pos[i];
        // the pair loop once per table location, so that each copy reads its
        // table through one address space (LDS or global, never flat)
        auto pairs = [&](const float *tabf) __attribute__((always_inline)) {
            STAGE_IMG_SPLIT(all_staged, has_img,
                walk_list<STAGED, IMG, true>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                    [&](bool ok, int32_t, double, double, double, double r2) {
                        const bool in = ok && r2 < rrho2;
                        double f;
                        if (MIXED) {
                            // r (hardware square root) and the table argument in
                            // binary32, like the table
                            float ff, fu;
                            const float uf = (__builtin_amdgcn_sqrtf((float)r2) - x0f) * ihf;
                            spl32f(tabf, uf, nk, ff, fu);
                            f = (double)ff;
                        } else {
                            double fu;
                            spl64(a.tab[1], (sqrt_pair(r2) - x0) * ih, nk, f, fu);
                        }
                        rho += in ? f : 0.0;
                    });
            )
        };
        if (lt) pairs(reinterpret_cast<const float *>(ltab));
        else pairs(a.tabf[1]);
        if (valid) {
            double F, Fp;
            embed64(a, rho, F, Fp);
            a.rho[i] = rho;
            a.fp[i] = Fp;
        }
    BRICK_TASK_END
}

// ---------------------------------------------------------------- EAM pass 2: forces
// EN: the launch returns energy or virial (steps that record no energy skip
// their per-pair terms).  The mixed pass is held to 128 VGPRs, so that two
// 512-thread workgroups share a CU (the few spills this costs are per atom,
// outside the pair loop); the binary64 passes would spill inside the pair loop
// at that bound (81 VGPRs without energies: 224 MB of scratch writes per launch
// on the replica batch) and run one workgroup per CU instead (7 % faster).
template <bool MIXED, bool EN>
__global__ __launch_bounds__(TASK_MAX_THREADS, MIXED ? 4 : 1) void k_eam_force(ForceArgs a)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    const Stage st = stage_slice(lds_raw, a.cap, 1, false);
    if (a.flag_clear != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *a.flag_clear = 0;
    const int nkp = a.nk[0], nkr = a.nk[1];
    const double x0p = a.x0[0], ihp = a.inv_h[0], x0r = a.x0[1], ihr = a.inv_h[1];
    const float x0pf = (float)x0p, ihpf = (float)ihp, x0rf = (float)x0r, ihrf = (float)ihr;
    const double rphi2 = a.rphi2, rrho2 = a.rrho2;
    double accE = 0.0, accW = 0.0, accK = 0.0;
    BRICK_TASK_BEGIN(st, a.pos, a.fp, nullptr)
        double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0, w = 0.0;
        const double4 xi = a.pos[i];
        const double fpi = a.fp[i];
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    const bool in_phi = ok && r2 < rphi2, in_rho = ok && r2 < rrho2;
                    const double fpj = (STAGED || k < st.cap) ? st.ex[k] : a.fp[candidate_index(st, a.bd, k)];
                    double gsc, grr, ep, r;
                    if (MIXED) {
                        // pair scalar in binary32 (r, table arguments, dV/dr / r with
                        // the binary32 reciprocal); r2 and the cutoff tests stay binary64
                        const float rf = __builtin_amdgcn_sqrtf((float)r2);
                        float f, fu, g, h;
                        spl32f(a.tabf[0], (rf - x0pf) * ihpf, nkp, f, fu);
                        spl32f(a.tabf[1], (rf - x0rf) * ihrf, nkr, g, h);
                        const float gp = in_phi ? fu * ihpf : 0.0f;
                        const float gr = in_rho ? (float)(fpi + fpj) * h * ihrf : 0.0f;
                        const float gsf = gp + gr;
                        gsc = (double)gsf;
                        grr = (double)(gsf * __builtin_amdgcn_rcpf(rf));
                        ep = in_phi ? (double)f : 0.0;
                        r = (double)rf;
                    } else {
                        r = sqrt_pair(r2);
                        double f, fu, g, h;
                        spl64(a.tab[0], (r - x0p) * ihp, nkp, f, fu);
                        spl64(a.tab[1], (r - x0r) * ihr, nkr, g, h);
                        const double gp = in_phi ? fu * ihp : 0.0;
                        const double gr = in_rho ? (fpi + fpj) * (h * ihr) : 0.0;
                        gsc = gp + gr;
                        grr = (in_phi || in_rho) ? gsc * rcp64(r) : 0.0;
                        ep = in_phi ? f : 0.0;
                    }
                    fx = fma(-grr, dx, fx);
                    fy = fma(-grr, dy, fy);
                    fz = fma(-grr, dz, fz);
                    if (EN) {
                        e += ep;
                        w -= (in_phi || in_rho) ? gsc * r : 0.0;
                    }
                });
        )
        if (valid) {
            double F, Fp;
            embed64(a, a.rho[i], F, Fp);
            finish_atom(a, i, xi, fx, fy, fz, F + 0.5 * e, 0.5 * w, accE, accW, accK);
        }
    BRICK_TASK_END
    finish_block(a, accE, accW, accK, lds);
}

// ---------------------------------------------------------------- small kernels
__global__ void k_zero(double *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

__global__ void k_to_user(int64_t n, const int32_t *__restrict__ id, const double *__restrict__ src,
                          double *__restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = id[i];
        dst[u] = src[i];
        dst[n + u] = src[n + i];
        dst[2 * n + u] = src[2 * n + i];
    }
}

// user-ordered [3][n] -> sorted (x, y, z, 0) per atom: a kernel that gathers
// the vector of a partner reads one 32-byte record instead of three arrays
__global__ void k_from_user(int64_t n, const int32_t *__restrict__ id, const double *__restrict__ src,
                            double4 *__restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = id[i];
        dst[i] = make_double4(src[u], src[n + u], src[2 * n + u], 0.0);
    }
}

__device__ __forceinline__ double wrap1(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w >= L) w = w - L;
    if (w < 0.0) w = 0.0;
    return w;
}

__global__ void k_pos_to_user(int64_t n, const RepDesc *__restrict__ reps,
                              const int32_t *__restrict__ rep_of, const int32_t *__restrict__ id,
                              const double4 *__restrict__ pos, double *__restrict__ dst)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const RepDesc &r = reps[rep_of[i]];
        const double4 p = pos[i];
        const int64_t u = id[i];
        dst[u] = wrap1(p.x, r.L[0]);
        dst[n + u] = wrap1(p.y, r.L[1]);
        dst[2 * n + u] = wrap1(p.z, r.L[2]);
    }
}

__global__ void k_tables_f32(const double *__restrict__ src, float *__restrict__ dst, int64_t m)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

// per-replica energy and virial in a fixed order: one workgroup per replica
__global__ __launch_bounds__(256) void k_replica_sums(const RepDesc *__restrict__ reps,
                                                      const double *__restrict__ eatom,
                                                      const double *__restrict__ watom,
                                                      double *energy, double *virial)
{
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    const RepDesc &r = reps[blockIdx.x];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = r.atom_off + threadIdx.x; i < r.atom_end; i += blockDim.x) {
        v[0] += eatom[i];
        v[1] += watom[i];
    }
    mdred::block_sum4(v, lds);
    if (threadIdx.x == 0) {
        if (energy) energy[blockIdx.x] = v[0];
        if (virial) virial[blockIdx.x] = v[1];
    }
}

#define MD_LAUNCH_TASKS(KERNEL, NEXTRA, WITH_J)                                          \
    const size_t lds = stage_bytes(a.cap, NEXTRA, WITH_J, a.bd.stride);                    \
    int used_ = 0;                                                                          \
    if (mixed) {                                                                            \
        allow_lds(KERNEL<true>, lds);                                                       \
        used_ = resident_grid(KERNEL<true>, grid, threads, lds);                            \
        hipLaunchKernelGGL((KERNEL<true>), dim3(used_), dim3(threads), lds, s, a);          \
    } else {                                                                                \
        allow_lds(KERNEL<false>, lds);                                                      \
        used_ = resident_grid(KERNEL<false>, grid, threads, lds);                           \
        hipLaunchKernelGGL((KERNEL<false>), dim3(used_), dim3(threads), lds, s, a);         \
    }

// the energy, virial and kinetic-energy totals of a force launch of g workgroups
void finish_sums(hipStream_t s, const ForceArgs &a, int g, int threads)
{
    if (a.outE == nullptr && a.outW == nullptr && a.outK == nullptr) return;
    launch_sum_partials(s, a.partial, g, threads, SumOut{{a.outE, a.outW, a.outK, nullptr}, {1.0, 1.0, 0.5 * a.mass, 0.0}});
}

} // namespace

void launch_lj_full(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a)
{
    const size_t lds = stage_bytes(a.cap, 0, false, a.bd.stride);
    const bool en = a.outE != nullptr || a.outW != nullptr || a.eatom != nullptr;
    int used = 0;
    auto go = [&](auto kernel) {
        allow_lds(kernel, lds);
        used = resident_grid(kernel, grid, threads, lds);
        hipLaunchKernelGGL(kernel, dim3(used), dim3(threads), lds, s, a);
    };
    if (mixed) {
        if (en) go(k_lj_full<true, true>);
        else go(k_lj_full<true, false>);
    } else {
        if (en) go(k_lj_full<false, true>);
        else go(k_lj_full<false, false>);
    }
    finish_sums(s, a, used, threads);
}

void launch_lj_half(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a)
{
    MD_LAUNCH_TASKS(k_lj_half, 0, true)
    finish_sums(s, a, used_, threads);
}

void launch_eam_density(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a)
{
    const size_t lds = stage_bytes(a.cap, 0, false, a.bd.stride) + (mixed && a.lds_tab ? (size_t)(a.nk[1] - 1) * 16 : 0);
    if (mixed) {
        allow_lds(k_eam_density<true>, lds);
        hipLaunchKernelGGL((k_eam_density<true>), dim3(resident_grid(k_eam_density<true>, grid, threads, lds)),
                           dim3(threads), lds, s, a);
    } else {
        allow_lds(k_eam_density<false>, lds);
        hipLaunchKernelGGL((k_eam_density<false>), dim3(resident_grid(k_eam_density<false>, grid, threads, lds)),
                           dim3(threads), lds, s, a);
    }
}

void launch_eam_force(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a)
{
    const size_t lds = stage_bytes(a.cap, 1, false, a.bd.stride);
    const bool en = a.outE != nullptr || a.outW != nullptr || a.eatom != nullptr;
    int used = 0;
    auto go = [&](auto kernel) {
        allow_lds(kernel, lds);
        used = resident_grid(kernel, grid, threads, lds);
        hipLaunchKernelGGL(kernel, dim3(used), dim3(threads), lds, s, a);
    };
    if (mixed) {
        if (en) go(k_eam_force<true, true>);
        else go(k_eam_force<true, false>);
    } else {
        if (en) go(k_eam_force<false, true>);
        else go(k_eam_force<false, false>);
    }
    finish_sums(s, a, used, threads);
}

void launch_lj_wave(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a)
{
    MD_LAUNCH_TASKS(k_lj_wave, 3, true)
}

void launch_lj_deps(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a, const DepArgs &d,
                    const int32_t *npred, const int32_t *init_q, int32_t nroots)
{
    hipLaunchKernelGGL(k_deps_init, dim3((d.T + 255) / 256), dim3(256), 0, s, d.T, npred, init_q, nroots, d.ref,
                       d.queue, d.sched);
    const size_t lds = stage_bytes(a.cap, 3, true, a.bd.stride);
    auto go = [&](auto kernel) {
        allow_lds(kernel, lds);
        hipLaunchKernelGGL(kernel, dim3(resident_grid(kernel, grid, threads, lds)), dim3(threads), lds, s, a, d);
    };
    if (mixed) go(k_lj_deps<true>);
    else go(k_lj_deps<false>);
}

void launch_atom_sums(hipStream_t s, int grid, int64_t n, const double *eatom, const double *watom,
                      double *energy, double *virial, double *partial)
{
    hipLaunchKernelGGL(k_atom_sums, dim3(grid), dim3(256), 0, s, n, eatom, watom, partial);
    launch_sum_partials(s, partial, grid, 256, SumOut{{energy, virial, nullptr, nullptr}, {1.0, 1.0, 0.0, 0.0}});
}

void launch_integrate(hipStream_t s, int grid, const ForceArgs &a)
{
    hipLaunchKernelGGL(k_integrate, dim3(grid), dim3(256), 0, s, a);
    finish_sums(s, a, grid, 256);
}

void launch_sum_partials(hipStream_t s, const double *partial, int g, int threads, SumOut o)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(threads), 0, s, partial, (int32_t)g, o);
}

void launch_zero(hipStream_t s, int grid, double *p, int64_t n)
{
    hipLaunchKernelGGL(k_zero, dim3(grid), dim3(256), 0, s, p, n);
}

void launch_replica_sums(hipStream_t s, int32_t R, const RepDesc *reps, const double *eatom,
                         const double *watom, double *energy, double *virial)
{
    hipLaunchKernelGGL(k_replica_sums, dim3(R), dim3(256), 0, s, reps, eatom, watom, energy, virial);
}

void launch_to_user(hipStream_t s, int grid, int64_t n, const int32_t *id, const double *src3,
                    double *dst_user)
{
    hipLaunchKernelGGL(k_to_user, dim3(grid), dim3(256), 0, s, n, id, src3, dst_user);
}

void launch_from_user(hipStream_t s, int grid, int64_t n, const int32_t *id,
                      const double *src_user, double4 *dst)
{
    hipLaunchKernelGGL(k_from_user, dim3(grid), dim3(256), 0, s, n, id, src_user, dst);
}

void launch_pos_to_user(hipStream_t s, int grid, int64_t n, int32_t R, const RepDesc *reps,
                        const int32_t *rep_of, const int32_t *id, const double4 *pos,
                        double *dst_user)
{
    (void)R;
    hipLaunchKernelGGL(k_pos_to_user, dim3(grid), dim3(256), 0, s, n, reps, rep_of, id, pos, dst_user);
}

void launch_tables_f32(hipStream_t s, const double *src, float *dst, int64_t m)
{
    hipLaunchKernelGGL(k_tables_f32, dim3(64), dim3(256), 0, s, src, dst, m);
}
