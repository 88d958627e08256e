// md_internal.h -- device-side layout and kernel launchers of the MD hot path.
//
// Layout in HBM (all arrays in cell-sorted order unless named *_user):
//   pos      double4[N]  x, y, z, (unused)   -- gathered by neighbour loops
//   vel      double[3][N]                     -- streamed once per step
//   force    double[3][N]
//   xref     double4[N]  positions at the last list build
//   id       int32[N]    user index of each sorted slot
//   nbr      uint32[ceil(N/64)*64*M] Verlet lists, interleaved by groups of 64
//            atoms and 4 entries (md_brick.h); entry = candidate index in the
//            brick's halo (low 26 bits) | image code (high 6 bits, 2 per axis:
//            01 = add L, 10 = subtract L) fixed when the list is built
//   cnt      int32[N]    list length of each atom
//   brec     int32[B*stride] one record per brick of cells (md_brick.h)
//   bcost    int32[B]    cost of each brick in the last list build
//   bwork    int64[B+1]  prefix of bcost: the force kernels' balanced schedule
// Positions are wrapped into [0, L) when the cells are built; between builds they
// move freely and each pair uses the image fixed at build time (exact as long as
// no atom moves more than skin/2, which the rebuild trigger guarantees).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/md.h"

#define MD_WAVE 64
#define MD_IDX_BITS 26
#define MD_IDX_MASK ((1u << MD_IDX_BITS) - 1u)
#define MD_MAX_ATOMS (1ll << MD_IDX_BITS)

// error bits of the sticky device word
#define MD_FLAG_OVERFLOW 1
#define MD_FLAG_NONFINITE 2
#define MD_FLAG_SCHEDULE 4     // a dependent-schedule wait ran past its limit

struct RepDesc {
    double L[3];
    double hL[3];
    int32_t nc[3];      // cells per axis
    int32_t bd[3];      // brick extent per axis (cells), <= nc
    int32_t nb[3];      // bricks per axis
    int32_t pad;
    int64_t cell_off;   // first global cell of this replica
    int64_t brick_off;  // first global brick of this replica
    int64_t atom_off;   // first atom (user and sorted order agree on replica ranges)
    int64_t atom_end;
};

// Dependent schedule of the half-list tasks (one persistent launch).
struct DepArgs {
    const int32_t *off;    // [T+1] successor list offsets
    const int32_t *succ;   // successor task ids
    int32_t *ref;          // [T] predecessors still running (working copy)
    int32_t *queue;        // [T] ready tasks, -1 = slot not filled yet
    int32_t *sched;        // [0] next slot to take, [1] next slot to fill, [2] abort
    int32_t T;             // tasks (= bricks)
    uint64_t limit;        // wall-clock ticks a workgroup may wait for its slot
};

// Device-resident control words.
struct DevCtl {
    int32_t rebuild[2];   // rebuild request, indexed by step parity
    int32_t err;          // sticky MD_FLAG_* bits
    int32_t max_cnt;      // largest per-atom list length of the last build
    int32_t nrebuild;     // rebuilds performed inside md_verlet_step
    int32_t max_nbhd;     // largest brick halo (candidates) seen
    int32_t max_brick;    // largest brick (atoms) seen
    int32_t sched[4];     // dependent-schedule slot counters and abort word
};

// ---------------------------------------------------------------- launchers
// cells
void launch_load_user(hipStream_t s, int grid, int64_t n, const double *pos_user,
                      const double *vel_user, double4 *pos, double *vel, int32_t *id);
void launch_bin(hipStream_t s, int grid, const int32_t *pred, int64_t n, int32_t R,
                const RepDesc *reps, const int32_t *rep_of, double4 *pos, int32_t *cell_of,
                int32_t *slot, int32_t *count, int32_t *err);
void launch_scan(hipStream_t s, const int32_t *pred, int64_t C, int32_t *count,
                 int32_t *start, DevCtl *ctl);
void launch_scatter(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                    const int32_t *cell_of, const int32_t *slot, const int32_t *start,
                    int32_t *perm);
void launch_sort_cells(hipStream_t s, int grid, const int32_t *pred, int64_t C,
                       const int32_t *start, int32_t *count, const int32_t *perm, const int32_t *id,
                       const double4 *pos, const double *vel, int64_t n, double4 *pos_out,
                       double *vel_out, int32_t *id_out);
void launch_copy_back(hipStream_t s, int grid, const int32_t *pred, int64_t n,
                      const double4 *pos_t, const double *vel_t, const int32_t *id_t,
                      double4 *pos, double *vel, int32_t *id, double4 *xref);

// Work queue of the brick tasks: the bricks are split into eight contiguous
// ranges, one per XCD; a workgroup takes bricks from its XCD's range first and
// then from the others' (next[x] counts the bricks handed out of range x).  The
// last workgroup of a launch resets it.
struct TaskQueue {
    uint32_t next[8 * 32];   // counter of range x at next[32 x]: one 128-byte line each
    uint32_t done;
    uint32_t pad[31];
};

// brick record sizes: halo cells and own cells of the largest brick, record stride
struct BrickDims {
    int32_t Hm, Em, stride;
};

// neighbour list
struct ListArgs {
    const int32_t *pred;      // predicate word (build only if non-zero), may point at a constant 1
    int64_t B;                // total bricks
    int32_t R;
    const RepDesc *reps;
    const int32_t *start;     // cell_start[C+1]
    int32_t *brec;            // brick records (written)
    BrickDims bd;
    TaskQueue *tq;
    int32_t *bcost;           // [B] cost of each brick (list entries + 8 atoms + 512), written
    int64_t *bwork;           // [B+1] exclusive prefix of bcost, written by the last workgroup
    const double4 *src;       // sorted positions the list is built from
    int64_t n;
    uint32_t *nbr;
    int32_t *cnt;
    int32_t M;
    double rl2;
    int half;
    int32_t cap;              // candidates the list build stages in LDS per brick
    int32_t shift_cap;        // stage of the force and adjoint tasks: bricks whose whole
                              // halo fits it (and no axis wraps onto itself) get BR_SHIFT
                              // and 16-bit entries, whatever the list build stages itself
    // optional copy of the freshly sorted state into the working buffers
    const double *vel_src;
    const int32_t *id_src;
    double4 *pos_dst;
    double *vel_dst;
    int32_t *id_dst;
    double4 *xref;
    DevCtl *ctl;
};
void launch_shell_filter(hipStream_t s, int grid, int threads, const ListArgs &a);
void launch_build_list(hipStream_t s, int grid, int threads, const ListArgs &a);
size_t list_static_lds(int half);   // static LDS of the list build kernel (bytes)

// forces
struct ForceArgs {
    TaskQueue *ftq;       // brick queue of the force and adjoint kernels (dyn = 1)
    int32_t lds_tab;      // mixed EAM density pass: its binary32 table is copied to LDS
    int32_t dyn;          // 1: bricks from the queue; 0: static cost-balanced ranges
    int64_t n;
    int32_t R;
    const RepDesc *reps;      // R entries (device)
    RepDesc rep0;             // replica 0 by value (single-replica fast path)
    const int32_t *rep_of;    // replica of each sorted atom
    const double4 *pos;
    double4 *pos_next;        // drift output
    const double4 *xref;
    double *vel;              // [3][n]
    double *force;            // [3][n] sorted out (may be null)
    const uint32_t *nbr;
    const int32_t *cnt;
    int32_t M;
    int64_t B;                // bricks
    const int32_t *brec;      // brick records
    BrickDims bd;
    const int64_t *bwork;     // [B+1] prefix of the bricks' costs (from the list build)
    int32_t cap;              // candidates staged in LDS per brick task
    double rc2;
    const double *lj;         // device {eps, sigma}
    // EAM
    const double *tab[3];     // phi, rho, embed coefficient tables (binary64)
    const float *tabf[3];     // binary32 copies (mixed precision)
    int32_t nk[3];
    double x0[3], inv_h[3];
    double rphi2, rrho2;
    double *rho;              // [n] density, sorted
    double *fp;               // [n] F'(rho), sorted
    // integration
    int mode;                 // 0 forces only, 1 first (kick+drift), 2 middle, 3 last
    double cdt;               // dt / (2m)
    double dt;
    double mass;
    double thr2;              // (skin/2)^2
    int32_t *flag_set;        // rebuild request for the next step (may be null)
    int32_t *flag_clear;      // this step's request, cleared by block 0 (may be null)
    // reductions
    double *partial;          // [grid][4]
    double *outE;             // final sums of this launch (each may be null):
    double *outK;             //   potential energy, kinetic energy,
    double *outW;             //   scalar virial
    double *eatom;            // per-atom energy (multi-replica outputs), or null
    double *watom;            // per-atom virial, or null
    DevCtl *ctl;
    // waves of bricks (half list without global atomics)
    const int32_t *wbr;       // the bricks of this launch's wave
    int32_t nwb;
};
void launch_lj_full(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a);
void launch_lj_half(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a);
void launch_lj_wave(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a);
void launch_lj_deps(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a, const DepArgs &d,
                    const int32_t *npred, const int32_t *init_q, int32_t nroots);
void launch_atom_sums(hipStream_t s, int grid, int64_t n, const double *eatom, const double *watom,
                      double *energy, double *virial, double *partial);
// where the totals of a launch's per-workgroup partial sums go: out[c] (if not
// null) receives scale[c] times total c
struct SumOut {
    double *out[4];
    double scale[4];
};
// adds the partials of a launch of g workgroups in workgroup order (one
// workgroup of `threads`, the producing launch's size, which fixes the order)
void launch_sum_partials(hipStream_t s, const double *partial, int g, int threads, SumOut o);
void launch_eam_density(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a);
void launch_eam_force(hipStream_t s, int grid, int threads, bool mixed, const ForceArgs &a);
void launch_integrate(hipStream_t s, int grid, const ForceArgs &a);
void launch_zero(hipStream_t s, int grid, double *p, int64_t n);
void launch_replica_sums(hipStream_t s, int32_t R, const RepDesc *reps, const double *eatom,
                         const double *watom, double *energy, double *virial);
void launch_to_user(hipStream_t s, int grid, int64_t n, const int32_t *id, const double *src3,
                    double *dst_user);
void launch_pos_to_user(hipStream_t s, int grid, int64_t n, int32_t R, const RepDesc *reps,
                        const int32_t *rep_of, const int32_t *id, const double4 *pos,
                        double *dst_user);
void launch_from_user(hipStream_t s, int grid, int64_t n, const int32_t *id,
                      const double *src_user, double4 *dst);
void launch_tables_f32(hipStream_t s, const double *src, float *dst, int64_t m);

// adjoint
struct VjpArgs {
    ForceArgs f;
    const double4 *u;         // [n] sorted cotangent (x, y, z, 0)
    const double *vE;         // [R]
    double *gx;               // [3][n] sorted out
    double *gpart;            // LJ: [grid][4] parameter partials
    double *gtab;             // EAM: [3][(nk-1)*4] parameter gradient (atomics)
    double *rdot;             // EAM pass A output: rho-dot
    double *fpp;              // EAM pass A output: q = F'' rho-dot
    double *gout;             // LJ: 2 doubles out (final)
    int32_t gw_p, gw_r;       // EAM: trailing intervals of the phi and rho tables whose
                              // parameter gradient a workgroup sums in LDS first
                              // (embedding pass: gw_p = intervals of its table, or 0)
    int32_t gw_off;           // byte offset of those sums in the dynamic LDS
    int32_t stage_u;          // 1: stage the partners' cotangents (and EAM F', q) in LDS when they fit
};
void launch_lj_vjp(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max);
void launch_eam_vjp_a(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max);
void launch_eam_vjp_b(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max, int32_t limit);
void launch_eam_vjp_embed(hipStream_t s, int grid, const VjpArgs &a, int32_t lds_max, int32_t limit);

// ---------------------------------------------------------------- device helpers
#ifdef __HIPCC__
// Work item sequence of one unit (a wave or a whole block) of a persistent grid.
// The items are split into eight contiguous ranges and workgroup b serves range
// b % 8: workgroups are dispatched round-robin over the eight XCDs, so each XCD's
// L2 sees one compact region of the cell-sorted data.
struct ItemRange {
    int64_t first, end, stride;
};
__device__ __forceinline__ ItemRange xcd_items(int64_t nitems, int units_per_block, int unit)
{
    ItemRange r;
    const int G = gridDim.x;
    if (G % 8 != 0) {
        r.first = (int64_t)blockIdx.x * units_per_block + unit;
        r.stride = (int64_t)G * units_per_block;
        r.end = nitems;
        return r;
    }
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3, G8 = G >> 3;
    const int64_t per = (nitems + 7) / 8;
    const int64_t lo = (int64_t)x * per;
    r.end = lo + per < nitems ? lo + per : nitems;
    r.first = lo + (int64_t)slot * units_per_block + unit;
    r.stride = (int64_t)G8 * units_per_block;
    return r;
}

// make LDS stores of this wavefront visible to its other lanes
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
#endif
