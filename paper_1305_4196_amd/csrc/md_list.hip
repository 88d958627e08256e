// md_list.hip -- Verlet neighbour lists built brick by brick (Sec. II.A, II.C).
//
// One workgroup per brick of cells (md_brick.h).  It builds the brick's record
// (halo and own-cell offsets), writes it out for the force and adjoint tasks,
// and stages the halo's positions in LDS.  Each wavefront then takes one of the
// brick's cells and tests every atom of it against the atoms of the distinct
// cells of the 3x3x3 block around the cell (along an axis of 2 cells the block
// has 2 distinct layers):
//   d = x_i - x_j;  d > L/2 -> d - L,  d < -L/2 -> d + L;  r2 = (dx*dx + dy*dy) + dz*dz
// in binary64 with contraction off, keeping j iff r2 < (rc + skin)^2 and j != i
// (and, for the half list, j after i in the sorted order).  Only the wavefront
// of atom i's cell appends to i's list, so every list has exactly one writer
// and no atomics are needed (each task owns its lists, Sec. II.C).  An entry
// holds the candidate index and the pair's image code, except in bricks that
// stage their halo through the cell images (BR_SHIFT), where the code equals
// the candidate's halo-cell image and is left out and the bare index is stored
// in 16 bits (the narrow layout; half the list's bytes to write and read).
//
// The three cells of a stencil row along x are consecutive in the halo order
// (or, on a grid of at most bx + 1 cells, wrap around it), so each of the 9
// rows is one or two contiguous candidate ranges.  The cell's candidates are
// held in registers, 9 x 64 at a time, and reused by all atoms of the cell.
// Cells of more than 128 atoms are taken in groups of 128 atoms.
//
// Interior cells: along an axis with at least 5 cells, a neighbour of a cell
// that is not on the box face is at most 2 cell widths (< L/2) away, so the
// minimum-image test never fires and is skipped -- the arithmetic, and so the
// pair set, is unchanged.  Bricks that touch no box face skip it entirely.
#include "md_brick.h"

namespace {

// One wavefront, one own cell e of the brick: the cell's stencil rows are
// concatenated into one candidate sequence, the cell's own atoms first, and
// loaded into registers in tiles of at most TILE chunks of 64 (one candidate
// per lane and chunk; the chunks are spread evenly over the tiles).  Every atom
// of the cell (a uniform value per iteration: read from LDS by all lanes at
// once, the next atom's issued ahead; up to 128 atoms per pass) is tested
// against the tile: all of its chunk tests in one block without branches, then
// its stores.  Hits are compacted with a ballot and mbcnt, so atom a's entries
// keep the candidate order; the running list lengths live in LDS, one word per
// atom of the pass.  The atom itself is taken out of the one chunk of the
// own-cell tiles that holds it (a scalar mask).  Every lane stores: the row is
// addressed through a buffer descriptor whose record count ends at the
// capacity, a lane without a hit stores to an index past it, and the
// hardware's range check drops both that store and entries beyond the
// capacity (the overflow is still counted and flagged).  Most of the loop is
// then split about evenly between vector and scalar instructions, which share
// a CU's issue slots.
constexpr int TILE = 5;
// candidates per cell whose run starts are flagged in LDS (more: binary search)
constexpr int CRUN = 768;

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const uint64_t u = __double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
    return __longlong_as_double((int64_t)(((uint64_t)hi << 32) | lo));
}

// Runs of the stencil rows of own cell lc, built by the wavefront's lanes in
// parallel (lane t: layer sz = t / (2 np_y), row sy = (t / 2) % np_y, part t & 1,
// the order of a plain loop over sz, sy, part) and stored in LDS, with the own
// cell's atoms [ko, ko + na) taken out of their row and put first (so an atom's
// own candidate sits at its index in the cell):
// runs[0..nr) candidate index minus position (the cell's v-th candidate, v in
// run r, is v + runs[r]), runs[32..32+nr] prefix of the run lengths,
// runs[31] = nr.  Along an axis the stencil's halo coordinate is lc + s
// (s = 0..np-1), reduced by n when the halo covers the axis (lc + s < 2 n).
// With at most CRUN candidates, bit v of the bitmap crun is set exactly where a
// run starts.
__device__ __forceinline__ void build_runs(const Stage &st, const BrickGeom &g, const int32_t lc[3],
                                           const int32_t np[3], int32_t ko, int32_t na, int32_t *runs,
                                           uint32_t *crun)
{
    const int lane = threadIdx.x & 63;
    const int32_t *soff = st.rec + BR_HDR;
    const int32_t nt = 2 * np[1] * np[2];
    int32_t kb = 0, ke = 0;
    if (lane < nt) {
        const int32_t part = lane & 1, sy = (lane >> 1) % np[1], sz = (lane >> 1) / np[1];
        int32_t hy = lc[1] + sy, hz = lc[2] + sz;
        hy = hy >= g.nc[1] ? hy - g.nc[1] : hy;
        hz = hz >= g.nc[2] ? hz - g.nc[2] : hz;
        const int32_t rowh = g.hn[0] * (hy + g.hn[1] * hz);
        const int32_t xa = lc[0];
        const int32_t x1 = xa + np[0] < g.hn[0] ? xa + np[0] : g.hn[0];
        const int32_t x2 = xa + np[0] - x1;
        kb = part == 0 ? soff[rowh + xa] : soff[rowh];
        ke = part == 0 ? soff[rowh + x1] : soff[rowh + x2];
        ke = ke > kb ? ke : kb;
    }
    // the own cell is a distinct cell of its stencil: exactly one lane's range
    // holds it whole; that range is cut into the parts before and after it
    const bool own = lane < nt && ko >= kb && ko + na <= ke;
    const int32_t l1 = own ? ko - kb : ke - kb;          // [kb, kb + l1)
    const int32_t kb2 = ko + na;
    const int32_t l2 = own ? ke - kb2 : 0;               // [kb2, kb2 + l2)
    const int32_t pc = (l1 > 0 ? 1 : 0) + (l2 > 0 ? 1 : 0);
    // exclusive prefix over the lanes of the lengths (low 24 bits) and piece counts
    const int32_t packed = (l1 + l2) | (pc << 24);
    int32_t inc = packed;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    const int32_t ex = inc - packed;
    const int32_t pex = na + (ex & 0xffffff);            // after the own cell
    const int32_t rb = 1 + (ex >> 24);
    if (l1 > 0) {
        runs[rb] = kb - pex;
        runs[32 + rb] = pex;
    }
    if (l2 > 0) {
        const int32_t r = rb + (l1 > 0 ? 1 : 0);
        runs[r] = kb2 - (pex + l1);
        runs[32 + r] = pex + l1;
    }
    const int32_t last = __shfl(inc, 63, 64);            // with every lane active
    const int32_t nr = 1 + (last >> 24);
    const int32_t total = na + (last & 0xffffff);
    if (lane == 0) {
        runs[0] = ko;
        runs[32] = 0;
        runs[32 + nr] = total;
        runs[31] = nr;
    }
    if (total <= CRUN) {
        for (int32_t q = lane; q < (total + 31) >> 5; q += 64) crun[q] = 0u;
        wave_sync();
        if (lane == 0) atomicOr(&crun[0], 1u);
        if (l1 > 0) atomicOr(&crun[pex >> 5], 1u << (pex & 31));
        if (l2 > 0) atomicOr(&crun[(pex + l1) >> 5], 1u << ((pex + l1) & 31));
    }
    wave_sync();
}

// Entry p of an atom's row: word (p/4) * 256 + p%4 of the row, or in the
// narrow layout halfword (p/8) * 512 + p%8, in units of one entry.  The index
// grows with p, so an atom's entries below the capacity M are exactly those
// whose index is below entry_index(M).
template <bool NARROW>
__device__ __forceinline__ uint32_t entry_index(uint32_t p)
{
    return NARROW ? p + __umul24(p >> 3, 504u) : p + __umul24(p >> 2, 252u);
}

// Structured-buffer stores (records of `stride` bytes, index range-checked
// against the descriptor's record count: a store at or beyond it is dropped).
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__device__ void sbuf_store_i16(int16_t v, i32x4 rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                               int32_t aux) __asm("llvm.amdgcn.struct.buffer.store.i16");
__device__ void sbuf_store_i32(int32_t v, i32x4 rsrc, int32_t vindex, int32_t voffset, int32_t soffset,
                               int32_t aux) __asm("llvm.amdgcn.struct.buffer.store.i32");

// Buffer descriptor of gfx9: base address, stride in bits 16..29 of the
// second word, record count, and the default data format word.
__device__ __forceinline__ i32x4 buffer_desc(uintptr_t base, uint32_t stride, uint32_t nrec)
{
    i32x4 r;
    r.x = (int32_t)(uint32_t)base;
    r.y = (int32_t)(((uint32_t)((uint64_t)base >> 32) & 0xffffu) | (stride << 16));
    r.z = (int32_t)nrec;
    r.w = 0x00020000;
    return r;
}

// a where the lane's bit of mask is set, else b: one v_cndmask on the mask
// (a select on the inverse ballot compiles to a branch on exec instead, two
// scalar instructions more)
__device__ __forceinline__ int32_t select_lanes(uint64_t mask, int32_t a, int32_t b)
{
    int32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
    return r;
}

// What the tile tests of one cell share.
struct CellCtx {
    double L[3], hL[3];
    double rl2;
    i32x4 rows;                  // the rows from the cell's first atom's group of 64 on
    int32_t group_bytes;         // bytes of 64 rows
    int32_t row_entries;         // entries of a row below the capacity M (records of `rows`)
    bool wrap[3];
};

// The atoms at..at_end of a group (held in ax/ay/az, atom at in lane at - 64 half)
// against the NCH chunks of candidates in registers.  All NCH tests of an atom
// come first, so their binary64 chains overlap; then the hits of each chunk are
// stored in candidate order behind the atom's running length ni, by every lane:
// a lane without a hit stores to an index past the row, which the buffer's
// range check drops (no branch on the hit mask).  SELF: the tile holds
// candidates at sequence positions vself + at, the atoms themselves (the own
// cell comes first in the sequence), which are taken out of the masks.  i0:
// sorted index of the cell's first atom, g0: the group's first atom in the cell.
template <bool HALF, bool WRAP, bool NARROW, int NCH, bool SELF, bool ALL>
__device__ __forceinline__ void test_tile(const CellCtx &cc, const double *cx, const double *cy, const double *cz,
                                          const int32_t *ck, const int64_t *cj, const uint64_t *valid,
                                          int32_t at_begin, int32_t at_end, int half, double ax, double ay,
                                          double az, const double *own, int64_t i0, int32_t g0, int32_t vself,
                                          int32_t *cnt)
{
    const int lane = threadIdx.x & 63;
    // ALL: the group's atoms are staged, own[3 at ..] (broadcast LDS reads,
    // the next atom's issued ahead); else they come from lanes of ax/ay/az
    double xn = 0.0, yn = 0.0, zn = 0.0;
    if (ALL && at_begin < at_end) {
        xn = own[3 * at_begin];
        yn = own[3 * at_begin + 1];
        zn = own[3 * at_begin + 2];
    }
    for (int32_t at = at_begin; at < at_end; at++) {
        const int64_t i = i0 + g0 + at;
        double xi, yi, zi;
        if (ALL) {
            xi = xn;
            yi = yn;
            zi = zn;
            const int32_t an = at + 1 < at_end ? at + 1 : at;
            xn = own[3 * an];
            yn = own[3 * an + 1];
            zn = own[3 * an + 2];
        } else {
            const int l = at - 64 * half;
            xi = readlane_f64(ax, l);
            yi = readlane_f64(ay, l);
            zi = readlane_f64(az, l);
        }
        // the atom's running list length (per wavefront in LDS)
        int32_t ni = cnt[at];
        // the atom's row: 16 bytes per atom across a group of 64 rows, in either
        // layout, from the group of the cell's first atom on
        const int32_t row_off = (int32_t)((i >> 6) - (i0 >> 6)) * cc.group_bytes + (int32_t)((i & 63) << 4);
        const int32_t vs = vself + at;
        uint64_t m[NCH];
        uint32_t code[NCH];
        _Pragma("unroll")
        for (int c = 0; c < NCH; c++) {
            double dx = xi - cx[c], dy = yi - cy[c], dz = zi - cz[c];
            code[c] = 0;
            if (WRAP) {
                if (cc.wrap[0]) {
                    const bool gt = dx > cc.hL[0], lt = dx < -cc.hL[0];
                    dx = gt ? dx - cc.L[0] : (lt ? dx + cc.L[0] : dx);
                    code[c] |= gt ? 2u : (lt ? 1u : 0u);
                }
                if (cc.wrap[1]) {
                    const bool gt = dy > cc.hL[1], lt = dy < -cc.hL[1];
                    dy = gt ? dy - cc.L[1] : (lt ? dy + cc.L[1] : dy);
                    code[c] |= gt ? 8u : (lt ? 4u : 0u);
                }
                if (cc.wrap[2]) {
                    const bool gt = dz > cc.hL[2], lt = dz < -cc.hL[2];
                    dz = gt ? dz - cc.L[2] : (lt ? dz + cc.L[2] : dz);
                    code[c] |= gt ? 32u : (lt ? 16u : 0u);
                }
            }
            const double r2 = (dx * dx + dy * dy) + dz * dz;
            m[c] = valid[c] & __builtin_amdgcn_ballot_w64(r2 < cc.rl2);
            if (SELF && (vs >> 6) == c) m[c] &= ~(1ull << (vs & 63));
            if (HALF) m[c] &= __builtin_amdgcn_ballot_w64(cj[c] > i);
        }
        _Pragma("unroll")
        for (int c = 0; c < NCH; c++) {
            const uint32_t p = __builtin_amdgcn_mbcnt_hi((uint32_t)(m[c] >> 32),
                               __builtin_amdgcn_mbcnt_lo((uint32_t)m[c], (uint32_t)ni));
            const int32_t idx = select_lanes(m[c], (int32_t)entry_index<NARROW>(p), cc.row_entries);
            if (NARROW) {
                sbuf_store_i16((int16_t)ck[c], cc.rows, idx, 0, row_off, 0);
            } else {
                const uint32_t word = WRAP ? (uint32_t)ck[c] | (code[c] << MD_IDX_BITS) : (uint32_t)ck[c];
                sbuf_store_i32((int32_t)word, cc.rows, idx, 0, row_off, 0);
            }
            ni += (int32_t)__popcll(m[c]);
        }
        if (lane == 0) cnt[at] = ni;
    }
}

// WRAP: some axis of the cell needs the minimum-image test; otherwise the
// test and the image code are compiled out.  NARROW: the brick is staged
// through its cell images and stores bare 16-bit candidate indices.
template <bool HALF, bool WRAP, bool NARROW, bool ALL>
__device__ __forceinline__ void scan_cell(const ListArgs &a, const Stage &st, const BrickGeom &g,
                                          int32_t e, int32_t na_all, const int32_t lc[3],
                                          const bool wrap[3], const int32_t *runs, const uint32_t *crun,
                                          int32_t *cnt_w, int32_t &my_max, int32_t *bpairs)
{
    const int lane = threadIdx.x & 63;
    const int32_t *soff = st.rec + br_soff(a.bd);
    const int32_t *abeg = st.rec + br_abeg(a.bd);
    const int32_t hown = (lc[0] + 1) % g.nc[0] + g.hn[0] * ((lc[1] + 1) % g.nc[1] + g.hn[1] * ((lc[2] + 1) % g.nc[2]));
    const int32_t k_own = soff[hown];          // candidate index of the cell's first atom
    const int64_t i0_all = abeg[e];            // sorted index of the cell's first atom
    const int32_t nr = runs[31];
    const int32_t ncand = runs[32 + nr];
    const RepDesc &rep = a.reps[g.r];
    const int32_t M = a.nbr == nullptr ? 0 : a.M;
    CellCtx cc;
    for (int d = 0; d < 3; d++) {
        cc.L[d] = rep.L[d];
        cc.hL[d] = rep.hL[d];
        cc.wrap[d] = wrap[d];
    }
    cc.rl2 = a.rl2;
    // entries of an atom's row below entry M: a row is addressed as a buffer of
    // that many entry-sized records (the atom's row offset as the buffer's
    // scalar offset), so stores beyond M are dropped by the buffer's range
    // check, which is the capacity test
    cc.row_entries = (int32_t)entry_index<NARROW>((uint32_t)M);
    cc.group_bytes = (M >> 2) << 10;
    cc.rows = buffer_desc(reinterpret_cast<uintptr_t>(a.nbr) + (uintptr_t)((i0_all >> 6) * (int64_t)cc.group_bytes),
                          NARROW ? 2u : 4u, (uint32_t)cc.row_entries);
    // chunks of 64 candidates, in tiles of at most TILE chunks of balanced sizes
    const bool all_staged = ALL;                 // every candidate of the brick is in LDS
    const int32_t nchunks = (ncand + 63) >> 6;
    const int32_t ntiles = (nchunks + TILE - 1) / TILE;
    int32_t tot = 0;
    // the cell's atoms in groups of up to 128 (two per lane)
    for (int32_t g0 = 0; g0 < na_all; g0 += 128) {
    const int32_t na = na_all - g0 < 128 ? na_all - g0 : 128;
    const int64_t i0 = i0_all + g0;
    const int32_t k_grp = k_own + g0;
    // running list lengths of the group's atoms
    cnt_w[lane] = 0;
    cnt_w[64 + lane] = 0;
    wave_sync();
    double ax0 = 0.0, ay0 = 0.0, az0 = 0.0, ax1 = 0.0, ay1 = 0.0, az1 = 0.0;
    if (!ALL) {
        const int32_t k0 = k_grp + lane, k1 = k_grp + 64 + lane;
        if (lane < na) {
            if (ALL || k0 < st.cap) {
                ax0 = st.xyz[3 * k0];
                ay0 = st.xyz[3 * k0 + 1];
                az0 = st.xyz[3 * k0 + 2];
            } else {
                const double4 p = a.src[i0 + lane];
                ax0 = p.x;
                ay0 = p.y;
                az0 = p.z;
            }
        }
        if (lane + 64 < na) {
            if (ALL || k1 < st.cap) {
                ax1 = st.xyz[3 * k1];
                ay1 = st.xyz[3 * k1 + 1];
                az1 = st.xyz[3 * k1 + 2];
            } else {
                const double4 p = a.src[i0 + 64 + lane];
                ax1 = p.x;
                ay1 = p.y;
                az1 = p.z;
            }
        }
    }
    int32_t rbase = 0;                         // runs started before the current chunk
    int32_t c0 = 0;                            // first chunk of the tile
    for (int32_t t = 0; t < ntiles; t++) {
        const int32_t nch = nchunks / ntiles + (t < nchunks % ntiles ? 1 : 0);
        const int32_t t0 = 64 * c0;
        double cx[TILE], cy[TILE], cz[TILE];
        int32_t ck[TILE];
        int64_t cj[TILE];
        _Pragma("unroll")
        for (int c = 0; c < TILE; c++) {
            const int32_t v = t0 + 64 * c + lane;
            int32_t k = k_own;
            if (ncand <= CRUN) {
                // run of candidate v: the runs started before this chunk plus
                // the starts flagged up to v within it
                if (c < nch) {
                    const bool st0 = v < ncand && ((crun[v >> 5] >> (v & 31)) & 1u) != 0;
                    const uint64_t sm = __builtin_amdgcn_ballot_w64(st0);
                    const int32_t r = rbase + (int32_t)lanes_below(sm) + (st0 ? 1 : 0) - 1;
                    rbase += (int32_t)__popcll(sm);
                    if (v < ncand) k = v + runs[r];
                }
            } else if (c < nch && v < ncand) {
                int32_t lo = 0, hi = nr - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (runs[32 + mid] <= v) lo = mid; else hi = mid - 1;
                }
                k = v + runs[lo];
            }
            ck[c] = (c < nch && v < ncand) ? k : -1;
            cj[c] = 0;
            // (a wholly staged halo reads LDS only: no flat loads merging the two)
            if (all_staged || k < st.cap) {
                const double *q = st.xyz + 3 * k;
                cx[c] = q[0];
                cy[c] = q[1];
                cz[c] = q[2];
                if (HALF) cj[c] = st.j[k];
            } else {
                const int32_t j = candidate_index(st, a.bd, k);
                const double4 p = a.src[j];
                cx[c] = p.x;
                cy[c] = p.y;
                cz[c] = p.z;
                cj[c] = j;
            }
        }
        uint64_t valid[TILE];
        _Pragma("unroll")
        for (int c = 0; c < TILE; c++) valid[c] = __builtin_amdgcn_ballot_w64(ck[c] >= 0);
        // the cell's atoms come first in the sequence: atom g0 + at is candidate g0 + at
        const int32_t vself = g0 - t0;
        const bool self = t0 < na_all;
        // atoms 0..63 of the group from the first register set, 64..127 from the second
        const double *own = st.xyz + 3 * (int64_t)k_grp;
        for (int half = 0; half < 2; half++) {
            const int32_t at_end = half == 0 ? (na < 64 ? na : 64) : na;
            const double ax = half == 0 ? ax0 : ax1, ay = half == 0 ? ay0 : ay1, az = half == 0 ? az0 : az1;
            const int32_t at0 = 64 * half;
#define MD_TILE(NCH, SELF) test_tile<HALF, WRAP, NARROW, NCH, SELF, ALL>(cc, cx, cy, cz, ck, cj, valid, at0, at_end, \
                                                                         half, ax, ay, az, own, i0_all, g0, vself, cnt_w)
            if (self) {
                if (nch == 5) MD_TILE(5, true);
                else if (nch == 4) MD_TILE(4, true);
                else if (nch == 3) MD_TILE(3, true);
                else if (nch == 2) MD_TILE(2, true);
                else MD_TILE(1, true);
            } else {
                if (nch == 5) MD_TILE(5, false);
                else if (nch == 4) MD_TILE(4, false);
                else if (nch == 3) MD_TILE(3, false);
                else if (nch == 2) MD_TILE(2, false);
                else MD_TILE(1, false);
            }
#undef MD_TILE
        }
        c0 += nch;
    }
    wave_sync();
    const int32_t cnt0 = cnt_w[lane], cnt1 = cnt_w[64 + lane];
    if (lane < na) {
        a.cnt[i0 + lane] = cnt0;
        my_max = cnt0 > my_max ? cnt0 : my_max;
        tot += cnt0;
    }
    if (lane + 64 < na) {
        a.cnt[i0 + 64 + lane] = cnt1;
        my_max = cnt1 > my_max ? cnt1 : my_max;
        tot += cnt1;
    }
    }
    for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
    if (lane == 0) atomicAdd(bpairs, tot);
}

// next own cell for this wavefront (uniform)
__device__ __forceinline__ int32_t take_cell(int32_t *next_cell)
{
    int32_t v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(next_cell, 1);
    return __builtin_amdgcn_readfirstlane(v);
}

template <bool HALF>
__global__ __launch_bounds__(TASK_MAX_THREADS, 4) void k_build_list(ListArgs a)
{
    if (*a.pred == 0) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t smax[TASK_MAX_THREADS / 64], stot[TASK_MAX_THREADS / 64], sbr[TASK_MAX_THREADS / 64];
    __shared__ int32_t runs_lds[64 * (TASK_MAX_THREADS / 64)];
    __shared__ uint32_t crun_lds[CRUN / 32 * (TASK_MAX_THREADS / 64)];
    __shared__ int32_t order[64];
    __shared__ int32_t cnt_lds[128 * (TASK_MAX_THREADS / 64)];
    const Stage st = stage_slice(lds_raw, a.cap, 0, HALF);
    const int lane = threadIdx.x & 63;
    // the wavefront index as a scalar, so that everything derived per cell is uniform
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ int32_t slot, bpairs, next_cell;
    int32_t my_max = 0, my_tot = 0, my_br = 0;

    for (;;) {
        const int64_t b = next_brick(a.tq, a.B, &slot);
        if (b < 0) break;
        if (threadIdx.x == 0) {
            bpairs = 0;
            next_cell = (int32_t)(blockDim.x >> 6);
        }
        const BrickGeom g = brick_geom(a.reps, a.R, b);
        brick_setup(st, a.bd, g, a.start, a.shift_cap);
        int32_t *grec = a.brec + b * (int64_t)a.bd.stride;
        for (int32_t t = threadIdx.x; t < a.bd.stride; t += blockDim.x) grec[t] = st.rec[t];
        const int32_t natoms = st.rec[BR_ATOMS];
        if (natoms == 0) {
            if (threadIdx.x == 0) __hip_atomic_store(&a.bcost[b], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const int32_t total = st.rec[BR_TOTAL];
        my_tot = total > my_tot ? total : my_tot;
        my_br = natoms > my_br ? natoms : my_br;
        const int32_t lim = total < st.cap ? total : st.cap;
        for (int32_t k = threadIdx.x; k < lim; k += blockDim.x) {
            const int32_t jj = candidate_index(st, a.bd, k);
            const double4 p = at32(a.src, jj);
            st.xyz[3 * k] = p.x;
            st.xyz[3 * k + 1] = p.y;
            st.xyz[3 * k + 2] = p.z;
            if (st.j != nullptr) st.j[k] = jj;
        }
        __syncthreads();
        const int32_t E = st.rec[BR_E];
        const int32_t *aoff = st.rec + br_aoff(a.bd);
        // cells by decreasing atom count (ties by index): the cheap ones come
        // last, so the wavefronts finish the brick close together
        if (w == 0) {
            const int32_t my = lane < E ? aoff[lane + 1] - aoff[lane] : -1;
            int32_t rank = 0;
            for (int32_t q = 0; q < E; q++) {
                const int32_t o = __shfl(my, q, 64);
                rank += (o > my || (o == my && q < lane)) ? 1 : 0;
            }
            if (lane < E) order[rank] = lane;
        }
        __syncthreads();
        // own cells in that order, one wavefront per cell: the first one per
        // wavefront fixed, the others taken from a counter as wavefronts finish
        for (int32_t t = w; t < E;) {
            const int32_t e = order[t];
            const int32_t na = aoff[e + 1] - aoff[e];
            if (na == 0) break;                      // the rest are empty too
            const int32_t lc[3] = {e % g.e[0], (e / g.e[0]) % g.e[1], e / (g.e[0] * g.e[1])};
            int32_t np[3];
            bool wrap[3];
            for (int d = 0; d < 3; d++) {
                const int32_t c = g.o[d] + lc[d];
                np[d] = g.nc[d] >= 3 ? 3 : 2;
                wrap[d] = !(g.nc[d] >= 5 && c >= 1 && c <= g.nc[d] - 2);
            }
            int32_t *runs = runs_lds + 64 * w;
            uint32_t *crun = crun_lds + CRUN / 32 * w;
            const int32_t hown = (lc[0] + 1) % g.nc[0] + g.hn[0] * ((lc[1] + 1) % g.nc[1] + g.hn[1] * ((lc[2] + 1) % g.nc[2]));
            build_runs(st, g, lc, np, st.rec[BR_HDR + hown], na, runs, crun);
            const bool any_wrap = wrap[0] || wrap[1] || wrap[2];
            // (bricks staged through their cell images have their whole halo in
            // the force tasks' stage, which may be larger than this one)
            if (st.rec[BR_SHIFT] != 0 && st.rec[BR_TOTAL] <= st.cap) {
                if (any_wrap) scan_cell<HALF, true, true, true>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
                else scan_cell<HALF, false, true, true>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
            } else if (st.rec[BR_SHIFT] != 0) {
                if (any_wrap) scan_cell<HALF, true, true, false>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
                else scan_cell<HALF, false, true, false>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
            } else if (st.rec[BR_TOTAL] <= st.cap) {
                if (any_wrap) scan_cell<HALF, true, false, true>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
                else scan_cell<HALF, false, false, true>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
            } else {
                if (any_wrap) scan_cell<HALF, true, false, false>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
                else scan_cell<HALF, false, false, false>(a, st, g, e, na, lc, wrap, runs, crun, cnt_lds + 128 * w, my_max, &bpairs);
            }
            t = take_cell(&next_cell);
        }
        // copy the freshly sorted state of the brick's atoms into the working buffers
        if (a.pos_dst != nullptr) {
            for (int32_t la = threadIdx.x; la < natoms; la += blockDim.x) {
                const int64_t i = brick_atom(st, a.bd, la);
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
        // the brick's cost for the balanced schedules of the force kernels
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&a.bcost[b], bpairs + 8 * natoms + 512, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // one atomic per workgroup (a per-atom atomic on one word would serialise in L2)
    for (int o = 32; o > 0; o >>= 1) {
        my_max = max(my_max, __shfl_xor(my_max, o, 64));
        my_tot = max(my_tot, __shfl_xor(my_tot, o, 64));
        my_br = max(my_br, __shfl_xor(my_br, o, 64));
    }
    if (lane == 0) {
        smax[w] = my_max;
        stot[w] = my_tot;
        sbr[w] = my_br;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = smax[0], t = stot[0], q = sbr[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); k++) {
            m = max(m, smax[k]);
            t = max(t, stot[k]);
            q = max(q, sbr[k]);
        }
        atomicMax(&a.ctl->max_cnt, m);
        atomicMax(&a.ctl->max_nbhd, t);
        atomicMax(&a.ctl->max_brick, q);
        if (m > a.M && a.M > 0) atomicOr(&a.ctl->err, MD_FLAG_OVERFLOW);
    }
    // the last workgroup turns the bricks' costs into their prefix
    if (!tasks_done(a.tq)) return;
    __shared__ int64_t wsum[TASK_MAX_THREADS / 64];
    const int nw = (int)(blockDim.x >> 6);
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < a.B; c0 += 4 * (int64_t)blockDim.x) {
        const int64_t k0 = c0 + 4 * (int64_t)threadIdx.x;
        int64_t v[4], s = 0;
        for (int q = 0; q < 4; q++) {
            v[q] = k0 + q < a.B ? (int64_t)__hip_atomic_load(&a.bcost[k0 + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
            s += v[q];
        }
        int64_t inc = s;
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        int64_t before = 0, total = 0;
        for (int k = 0; k < nw; k++) {
            before += k < w ? wsum[k] : 0;
            total += wsum[k];
        }
        int64_t run = carry + before + inc - s;
        for (int q = 0; q < 4; q++)
            if (k0 + q < a.B) {
                a.bwork[k0 + q] = run;
                run += v[q];
            }
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) a.bwork[a.B] = carry;
}

} // namespace

// Half list over 14 of the 27 cells (Sec. II.D.3), from a full list in place:
// an atom keeps a partner whose cell, seen through the entry's image, lies in
// the forward half of its neighbourhood -- above in z; at the same z, above in
// y; at the same z and y, above in x -- or in its own cell with a larger sorted
// index.  The partner's cell is its halo cell (the record's soff table), moved
// by the entry's image code (per-entry bits, or the halo cell's image in
// bricks staged through their images); the offset is taken in whole cells,
// (o - 1 + t) mod n + s n - (own cell), so the two atoms of a pair see
// opposite offsets and exactly one keeps it.  Partners then lie in a
// 3 x 3 x 2 block of cells: the atom's cell and the layer above it in z, one
// cell around in x and y.  Each lane compacts its own atom's row.
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_shell_filter(ListArgs a)
{
    if (*a.pred == 0) return;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const Stage st = stage_slice(lds_raw, 0, 0, false);
    const int32_t M = a.M;
    uint16_t *nbr16 = reinterpret_cast<uint16_t *>(a.nbr);
    for (int64_t b = blockIdx.x; b < a.B; b += gridDim.x) {
        const int32_t *grec = a.brec + b * (int64_t)a.bd.stride;
        const int32_t natoms = __builtin_amdgcn_readfirstlane(grec[BR_ATOMS]);
        if (natoms == 0) continue;
        __syncthreads();
        for (int32_t t = threadIdx.x; t < a.bd.stride; t += blockDim.x) st.rec[t] = grec[t];
        __syncthreads();
        const BrickGeom g = brick_geom(a.reps, a.R, b);
        const bool shifted = st.rec[BR_SHIFT] != 0;
        const int32_t *soff = st.rec + br_soff(a.bd), *sbeg = st.rec + br_sbeg(a.bd);
        const int32_t *himg = st.rec + br_himg(a.bd);
        for (int32_t la = threadIdx.x; la < natoms; la += blockDim.x) {
            int32_t e = 0;
            const int64_t i = brick_atom(st, a.bd, la, &e);
            const int32_t ci[3] = {g.o[0] + e % g.e[0], g.o[1] + (e / g.e[0]) % g.e[1], g.o[2] + e / (g.e[0] * g.e[1])};
            const int32_t m = min(a.cnt[i], M);
            int32_t q = 0;
            for (int32_t p = 0; p < m; p++) {
                const uint32_t w = shifted ? (uint32_t)nbr16[ell_half(i, p, M)] : a.nbr[ell_word(i, p, M)];
                const int32_t k = shifted ? (int32_t)w : (int32_t)(w & MD_IDX_MASK);
                const int32_t h = halo_cell(st, k);
                const uint32_t code = shifted ? (uint32_t)himg[h] : (w >> MD_IDX_BITS);
                const int32_t t[3] = {h % g.hn[0], (h / g.hn[0]) % g.hn[1], h / (g.hn[0] * g.hn[1])};
                int32_t off[3];
                for (int d = 0; d < 3; d++) {
                    const uint32_t c = (code >> (2 * d)) & 3u;
                    const int32_t sft = c == 2u ? 1 : (c == 1u ? -1 : 0);   // bit 1: partner at x + L
                    off[d] = (g.o[d] - 1 + t[d] + g.nc[d]) % g.nc[d] + sft * g.nc[d] - ci[d];
                }
                const int64_t j = sbeg[h] + (k - soff[h]);
                const bool fwd = off[2] != 0 ? off[2] > 0
                               : off[1] != 0 ? off[1] > 0
                               : off[0] != 0 ? off[0] > 0 : j > i;
                if (fwd) {
                    if (shifted) nbr16[ell_half(i, q, M)] = (uint16_t)w;
                    else a.nbr[ell_word(i, q, M)] = w;
                    q++;
                }
            }
            a.cnt[i] = q;
        }
    }
}

void launch_shell_filter(hipStream_t s, int grid, int threads, const ListArgs &a)
{
    const size_t lds = stage_bytes(0, 0, false, a.bd.stride);
    allow_lds(k_shell_filter, lds);
    hipLaunchKernelGGL(k_shell_filter, dim3(grid), dim3(threads), lds, s, a);
}

size_t list_static_lds(int half)
{
    auto query = [](const void *k) -> size_t {
        hipFuncAttributes attr{};
        return hipFuncGetAttributes(&attr, k) == hipSuccess ? attr.sharedSizeBytes : 8192;
    };
    static const size_t bytes[2] = {query(reinterpret_cast<const void *>(k_build_list<false>)),
                                    query(reinterpret_cast<const void *>(k_build_list<true>))};
    return bytes[half != 0];
}

void launch_build_list(hipStream_t s, int grid, int threads, const ListArgs &a)
{
    const size_t lds = stage_bytes(a.cap, 0, a.half != 0, a.bd.stride);
    if (a.half) {
        allow_lds(k_build_list<true>, lds);
        hipLaunchKernelGGL(k_build_list<true>, dim3(grid), dim3(threads), lds, s, a);
    } else {
        allow_lds(k_build_list<false>, lds);
        hipLaunchKernelGGL(k_build_list<false>, dim3(grid), dim3(threads), lds, s, a);
    }
}
