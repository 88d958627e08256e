/*
 * md_oracle.c -- plain, slow, FP64 CPU reference of the short-range MD hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library; the product path never does.
 * It shares no source, header, table or helper with the HIP library.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC, so
 * that every floating-point operation below is one individually rounded binary64
 * operation in the order written.  Only orc_verlet_omp (the all-cores CPU
 * baseline, at the end) runs threads; every other routine is serial.
 *
 * What it computes (the paper cites, but does not write out, the physics; the
 * definitions below are the textbook ones for the potentials the paper names):
 *   - linked cells of width >= cutoff, a particle interacting only with its own
 *     and the 26 surrounding cells (Sec. II.A);
 *   - Verlet neighbor lists generated cell by cell (Sec. II.A), full lists
 *     (each pair twice) or Newton-3 half lists (each pair once, Sec. II.D.3);
 *   - Lennard-Jones pair forces and a Finnis-Sinclair-type embedded-atom
 *     potential (the many-body family of Sec. II.C);
 *   - velocity-Verlet integration, "simple loops over the particles" (Sec. II.A);
 *   - hand-derived adjoints (vector-Jacobian products) of forces and energy.
 *
 * Conventions shared with every caller (readings of what the paper leaves open):
 *   positions are structure-of-arrays x[3][n]; boxes are orthorhombic, periodic,
 *   origin 0; wrap x -> x - L floor(x/L), then x >= L -> x - L, x < 0 -> 0;
 *   minimum image d > L/2 -> d - L, d < -L/2 -> d + L; r2 = (dx*dx + dy*dy) + dz*dz;
 *   a pair is inside a cutoff r iff r2 < r*r (strict).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define X(a, n, i) ((a)[(i)])
#define Y(a, n, i) ((a)[(n) + (i)])
#define Z(a, n, i) ((a)[2 * (n) + (i)])

/* ------------------------------------------------------------------------- */
/* periodic geometry                                                         */
/* ------------------------------------------------------------------------- */

static double wrap1(double x, double L)
{
    x = x - L * floor(x / L);
    if (x >= L) x = x - L;
    if (x < 0.0) x = 0.0;
    return x;
}

static double minimg1(double d, double L)
{
    if (d > 0.5 * L) d = d - L;
    else if (d < -0.5 * L) d = d + L;
    return d;
}

/* minimum-image separation d = x_i - x_j and its squared length */
static double sep(const double *x, int64_t n, int64_t i, int64_t j, const double L[3], double d[3])
{
    d[0] = minimg1(X(x, n, i) - X(x, n, j), L[0]);
    d[1] = minimg1(Y(x, n, i) - Y(x, n, j), L[1]);
    d[2] = minimg1(Z(x, n, i) - Z(x, n, j), L[2]);
    return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
}

void orc_wrap(int64_t n, double *x, const double L[3])
{
    for (int64_t i = 0; i < n; i++) {
        X(x, n, i) = wrap1(X(x, n, i), L[0]);
        Y(x, n, i) = wrap1(Y(x, n, i), L[1]);
        Z(x, n, i) = wrap1(Z(x, n, i), L[2]);
    }
}

/* ------------------------------------------------------------------------- */
/* linked cells (Sec. II.A): cells of width >= r_list, n_c = floor(L / r_list) */
/* ------------------------------------------------------------------------- */

/* returns 0, or -2 when some L_d < 2 r_list (minimum image not unique) */
int orc_grid(const double L[3], double rl, int32_t nc[3])
{
    for (int d = 0; d < 3; d++) {
        if (!(L[d] >= 2.0 * rl)) return -2;
        nc[d] = (int32_t)floor(L[d] / rl);
        if (nc[d] < 1) nc[d] = 1;
    }
    return 0;
}

static int32_t cell_coord(double x, int32_t nc, double L)
{
    int32_t c = (int32_t)floor(x * (double)nc / L);
    if (c > nc - 1) c = nc - 1;
    if (c < 0) c = 0;
    return c;
}

/* Bin wrapped positions.  cell index has x fastest.  order[] lists atoms cell
 * by cell, within a cell by ascending atom id (a stable counting sort). */
void orc_bin(int64_t n, const double *x, const double L[3], const int32_t nc[3],
             int32_t *cell_of, int32_t *cell_start, int32_t *order)
{
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    for (int64_t c = 0; c <= ncell; c++) cell_start[c] = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t cx = cell_coord(X(x, n, i), nc[0], L[0]);
        int32_t cy = cell_coord(Y(x, n, i), nc[1], L[1]);
        int32_t cz = cell_coord(Z(x, n, i), nc[2], L[2]);
        cell_of[i] = cx + nc[0] * (cy + nc[1] * cz);
        cell_start[cell_of[i] + 1] += 1;
    }
    for (int64_t c = 0; c < ncell; c++) cell_start[c + 1] += cell_start[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell > 0 ? ncell : 1));
    for (int64_t c = 0; c < ncell; c++) fill[c] = cell_start[c];
    for (int64_t i = 0; i < n; i++) order[fill[cell_of[i]]++] = (int32_t)i;
    free(fill);
}

/* the distinct cells of the 3x3x3 neighbourhood of (cx,cy,cz); returns count */
static int stencil(const int32_t nc[3], int32_t cx, int32_t cy, int32_t cz, int32_t out[27])
{
    int m = 0;
    for (int dz = -1; dz <= 1; dz++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                int32_t x = (cx + dx + nc[0]) % nc[0];
                int32_t y = (cy + dy + nc[1]) % nc[1];
                int32_t z = (cz + dz + nc[2]) % nc[2];
                int32_t c = x + nc[0] * (y + nc[1] * z);
                int dup = 0;
                for (int k = 0; k < m; k++) dup |= (out[k] == c);
                if (!dup) out[m++] = c;
            }
    return m;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------------- */
/* pair sets                                                                 */
/* ------------------------------------------------------------------------- */

/* All pairs with r2 < cut*cut by exhaustive enumeration.  full != 0: ordered
 * pairs (i, j), j != i; full == 0: i < j.  Writes up to cap pairs; returns the
 * total count. */
int64_t orc_pairs_brute(int64_t n, const double *x, const double L[3], double cut, int full,
                        int64_t cap, int32_t *pi, int32_t *pj)
{
    double cut2 = cut * cut, d[3];
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = full ? 0 : i + 1; j < n; j++) {
            if (j == i) continue;
            if (sep(x, n, i, j, L, d) < cut2) {
                if (m < cap) { pi[m] = (int32_t)i; pj[m] = (int32_t)j; }
                m++;
            }
        }
    return m;
}

/* Verlet lists built cell by cell (Sec. II.A): for every atom, the distinct
 * cells of its 27-cell neighbourhood are scanned and atoms with r2 < rl^2 kept.
 * x must be wrapped.  full == 1: every neighbour; full == 0: only neighbours
 * that come later in the cell-sorted order (rank[j] > rank[i]), so each pair is
 * held once (Sec. II.D.3); full == 2: the half list over 14 of the 27 cells
 * (Sec. II.D.3): j is kept when its cell, seen through the pair's minimum image,
 * lies in the forward half of the neighbourhood (shell_forward), so an atom's
 * partners lie in its own cell, the cell above in x, the three above in y and
 * the nine above in z -- a 3 x 3 x 2 block of cells.  start[n+1] receives
 * offsets; each atom's entries are ascending atom ids.  Writes up to cap
 * entries; returns the total. */
/* Unwrapped cell offset of j seen from i along one axis: j's cell, shifted by
 * nc when the minimum image moves j by a whole box (x_i - x_j > L/2: j is seen
 * at x_j + L), minus i's cell. */
static int32_t cell_offset(double xi, double xj, double L, int32_t ci, int32_t cj, int32_t nc)
{
    double d = xi - xj;
    int32_t s = d > 0.5 * L ? 1 : (d < -0.5 * L ? -1 : 0);
    return cj + s * nc - ci;
}

/* forward half of the cell neighbourhood: above in z; else above in y; else
 * above in x; within the same cell, later in the sorted order */
static int shell_forward(int32_t ox, int32_t oy, int32_t oz, int32_t ri, int32_t rj)
{
    if (oz != 0) return oz > 0;
    if (oy != 0) return oy > 0;
    if (ox != 0) return ox > 0;
    return rj > ri;
}

int64_t orc_neighbor_list(int64_t n, const double *x, const double L[3], double rl, int full,
                          int64_t *start, int64_t cap, int32_t *nbr)
{
    int32_t nc[3];
    if (orc_grid(L, rl, nc) != 0) return -2;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cstart = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    orc_bin(n, x, L, nc, cell_of, cstart, order);
    for (int64_t s = 0; s < n; s++) rank[order[s]] = (int32_t)s;
    double rl2 = rl * rl, d[3];
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t c = cell_of[i];
        int32_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
        int32_t cells[27];
        int ns = stencil(nc, cx, cy, cz, cells);
        start[i] = total;
        int64_t first = total;
        for (int k = 0; k < ns; k++)
            for (int32_t s = cstart[cells[k]]; s < cstart[cells[k] + 1]; s++) {
                int32_t j = order[s];
                if (j == i) continue;
                if (full == 0 && !(rank[j] > rank[i])) continue;
                if (full == 2) {
                    int32_t c2 = cell_of[j];
                    int32_t jx = c2 % nc[0], jy = (c2 / nc[0]) % nc[1], jz = c2 / (nc[0] * nc[1]);
                    int32_t ox = cell_offset(X(x, n, i), X(x, n, j), L[0], cx, jx, nc[0]);
                    int32_t oy = cell_offset(Y(x, n, i), Y(x, n, j), L[1], cy, jy, nc[1]);
                    int32_t oz = cell_offset(Z(x, n, i), Z(x, n, j), L[2], cz, jz, nc[2]);
                    if (!shell_forward(ox, oy, oz, rank[i], rank[j])) continue;
                }
                if (sep(x, n, i, j, L, d) < rl2) {
                    if (total < cap) nbr[total] = j;
                    total++;
                }
            }
        if (nbr != NULL && total <= cap)
            qsort(nbr + first, (size_t)(total - first), sizeof(int32_t), cmp_i32);
    }
    start[n] = total;
    free(cell_of); free(cstart); free(order); free(rank);
    return total;
}

/* ------------------------------------------------------------------------- */
/* Lennard-Jones: V(r) = 4 eps [(s/r)^12 - (s/r)^6] for r < rc (unshifted)   */
/* ------------------------------------------------------------------------- */

/* Forces, E = sum_{i<j} V and scalar virial W = sum_{i<j} d_ij . f_ij over an
 * explicit list of unordered pairs (each once); the rc test is applied here. */
void orc_lj(int64_t n, const double *x, const double L[3], double rc, double eps, double sigma,
            int64_t np, const int32_t *pi, const int32_t *pj, double *F, double ew[2])
{
    double rc2 = rc * rc, d[3], E = 0.0, W = 0.0;
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t p = 0; p < np; p++) {
        int64_t i = pi[p], j = pj[p];
        double r2 = sep(x, n, i, j, L, d);
        if (!(r2 < rc2)) continue;
        double sr2 = (sigma * sigma) / r2;
        double sr6 = sr2 * sr2 * sr2;
        double sr12 = sr6 * sr6;
        double V = 4.0 * eps * (sr12 - sr6);
        double fs = 24.0 * eps * (2.0 * sr12 - sr6) / r2;   /* f_ij = fs * d_ij */
        double f[3] = { fs * d[0], fs * d[1], fs * d[2] };
        X(F, n, i) += f[0]; Y(F, n, i) += f[1]; Z(F, n, i) += f[2];
        X(F, n, j) -= f[0]; Y(F, n, j) -= f[1]; Z(F, n, j) -= f[2];
        E += V;
        W += (d[0] * f[0] + d[1] * f[1]) + d[2] * f[2];
    }
    ew[0] = E;
    ew[1] = W;
}

/* Force and half pair energy (1/2 sum_j V) of selected atoms, by exhaustive
 * enumeration over all other atoms: an independent per-atom check usable on
 * systems far too large for a full O(N^2) pass. */
void orc_lj_atoms(int64_t n, const double *x, const double L[3], double rc, double eps,
                  double sigma, int64_t m, const int32_t *atoms, double *F, double *e)
{
    double rc2 = rc * rc, d[3];
    for (int64_t a = 0; a < m; a++) {
        int64_t i = atoms[a];
        double f[3] = { 0.0, 0.0, 0.0 }, ei = 0.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double r2 = sep(x, n, i, j, L, d);
            if (!(r2 < rc2)) continue;
            double sr2 = (sigma * sigma) / r2;
            double sr6 = sr2 * sr2 * sr2;
            double sr12 = sr6 * sr6;
            double fs = 24.0 * eps * (2.0 * sr12 - sr6) / r2;
            f[0] += fs * d[0]; f[1] += fs * d[1]; f[2] += fs * d[2];
            ei += 0.5 * (4.0 * eps * (sr12 - sr6));
        }
        F[a] = f[0]; F[m + a] = f[1]; F[2 * m + a] = f[2];
        e[a] = ei;
    }
}

/* ------------------------------------------------------------------------- */
/* uniform-knot cubic tables: f(x) = sum_p a_{k,p} t^p,  u = (x - x0) / h,    */
/* k = min(floor(u), n-2), t = u - k.  With extrap != 0, u > n-1 continues    */
/* linearly from the last knot (the embedding function beyond its table).     */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t n_knots;
    double x0, h;
    const double *coef; /* (n_knots - 1) x 4 */
} orc_spline;

typedef struct {
    orc_spline phi, rho, emb;
    double rc_phi, rc_rho;
} orc_eam_pot;

/* value and first two derivatives in x; also the interval k, t, and whether
 * the linear continuation was used */
static void spline_eval(const orc_spline *s, double x, int extrap, double *f, double *fp,
                        double *fpp, int32_t *kk, double *tt, int *lin)
{
    int32_t last = s->n_knots - 2;
    double inv_h = 1.0 / s->h;
    double u = (x - s->x0) * inv_h;
    if (extrap && u > (double)(s->n_knots - 1)) {
        const double *a = s->coef + 4 * (int64_t)last;
        double fend = a[0] + a[1] + a[2] + a[3];
        double sl = a[1] + 2.0 * a[2] + 3.0 * a[3];       /* df/dt at t = 1 */
        double e = u - (double)(s->n_knots - 1);
        *f = fend + sl * e;
        *fp = sl * inv_h;
        *fpp = 0.0;
        *kk = last; *tt = e; *lin = 1;
        return;
    }
    int32_t k = (int32_t)floor(u);
    if (k > last) k = last;
    if (k < 0) k = 0;
    double t = u - (double)k;
    const double *a = s->coef + 4 * (int64_t)k;
    double t2 = t * t, t3 = t2 * t;
    *f = a[0] + a[1] * t + a[2] * t2 + a[3] * t3;
    *fp = (a[1] + 2.0 * a[2] * t + 3.0 * a[3] * t2) * inv_h;
    *fpp = (2.0 * a[2] + 6.0 * a[3] * t) * (inv_h * inv_h);
    *kk = k; *tt = t; *lin = 0;
}

/* exported for tests of the tables themselves */
void orc_spline_eval(int32_t n_knots, double x0, double h, const double *coef, int extrap,
                     int64_t m, const double *xs, double *out /* [3][m]: f, f', f'' */)
{
    orc_spline s = { n_knots, x0, h, coef };
    int32_t k; double t; int lin;
    for (int64_t i = 0; i < m; i++)
        spline_eval(&s, xs[i], extrap, &out[i], &out[m + i], &out[2 * m + i], &k, &t, &lin);
}

static orc_eam_pot make_eam(const int32_t nk[3], const double x0[3], const double h[3],
                            const double *cphi, const double *crho, const double *cemb,
                            double rc_phi, double rc_rho)
{
    orc_eam_pot p;
    p.phi.n_knots = nk[0]; p.phi.x0 = x0[0]; p.phi.h = h[0]; p.phi.coef = cphi;
    p.rho.n_knots = nk[1]; p.rho.x0 = x0[1]; p.rho.h = h[1]; p.rho.coef = crho;
    p.emb.n_knots = nk[2]; p.emb.x0 = x0[2]; p.emb.h = h[2]; p.emb.coef = cemb;
    p.rc_phi = rc_phi; p.rc_rho = rc_rho;
    return p;
}

/* E = sum_i F(rho_i) + sum_{i<j} phi(r_ij), rho_i = sum_{j != i} rho(r_ij);
 * F_i = -sum_j [phi'(r) + (F'(rho_i) + F'(rho_j)) rho'(r)] d_ij / r.
 * Pairs are unordered (each once).  Also returns rho_i and F'(rho_i). */
static void eam_forces(int64_t n, const double *x, const double L[3], const orc_eam_pot *p,
                       int64_t np, const int32_t *pi, const int32_t *pj, double *F, double ew[2],
                       double *rho, double *Fp)
{
    double cphi2 = p->rc_phi * p->rc_phi, crho2 = p->rc_rho * p->rc_rho, d[3];
    double f, fp, fpp, t; int32_t k; int lin;
    double E = 0.0, W = 0.0;
    memset(rho, 0, sizeof(double) * (size_t)n);
    for (int64_t q = 0; q < np; q++) {
        int64_t i = pi[q], j = pj[q];
        double r2 = sep(x, n, i, j, L, d);
        if (r2 < crho2) {
            spline_eval(&p->rho, sqrt(r2), 0, &f, &fp, &fpp, &k, &t, &lin);
            rho[i] += f;
            rho[j] += f;
        }
    }
    for (int64_t i = 0; i < n; i++) {
        spline_eval(&p->emb, rho[i], 1, &f, &fp, &fpp, &k, &t, &lin);
        E += f;
        Fp[i] = fp;
    }
    memset(F, 0, sizeof(double) * 3 * (size_t)n);
    for (int64_t q = 0; q < np; q++) {
        int64_t i = pi[q], j = pj[q];
        double r2 = sep(x, n, i, j, L, d);
        double r = sqrt(r2), g = 0.0;
        if (r2 < cphi2) {
            spline_eval(&p->phi, r, 0, &f, &fp, &fpp, &k, &t, &lin);
            E += f;
            g += fp;
        }
        if (r2 < crho2) {
            spline_eval(&p->rho, r, 0, &f, &fp, &fpp, &k, &t, &lin);
            g += (Fp[i] + Fp[j]) * fp;
        }
        if (!(r2 < cphi2) && !(r2 < crho2)) continue;
        double fi[3] = { -g * d[0] / r, -g * d[1] / r, -g * d[2] / r };  /* force on i */
        X(F, n, i) += fi[0]; Y(F, n, i) += fi[1]; Z(F, n, i) += fi[2];
        X(F, n, j) -= fi[0]; Y(F, n, j) -= fi[1]; Z(F, n, j) -= fi[2];
        W += (d[0] * fi[0] + d[1] * fi[1]) + d[2] * fi[2];
    }
    ew[0] = E;
    ew[1] = W;
}

void orc_eam(int64_t n, const double *x, const double L[3], const int32_t nk[3],
             const double x0[3], const double h[3], const double *cphi, const double *crho,
             const double *cemb, double rc_phi, double rc_rho, int64_t np, const int32_t *pi,
             const int32_t *pj, double *F, double ew[2], double *rho, double *Fp)
{
    orc_eam_pot p = make_eam(nk, x0, h, cphi, crho, cemb, rc_phi, rc_rho);
    eam_forces(n, x, L, &p, np, pi, pj, F, ew, rho, Fp);
}

/* ------------------------------------------------------------------------- */
/* velocity Verlet with a displacement-triggered list rebuild                 */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t np, cap;
    int32_t *pi, *pj;
} pairlist;

/* half pair list within rl, by the linked-cell lists above */
static int build_pairs(int64_t n, const double *x, const double L[3], double rl, pairlist *pl)
{
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t tot = orc_neighbor_list(n, x, L, rl, 0, start, 0, NULL);
    if (tot < 0) { free(start); return -2; }
    int32_t *nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    orc_neighbor_list(n, x, L, rl, 0, start, tot, nbr);
    if (tot > pl->cap) {
        free(pl->pi); free(pl->pj);
        pl->cap = tot + tot / 4 + 16;
        pl->pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)pl->cap);
        pl->pj = (int32_t *)malloc(sizeof(int32_t) * (size_t)pl->cap);
    }
    for (int64_t i = 0; i < n; i++)
        for (int64_t s = start[i]; s < start[i + 1]; s++) { pl->pi[s] = (int32_t)i; pl->pj[s] = nbr[s]; }
    pl->np = tot;
    free(start); free(nbr);
    return 0;
}

/* kind 0 = LJ (lj[0] = eps, lj[1] = sigma), 1 = EAM (tables).  rc is the
 * interaction cutoff; lists use rl = rc + skin.  Forces at t = 0 are computed
 * first; each step: v += dt/(2m) F; x += dt v; wrap; rebuild the list if the
 * largest minimum-image displacement since the last build satisfies
 * |dx|^2 > (skin/2)^2; F <- F(x); v += dt/(2m) F; record (E_pot, KE, W).
 * F on entry is ignored; on exit it holds the final forces.  Returns 0 or -2. */
int orc_verlet(int64_t n, double *x, double *v, double *F, const double L[3], int kind,
               const double *lj, const int32_t nk[3], const double x0[3], const double h[3],
               const double *cphi, const double *crho, const double *cemb, double rc_phi,
               double rc_rho, double rc, double skin, double dt, double mass, int32_t nsteps,
               double *hist, int32_t *nrebuild)
{
    orc_eam_pot pot;
    if (kind == 1) pot = make_eam(nk, x0, h, cphi, crho, cemb, rc_phi, rc_rho);
    double rl = rc + skin;
    double thr = (0.5 * skin) * (0.5 * skin);
    double c = 0.5 * dt / mass;
    double ew[2], d[3];
    double *xref = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fp = (double *)malloc(sizeof(double) * (size_t)n);
    pairlist pl = { 0, 0, NULL, NULL };
    orc_wrap(n, x, L);
    if (build_pairs(n, x, L, rl, &pl) != 0) { free(xref); free(rho); free(Fp); return -2; }
    memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
    *nrebuild = 0;
    if (kind == 0) orc_lj(n, x, L, rc, lj[0], lj[1], pl.np, pl.pi, pl.pj, F, ew);
    else eam_forces(n, x, L, &pot, pl.np, pl.pi, pl.pj, F, ew, rho, Fp);
    for (int32_t s = 0; s < nsteps; s++) {
        for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + c * F[i];
        for (int64_t i = 0; i < 3 * n; i++) x[i] = x[i] + dt * v[i];
        orc_wrap(n, x, L);
        double dmax = 0.0;
        for (int64_t i = 0; i < n; i++) {
            double dd[3];
            dd[0] = minimg1(X(x, n, i) - X(xref, n, i), L[0]);
            dd[1] = minimg1(Y(x, n, i) - Y(xref, n, i), L[1]);
            dd[2] = minimg1(Z(x, n, i) - Z(xref, n, i), L[2]);
            double r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
            if (r2 > dmax) dmax = r2;
        }
        if (dmax > thr) {
            build_pairs(n, x, L, rl, &pl);
            memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
            *nrebuild += 1;
        }
        if (kind == 0) orc_lj(n, x, L, rc, lj[0], lj[1], pl.np, pl.pi, pl.pj, F, ew);
        else eam_forces(n, x, L, &pot, pl.np, pl.pi, pl.pj, F, ew, rho, Fp);
        for (int64_t i = 0; i < 3 * n; i++) v[i] = v[i] + c * F[i];
        double ke = 0.0;
        for (int64_t i = 0; i < n; i++)
            ke += (X(v, n, i) * X(v, n, i) + Y(v, n, i) * Y(v, n, i)) + Z(v, n, i) * Z(v, n, i);
        hist[3 * s + 0] = ew[0];
        hist[3 * s + 1] = 0.5 * mass * ke;
        hist[3 * s + 2] = ew[1];
    }
    (void)d;
    free(xref); free(rho); free(Fp); free(pl.pi); free(pl.pj);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* adjoints: given cotangents u (on F, [3][n]) and vE (on E), return           */
/*   g_x = d(vE E + u.F)/dx = -vE F - H u   and   g_theta = d(vE E + u.F)/dtheta */
/* ------------------------------------------------------------------------- */

/* LJ, theta = (eps, sigma).  Pairs unordered, each once. */
void orc_lj_vjp(int64_t n, const double *x, const double L[3], double rc, double eps,
                double sigma, int64_t np, const int32_t *pi, const int32_t *pj, const double *u,
                double vE, double *gx, double gp[2])
{
    double rc2 = rc * rc, d[3], ew[2];
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    orc_lj(n, x, L, rc, eps, sigma, np, pi, pj, F, ew);
    for (int64_t i = 0; i < 3 * n; i++) gx[i] = -vE * F[i];
    gp[0] = 0.0; gp[1] = 0.0;
    for (int64_t q = 0; q < np; q++) {
        int64_t i = pi[q], j = pj[q];
        double r2 = sep(x, n, i, j, L, d);
        if (!(r2 < rc2)) continue;
        double sr2 = (sigma * sigma) / r2;
        double sr6 = sr2 * sr2 * sr2;
        double sr12 = sr6 * sr6;
        double uij[3] = { X(u, n, i) - X(u, n, j), Y(u, n, i) - Y(u, n, j), Z(u, n, i) - Z(u, n, j) };
        double du = (d[0] * uij[0] + d[1] * uij[1]) + d[2] * uij[2];
        /* Hessian block K = V'' rr^T + (V'/r)(I - rr^T):  K u = B u + C (d.u) d */
        double B = -24.0 * eps * (2.0 * sr12 - sr6) / r2;
        double C = 96.0 * eps * (7.0 * sr12 - 2.0 * sr6) / (r2 * r2);
        for (int a = 0; a < 3; a++) {
            double hu = B * uij[a] + C * du * d[a];
            gx[a * n + i] -= hu;
            gx[a * n + j] += hu;
        }
        /* dV/deps, dV/dsigma and d(u_ij . f_ij)/deps, /dsigma */
        double dV_de = 4.0 * (sr12 - sr6);
        double dV_ds = 24.0 * eps * (2.0 * sr12 - sr6) / sigma;
        double duf_de = du * 24.0 * (2.0 * sr12 - sr6) / r2;
        double duf_ds = du * 144.0 * eps * (4.0 * sr12 - sr6) / (sigma * r2);
        gp[0] += vE * dV_de + duf_de;
        gp[1] += vE * dV_ds + duf_ds;
    }
    free(F);
}

/* EAM: theta = the three coefficient tables.  g_phi, g_rho, g_emb have the
 * tables' shapes ((n_knots-1) x 4) and are overwritten. */
void orc_eam_vjp(int64_t n, const double *x, const double L[3], const int32_t nk[3],
                 const double x0[3], const double h[3], const double *cphi, const double *crho,
                 const double *cemb, double rc_phi, double rc_rho, int64_t np, const int32_t *pi,
                 const int32_t *pj, const double *u, double vE, double *gx, double *g_phi,
                 double *g_rho, double *g_emb)
{
    orc_eam_pot p = make_eam(nk, x0, h, cphi, crho, cemb, rc_phi, rc_rho);
    double cphi2 = rc_phi * rc_phi, crho2 = rc_rho * rc_rho, d[3], ew[2];
    double f, fp, fpp, t; int32_t k; int lin;
    double *F = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fp = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fpp = (double *)malloc(sizeof(double) * (size_t)n);
    double *rdot = (double *)calloc((size_t)n, sizeof(double));
    eam_forces(n, x, L, &p, np, pi, pj, F, ew, rho, Fp);
    memset(g_phi, 0, sizeof(double) * 4 * (size_t)(nk[0] - 1));
    memset(g_rho, 0, sizeof(double) * 4 * (size_t)(nk[1] - 1));
    memset(g_emb, 0, sizeof(double) * 4 * (size_t)(nk[2] - 1));
    for (int64_t i = 0; i < n; i++) {
        spline_eval(&p.emb, rho[i], 1, &f, &fp, &fpp, &k, &t, &lin);
        Fpp[i] = fpp;
    }
    /* pass A: rho-dot_i = sum_j rho'(r_ij) s_ij,  s_ij = (d_ij / r) . (u_i - u_j) */
    for (int64_t q = 0; q < np; q++) {
        int64_t i = pi[q], j = pj[q];
        double r2 = sep(x, n, i, j, L, d);
        if (!(r2 < crho2)) continue;
        double r = sqrt(r2);
        double uij[3] = { X(u, n, i) - X(u, n, j), Y(u, n, i) - Y(u, n, j), Z(u, n, i) - Z(u, n, j) };
        double s = ((d[0] * uij[0] + d[1] * uij[1]) + d[2] * uij[2]) / r;
        spline_eval(&p.rho, r, 0, &f, &fp, &fpp, &k, &t, &lin);
        rdot[i] += fp * s;
        rdot[j] += fp * s;
    }
    for (int64_t i = 0; i < 3 * n; i++) gx[i] = -vE * F[i];
    /* pass B: Hessian-vector product and pair parameter terms */
    for (int64_t q = 0; q < np; q++) {
        int64_t i = pi[q], j = pj[q];
        double r2 = sep(x, n, i, j, L, d);
        int in_phi = r2 < cphi2, in_rho = r2 < crho2;
        if (!in_phi && !in_rho) continue;
        double r = sqrt(r2);
        double e[3] = { d[0] / r, d[1] / r, d[2] / r };
        double uij[3] = { X(u, n, i) - X(u, n, j), Y(u, n, i) - Y(u, n, j), Z(u, n, i) - Z(u, n, j) };
        double s = (e[0] * uij[0] + e[1] * uij[1]) + e[2] * uij[2];
        double ph = 0, php = 0, phpp = 0, rh = 0, rhp = 0, rhpp = 0;
        int32_t kphi = 0, krho = 0; double tphi = 0, trho = 0;
        if (in_phi) spline_eval(&p.phi, r, 0, &ph, &php, &phpp, &kphi, &tphi, &lin);
        if (in_rho) spline_eval(&p.rho, r, 0, &rh, &rhp, &rhpp, &krho, &trho, &lin);
        double Fs = Fp[i] + Fp[j];
        double g = php + Fs * rhp;
        double gg = phpp + Fs * rhpp;
        double qq = Fpp[i] * rdot[i] + Fpp[j] * rdot[j];
        for (int a = 0; a < 3; a++) {
            double hu = gg * s * e[a] + (g / r) * (uij[a] - s * e[a]) + qq * rhp * e[a];
            gx[a * n + i] -= hu;
            gx[a * n + j] += hu;
        }
        double inv_hphi = 1.0 / p.phi.h, inv_hrho = 1.0 / p.rho.h;
        if (in_phi) {
            double tp[4] = { 1.0, tphi, tphi * tphi, tphi * tphi * tphi };
            for (int pw = 0; pw < 4; pw++) {
                double dtp = pw == 0 ? 0.0 : (double)pw * tp[pw - 1];
                g_phi[4 * (int64_t)kphi + pw] += vE * tp[pw] - s * dtp * inv_hphi;
            }
        }
        if (in_rho) {
            double tp[4] = { 1.0, trho, trho * trho, trho * trho * trho };
            for (int pw = 0; pw < 4; pw++) {
                double dtp = pw == 0 ? 0.0 : (double)pw * tp[pw - 1];
                g_rho[4 * (int64_t)krho + pw] += vE * Fs * tp[pw] - (s * Fs * dtp * inv_hrho + qq * tp[pw]);
            }
        }
    }
    /* embedding-table terms, one per atom */
    double inv_hemb = 1.0 / p.emb.h;
    for (int64_t i = 0; i < n; i++) {
        spline_eval(&p.emb, rho[i], 1, &f, &fp, &fpp, &k, &t, &lin);
        for (int pw = 0; pw < 4; pw++) {
            double dF, dFp;
            if (lin) {                       /* F = sum_p a_p + (sum_p p a_p) e, e = u - (n-1) */
                dF = 1.0 + (double)pw * t;
                dFp = (double)pw * inv_hemb;
            } else {
                double tp = pw == 0 ? 1.0 : (pw == 1 ? t : (pw == 2 ? t * t : t * t * t));
                double dtp = pw == 0 ? 0.0 : (pw == 1 ? 1.0 : (pw == 2 ? 2.0 * t : 3.0 * t * t));
                dF = tp;
                dFp = dtp * inv_hemb;
            }
            g_emb[4 * (int64_t)k + pw] += vE * dF - rdot[i] * dFp;
        }
    }
    free(F); free(rho); free(Fp); free(Fpp); free(rdot);
}

/* ------------------------------------------------------------------------- */
/* the same velocity Verlet threaded with OpenMP over atoms                   */
/* ------------------------------------------------------------------------- */
/* A CPU baseline on all host cores, not a reference: the serial orc_verlet
 * above is the definition this one is tested against.  It uses full lists
 * (every pair in both atoms' lists), so each thread computes and writes only
 * its own atoms' forces and no two threads update one particle -- the
 * invariant of Sec. II.A obtained by ownership, as the naive threaded loop of
 * Sec. I without Newton's third law.  Energies are summed per atom (half of
 * every listed pair) with a reduction whose order depends on the threads. */

typedef struct {
    int64_t cap;
    int64_t *start;   /* [n+1] */
    int32_t *nbr;
} fulllist;

static int build_full_omp(int64_t n, const double *x, const double L[3], double rl, fulllist *fl)
{
    int32_t nc[3];
    if (orc_grid(L, rl, nc) != 0) return -2;
    int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
    int32_t *cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *cstart = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncell + 1));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    orc_bin(n, x, L, nc, cell_of, cstart, order);
    double rl2 = rl * rl;
    for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; i++) {
            int32_t c = cell_of[i];
            int32_t cx = c % nc[0], cy = (c / nc[0]) % nc[1], cz = c / (nc[0] * nc[1]);
            int32_t cells[27];
            int ns = stencil(nc, cx, cy, cz, cells);
            int64_t m = 0, o = pass ? fl->start[i] : 0;
            double d[3];
            for (int k = 0; k < ns; k++)
                for (int32_t s = cstart[cells[k]]; s < cstart[cells[k] + 1]; s++) {
                    int32_t j = order[s];
                    if (j == i || !(sep(x, n, i, j, L, d) < rl2)) continue;
                    if (pass) fl->nbr[o + m] = j;
                    m++;
                }
            if (!pass) cnt[i] = m;
        }
        if (!pass) {
            if (fl->start == NULL) fl->start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
            fl->start[0] = 0;
            for (int64_t i = 0; i < n; i++) fl->start[i + 1] = fl->start[i] + cnt[i];
            if (fl->start[n] > fl->cap) {
                free(fl->nbr);
                fl->cap = fl->start[n] + fl->start[n] / 4 + 16;
                fl->nbr = (int32_t *)malloc(sizeof(int32_t) * (size_t)fl->cap);
            }
        }
    }
    free(cell_of); free(cstart); free(order); free(cnt);
    return 0;
}

/* forces over the full lists; ew = (E, W) */
static void full_forces_omp(int64_t n, const double *x, const double L[3], int kind, double rc,
                            const double *lj, const orc_eam_pot *p, const fulllist *fl, double *F,
                            double ew[2], double *rho, double *Fp)
{
    double E = 0.0, W = 0.0;
    if (kind == 0) {
        double rc2 = rc * rc, eps = lj[0], sigma = lj[1];
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : E, W)
        for (int64_t i = 0; i < n; i++) {
            double f[3] = { 0.0, 0.0, 0.0 }, d[3];
            for (int64_t q = fl->start[i]; q < fl->start[i + 1]; q++) {
                int64_t j = fl->nbr[q];
                double r2 = sep(x, n, i, j, L, d);
                if (!(r2 < rc2)) continue;
                double sr2 = (sigma * sigma) / r2;
                double sr6 = sr2 * sr2 * sr2;
                double sr12 = sr6 * sr6;
                double fs = 24.0 * eps * (2.0 * sr12 - sr6) / r2;
                f[0] += fs * d[0]; f[1] += fs * d[1]; f[2] += fs * d[2];
                E += 0.5 * (4.0 * eps * (sr12 - sr6));
                W += 0.5 * ((d[0] * fs * d[0] + d[1] * fs * d[1]) + d[2] * fs * d[2]);
            }
            X(F, n, i) = f[0]; Y(F, n, i) = f[1]; Z(F, n, i) = f[2];
        }
    } else {
        double cphi2 = p->rc_phi * p->rc_phi, crho2 = p->rc_rho * p->rc_rho;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : E)
        for (int64_t i = 0; i < n; i++) {
            double d[3], f, fp, fpp, t; int32_t k; int lin;
            double ri = 0.0;
            for (int64_t q = fl->start[i]; q < fl->start[i + 1]; q++) {
                double r2 = sep(x, n, i, fl->nbr[q], L, d);
                if (!(r2 < crho2)) continue;
                spline_eval(&p->rho, sqrt(r2), 0, &f, &fp, &fpp, &k, &t, &lin);
                ri += f;
            }
            rho[i] = ri;
            spline_eval(&p->emb, ri, 1, &f, &fp, &fpp, &k, &t, &lin);
            Fp[i] = fp;
            E += f;
        }
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : E, W)
        for (int64_t i = 0; i < n; i++) {
            double d[3], f, fp, fpp, t; int32_t k; int lin;
            double fi[3] = { 0.0, 0.0, 0.0 };
            for (int64_t q = fl->start[i]; q < fl->start[i + 1]; q++) {
                int64_t j = fl->nbr[q];
                double r2 = sep(x, n, i, j, L, d);
                int in_phi = r2 < cphi2, in_rho = r2 < crho2;
                if (!in_phi && !in_rho) continue;
                double r = sqrt(r2), g = 0.0;
                if (in_phi) {
                    spline_eval(&p->phi, r, 0, &f, &fp, &fpp, &k, &t, &lin);
                    E += 0.5 * f;
                    g += fp;
                }
                if (in_rho) {
                    spline_eval(&p->rho, r, 0, &f, &fp, &fpp, &k, &t, &lin);
                    g += (Fp[i] + Fp[j]) * fp;
                }
                double c[3] = { -g * d[0] / r, -g * d[1] / r, -g * d[2] / r };
                fi[0] += c[0]; fi[1] += c[1]; fi[2] += c[2];
                W += 0.5 * ((d[0] * c[0] + d[1] * c[1]) + d[2] * c[2]);
            }
            X(F, n, i) = fi[0]; Y(F, n, i) = fi[1]; Z(F, n, i) = fi[2];
        }
    }
    ew[0] = E;
    ew[1] = W;
}

/* Arguments and history as orc_verlet; nthreads > 0 sets the thread count.
 * Returns 0, or -2 (box too small). */
int orc_verlet_omp(int64_t n, double *x, double *v, double *F, const double L[3], int kind,
                   const double *lj, const int32_t nk[3], const double x0[3], const double h[3],
                   const double *cphi, const double *crho, const double *cemb, double rc_phi,
                   double rc_rho, double rc, double skin, double dt, double mass, int32_t nsteps,
                   double *hist, int32_t *nrebuild, int32_t nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    orc_eam_pot pot;
    memset(&pot, 0, sizeof(pot));
    if (kind == 1) pot = make_eam(nk, x0, h, cphi, crho, cemb, rc_phi, rc_rho);
    double rl = rc + skin;
    double thr = (0.5 * skin) * (0.5 * skin);
    double c = 0.5 * dt / mass;
    double ew[2];
    double *xref = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * (size_t)n);
    double *Fp = (double *)malloc(sizeof(double) * (size_t)n);
    fulllist fl = { 0, NULL, NULL };
    orc_wrap(n, x, L);
    if (build_full_omp(n, x, L, rl, &fl) != 0) { free(xref); free(rho); free(Fp); return -2; }
    memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
    *nrebuild = 0;
    full_forces_omp(n, x, L, kind, rc, lj, &pot, &fl, F, ew, rho, Fp);
    for (int32_t s = 0; s < nsteps; s++) {
        double dmax = 0.0;
#pragma omp parallel for reduction(max : dmax)
        for (int64_t i = 0; i < n; i++) {
            for (int a = 0; a < 3; a++) {
                v[a * n + i] = v[a * n + i] + c * F[a * n + i];
                x[a * n + i] = x[a * n + i] + dt * v[a * n + i];
                x[a * n + i] = wrap1(x[a * n + i], L[a]);
            }
            double dd[3];
            dd[0] = minimg1(X(x, n, i) - X(xref, n, i), L[0]);
            dd[1] = minimg1(Y(x, n, i) - Y(xref, n, i), L[1]);
            dd[2] = minimg1(Z(x, n, i) - Z(xref, n, i), L[2]);
            double r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
            if (r2 > dmax) dmax = r2;
        }
        if (dmax > thr) {
            build_full_omp(n, x, L, rl, &fl);
            memcpy(xref, x, sizeof(double) * 3 * (size_t)n);
            *nrebuild += 1;
        }
        full_forces_omp(n, x, L, kind, rc, lj, &pot, &fl, F, ew, rho, Fp);
        double ke = 0.0;
#pragma omp parallel for reduction(+ : ke)
        for (int64_t i = 0; i < n; i++) {
            for (int a = 0; a < 3; a++) v[a * n + i] = v[a * n + i] + c * F[a * n + i];
            ke += (X(v, n, i) * X(v, n, i) + Y(v, n, i) * Y(v, n, i)) + Z(v, n, i) * Z(v, n, i);
        }
        hist[3 * s + 0] = ew[0];
        hist[3 * s + 1] = 0.5 * mass * ke;
        hist[3 * s + 2] = ew[1];
    }
    free(xref); free(rho); free(Fp); free(fl.start); free(fl.nbr);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
