// md_vjp.hip -- hand-written adjoints of forces and energy.
//
// For cotangents u (on F) and v (on E, one per replica) the kernels return
//   g_x = d(v E + u.F)/dx = -v F - H u      and the parameter gradient.
// Derivation (d = x_i - x_j, r = |d|, e = d/r, u_ij = u_i - u_j, s = e.u_ij):
//   LJ:  H u |_i = sum_j [B u_ij + C (d.u_ij) d],  B = -24 eps (2 q12 - q6)/r^2,
//        C = 96 eps (7 q12 - 2 q6)/r^4,  q6 = (sigma/r)^6, q12 = q6^2;
//        dV/deps = 4 (q12 - q6), dV/dsigma = 24 eps (2 q12 - q6)/sigma,
//        d(u_ij.f_ij)/deps = (d.u_ij) 24 (2 q12 - q6)/r^2,
//        d(u_ij.f_ij)/dsigma = (d.u_ij) 144 eps (4 q12 - q6)/(sigma r^2).
//   EAM: pass A gives rho_i, F'_i, F''_i and rho-dot_i = sum_j rho'(r) s;
//        H u |_i = sum_j { [phi'' + (F'_i+F'_j) rho''] s e + (g/r)(u_ij - s e)
//                          + (F''_i rho-dot_i + F''_j rho-dot_j) rho' e },
//        g = phi' + (F'_i + F'_j) rho';  table coefficient (k, p) gradients are
//        histograms over pairs (phi, rho) and atoms (embedding) of t^p and
//        p t^(p-1)/h weights.
// The kernels are brick tasks like the force kernels (md_brick.h), one lane per
// atom.  The full list visits every pair from both atoms, so position terms
// need no atomics; pair parameter terms are taken once per pair (j after i).
// The adjoint always evaluates in binary64.
#include <math.h>

#include "md_brick.h"
#include "md_reduce.h"

namespace {

// row k, t and value / d/du / d2/du2 of a binary64 table at u
__device__ __forceinline__ void spl_full(const double *tab, double u, int nk, int &k, double &t,
                                         double &f, double &fu, double &fuu)
{
    k = (int)floor(u);
    k = k > nk - 2 ? nk - 2 : k;
    k = k < 0 ? 0 : k;
    t = u - (double)k;
    const double4 c = reinterpret_cast<const double4 *>(tab)[k];
    f = c.x + t * (c.y + t * (c.z + t * c.w));
    fu = c.y + t * (2.0 * c.z + 3.0 * t * c.w);
    fuu = 2.0 * c.z + 6.0 * t * c.w;
}

// embedding with linear continuation: F, F', F'', row k, t (t = u - (nk-1) when lin)
__device__ __forceinline__ void embed_full(const ForceArgs &a, double rho, double &F, double &Fp,
                                           double &Fpp, int &k, double &t, bool &lin)
{
    const int nk = a.nk[2];
    const double ih = a.inv_h[2];
    const double u = (rho - a.x0[2]) * ih;
    if (u > (double)(nk - 1)) {
        const double4 c = reinterpret_cast<const double4 *>(a.tab[2])[nk - 2];
        const double fend = ((c.x + c.y) + c.z) + c.w;
        const double sl = (c.y + 2.0 * c.z) + 3.0 * c.w;
        t = u - (double)(nk - 1);
        F = fend + sl * t;
        Fp = sl * ih;
        Fpp = 0.0;
        k = nk - 2;
        lin = true;
        return;
    }
    double fu, fuu;
    spl_full(a.tab[2], u, nk, k, t, F, fu, fuu);
    Fp = fu * ih;
    Fpp = fuu * (ih * ih);
    lin = false;
}

// binary64 add to an LDS word shared by the workgroup's lanes
__device__ __forceinline__ void lds_add(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// ---------------------------------------------------------------- LJ
// Partner cotangent u_j of candidate k: from the LDS stage (extras ex0..ex0+2)
// when the kernel stages it (STAGE_U) and k is staged, else gathered from HBM.
template <bool STAGE_U, bool STAGED>
__device__ __forceinline__ double4 partner_u(const Stage &st, const BrickDims &bd, const double4 *u, int32_t k,
                                             int ex0)
{
    if (STAGE_U && (STAGED || k < st.cap)) {
        const double *e = st.ex + (size_t)ex0 * st.cap + k;
        return make_double4(e[0], e[st.cap], e[2 * (size_t)st.cap], 0.0);
    }
    const int32_t j = STAGE_U ? candidate_index(st, bd, k) : candidate_j<STAGED>(st, bd, k);
    return at32(u, j);
}

// two 512-thread workgroups per CU (at most 128 VGPRs).  STAGE_U: the partner
// cotangents are staged in LDS beside the positions (when the larger stage
// fits the LDS), instead of gathered from HBM per pair.
template <bool STAGE_U>
__global__ __launch_bounds__(TASK_MAX_THREADS, 4) void k_lj_vjp(VjpArgs v)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double lds[4 * TASK_MAX_THREADS / 64];
    const ForceArgs &a = v.f;
    const Stage st = stage_slice(lds_raw, a.cap, STAGE_U ? 3 : 0, !STAGE_U);
    const int64_t n = a.n;
    const double eps = a.lj[0], sig = a.lj[1];
    const double s2 = sig * sig;
    const double rc2 = a.rc2;
    const double e24 = 24.0 * eps;
    double acc_e = 0.0, acc_s = 0.0;
    BRICK_TASK_BEGIN_V(st, a.pos, nullptr, nullptr, STAGE_U ? v.u : nullptr, 0)
        double F[3] = {0.0, 0.0, 0.0}, Hu[3] = {0.0, 0.0, 0.0};
        const double vE = v.vE[rep_r];
        const double4 xi = a.pos[i];
        const double4 ui4 = v.u[i];
        const double ui[3] = {ui4.x, ui4.y, ui4.z};
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    if (!ok || !(r2 < rc2)) return;
                    const double d[3] = {dx, dy, dz};
                    const double ir2 = rcp64(r2);
                    const double q2 = s2 * ir2;
                    const double q6 = q2 * q2 * q2;
                    const double q12 = q6 * q6;
                    const double t2 = 2.0 * q12 - q6;
                    const double t2r = t2 * ir2;
                    const double fs = e24 * t2r;
                    const double B = -fs;
                    const double C = 96.0 * eps * (7.0 * q12 - 2.0 * q6) * (ir2 * ir2);
                    const double4 uj = partner_u<STAGE_U, STAGED>(st, a.bd, v.u, k, 0);
                    const double uij[3] = {ui[0] - uj.x, ui[1] - uj.y, ui[2] - uj.z};
                    const double du = (d[0] * uij[0] + d[1] * uij[1]) + d[2] * uij[2];
                    const double Cd = C * du;
                    for (int c = 0; c < 3; c++) {
                        F[c] = fma(fs, d[c], F[c]);
                        Hu[c] = fma(B, uij[c], fma(Cd, d[c], Hu[c]));
                    }
                    // parameter terms, the common factors applied once at the end:
                    // vE dV/deps + d(u.f)/deps = 4 [vE (q12 - q6) + 6 du t2 / r^2],
                    // vE dV/dsigma + d(u.f)/dsigma = (24 eps / sigma) [vE t2 + 6 du (4 q12 - q6) / r^2]
                    const double du6 = 6.0 * du;
                    acc_e += fma(vE, q12 - q6, du6 * t2r);
                    acc_s += fma(vE, t2, du6 * ((4.0 * q12 - q6) * ir2));
                });
        )
        if (valid)
            for (int c = 0; c < 3; c++) v.gx[c * n + i] = -vE * F[c] - Hu[c];
    BRICK_TASK_END
    // each unordered pair is visited twice: half weight
    double s[4] = {2.0 * acc_e, 12.0 * eps * acc_s / sig, 0.0, 0.0};
    if (v.gout != nullptr) mdred::block_to_partial4(s, v.gpart, lds);
}

// ---------------------------------------------------------------- EAM pass A
// rho_i, F'_i and q_i = F''_i rho-dot_i (v.fpp holds q: pass B needs F'' only
// in that product).
template <bool STAGE_U>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_eam_vjp_a(VjpArgs v)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ForceArgs &a = v.f;
    const Stage st = stage_slice(lds_raw, a.cap, STAGE_U ? 3 : 0, !STAGE_U);
    const int nkr = a.nk[1];
    const double x0r = a.x0[1], ihr = a.inv_h[1], rrho2 = a.rrho2;
    BRICK_TASK_BEGIN_V(st, a.pos, nullptr, nullptr, STAGE_U ? v.u : nullptr, 0)
        double rho = 0.0, rdot = 0.0;
        const double4 xi = a.pos[i];
        const double4 ui4 = v.u[i];
        const double ui[3] = {ui4.x, ui4.y, ui4.z};
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    if (!ok || !(r2 < rrho2)) return;
                    const double r = sqrt_pair(r2);
                    int kk;
                    double tt, f, fu, fuu;
                    spl_full(a.tab[1], (r - x0r) * ihr, nkr, kk, tt, f, fu, fuu);
                    const double4 uj = partner_u<STAGE_U, STAGED>(st, a.bd, v.u, k, 0);
                    const double uij[3] = {ui[0] - uj.x, ui[1] - uj.y, ui[2] - uj.z};
                    const double s = ((dx * uij[0] + dy * uij[1]) + dz * uij[2]) * rcp64(r);
                    rho += f;
                    rdot += (fu * ihr) * s;
                });
        )
        if (valid) {
            double F, Fp, Fpp, tt;
            int kk;
            bool lin;
            embed_full(a, rho, F, Fp, Fpp, kk, tt, lin);
            a.rho[i] = rho;
            a.fp[i] = Fp;
            v.fpp[i] = Fpp * rdot;
            v.rdot[i] = rdot;
        }
    BRICK_TASK_END
}

// ---------------------------------------------------------------- EAM pass B
// STAGE_U: the partners' F', q = F'' rho-dot and cotangent are staged in LDS
// beside their positions (extras 0, 1 and 2..4) instead of gathered per pair.
template <bool STAGE_U>
__global__ __launch_bounds__(TASK_MAX_THREADS) void k_eam_vjp_b(VjpArgs v)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ForceArgs &a = v.f;
    const Stage st = stage_slice(lds_raw, a.cap, STAGE_U ? 5 : 0, true);
    const int64_t n = a.n;
    const int nkp = a.nk[0], nkr = a.nk[1];
    const double x0p = a.x0[0], ihp = a.inv_h[0], x0r = a.x0[1], ihr = a.inv_h[1];
    const double rphi2 = a.rphi2, rrho2 = a.rrho2;
    double *gphi = v.gtab;
    double *grho = v.gtab + 4 * (int64_t)(nkp - 1);
    // the last gw_p (gw_r) intervals of the phi (rho) table, where the pairs of
    // a crystal fall, are summed in LDS and added to the gradient once per
    // workgroup; pairs below them add to it directly
    const int32_t wp = v.gtab != nullptr ? v.gw_p : 0, wr = v.gtab != nullptr ? v.gw_r : 0;
    const int32_t kp0 = nkp - 1 - wp, kr0 = nkr - 1 - wr;
    double *lphi = reinterpret_cast<double *>(lds_raw + v.gw_off), *lrho = lphi + 4 * wp;
    for (int32_t t = threadIdx.x; t < 4 * (wp + wr); t += blockDim.x) lphi[t] = 0.0;
    __syncthreads();
    BRICK_TASK_BEGIN_V(st, a.pos, STAGE_U ? a.fp : nullptr, STAGE_U ? v.fpp : nullptr,
                       STAGE_U ? v.u : nullptr, 2)
        double F[3] = {0.0, 0.0, 0.0}, Hu[3] = {0.0, 0.0, 0.0};
        const double vE = v.vE[rep_r];
        const double4 xi = a.pos[i];
        const double4 ui4 = v.u[i];
        const double ui[3] = {ui4.x, ui4.y, ui4.z};
        const double fpi = a.fp[i];
        const double qi = v.fpp[i];
        STAGE_IMG_SPLIT(all_staged, has_img,
            walk_list<STAGED, IMG>(st, a.bd, a.pos, a.nbr, i, a.M, mm, xi, Lx, Ly, Lz,
                [&](bool ok, int32_t k, double dx, double dy, double dz, double r2) {
                    const bool in_phi = r2 < rphi2, in_rho = r2 < rrho2;
                    if (!ok || (!in_phi && !in_rho)) return;
                    // partner index (the parameter sums take each pair once, j > i),
                    // F'_j and q_j, staged or gathered
                    const int32_t j = candidate_j<STAGED>(st, a.bd, k);
                    double fpj, qj;
                    if (STAGE_U && (STAGED || k < st.cap)) {
                        fpj = st.ex[k];
                        qj = st.ex[st.cap + k];
                    } else {
                        fpj = at32(a.fp, j);
                        qj = at32(v.fpp, j);
                    }
                    const double r = sqrt_pair(r2);
                    // one refined reciprocal instead of four divisions
                    const double ir = rcp64(r);
                    const double e[3] = {dx * ir, dy * ir, dz * ir};
                    const double4 uj = partner_u<STAGE_U, STAGED>(st, a.bd, v.u, k, 2);
                    const double uij[3] = {ui[0] - uj.x, ui[1] - uj.y, ui[2] - uj.z};
                    const double s = (e[0] * uij[0] + e[1] * uij[1]) + e[2] * uij[2];
                    double ph = 0.0, php = 0.0, phpp = 0.0, rh = 0.0, rhp = 0.0, rhpp = 0.0;
                    double tp = 0.0, tr = 0.0;
                    int kp = 0, kr = 0;
                    if (in_phi) {
                        double fu, fuu;
                        spl_full(a.tab[0], (r - x0p) * ihp, nkp, kp, tp, ph, fu, fuu);
                        php = fu * ihp;
                        phpp = fuu * (ihp * ihp);
                    }
                    if (in_rho) {
                        double fu, fuu;
                        spl_full(a.tab[1], (r - x0r) * ihr, nkr, kr, tr, rh, fu, fuu);
                        rhp = fu * ihr;
                        rhpp = fuu * (ihr * ihr);
                    }
                    const double Fs = fpi + fpj;
                    const double gsc = php + Fs * rhp;
                    const double gg = phpp + Fs * rhpp;
                    const double qq = qi + qj;
                    // H u along e and along u_ij: (gg s - (gsc/r) s + qq rho') e + (gsc/r) u_ij
                    const double G = gsc * ir;
                    const double Ae = fma(gg - G, s, qq * rhp);
                    for (int c = 0; c < 3; c++) {
                        F[c] -= gsc * e[c];
                        Hu[c] = fma(G, uij[c], fma(Ae, e[c], Hu[c]));
                    }
                    if (v.gtab != nullptr && j > i) {
                        if (in_phi) {
                            const double t2 = tp * tp;
                            const double pw[4] = {1.0, tp, t2, t2 * tp};
                            const double dp[4] = {0.0, 1.0, 2.0 * tp, 3.0 * t2};
                            double gv[4];
                            for (int p = 0; p < 4; p++) gv[p] = vE * pw[p] - s * dp[p] * ihp;
                            // LDS sums at workgroup scope, HBM sums at agent scope: the
                            // two kinds of atomics cannot be merged into flat atomics
                            if (kp >= kp0)
                                for (int p = 0; p < 4; p++) lds_add(&lphi[4 * (kp - kp0) + p], gv[p]);
                            else
                                for (int p = 0; p < 4; p++) atomicAdd(&gphi[4 * (int64_t)kp + p], gv[p]);
                        }
                        if (in_rho) {
                            const double t2 = tr * tr;
                            const double pw[4] = {1.0, tr, t2, t2 * tr};
                            const double dp[4] = {0.0, 1.0, 2.0 * tr, 3.0 * t2};
                            double gv[4];
                            for (int p = 0; p < 4; p++) gv[p] = vE * Fs * pw[p] - (s * Fs * dp[p] * ihr + qq * pw[p]);
                            if (kr >= kr0)
                                for (int p = 0; p < 4; p++) lds_add(&lrho[4 * (kr - kr0) + p], gv[p]);
                            else
                                for (int p = 0; p < 4; p++) atomicAdd(&grho[4 * (int64_t)kr + p], gv[p]);
                        }
                    }
                });
        )
        if (valid)
            for (int c = 0; c < 3; c++) v.gx[c * n + i] = -vE * F[c] - Hu[c];
    BRICK_TASK_END
    __syncthreads();
    for (int32_t t = threadIdx.x; t < 4 * wp; t += blockDim.x)
        if (lphi[t] != 0.0) atomicAdd(&gphi[4 * (int64_t)kp0 + t], lphi[t]);
    for (int32_t t = threadIdx.x; t < 4 * wr; t += blockDim.x)
        if (lrho[t] != 0.0) atomicAdd(&grho[4 * (int64_t)kr0 + t], lrho[t]);
}

// embedding-table gradient: one entry per atom
__global__ __launch_bounds__(256) void k_eam_vjp_embed(VjpArgs v)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const ForceArgs &a = v.f;
    const int64_t n = a.n;
    const int nkp = a.nk[0], nkr = a.nk[1];
    double *gemb = v.gtab + 4 * (int64_t)(nkp - 1) + 4 * (int64_t)(nkr - 1);
    const double ih = a.inv_h[2];
    // with gw_p > 0 the workgroup sums the whole embedding table's gradient in
    // LDS (gw_p = its intervals) and adds it once at the end
    const int32_t wf = v.gw_p;
    double *lemb = reinterpret_cast<double *>(lds_raw);
    for (int32_t t = threadIdx.x; t < 4 * wf; t += blockDim.x) lemb[t] = 0.0;
    __syncthreads();
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double F, Fp, Fpp, t;
        int k;
        bool lin;
        embed_full(a, a.rho[i], F, Fp, Fpp, k, t, lin);
        const double vE = v.vE[a.R > 1 ? a.rep_of[i] : 0];
        const double rd = v.rdot[i];
        for (int p = 0; p < 4; p++) {
            double dF, dFp;
            if (lin) {
                dF = 1.0 + (double)p * t;
                dFp = (double)p * ih;
            } else {
                const double tp = p == 0 ? 1.0 : (p == 1 ? t : (p == 2 ? t * t : t * t * t));
                const double dtp = p == 0 ? 0.0 : (p == 1 ? 1.0 : (p == 2 ? 2.0 * t : 3.0 * t * t));
                dF = tp;
                dFp = dtp * ih;
            }
            if (wf > 0) atomicAdd(&lemb[4 * k + p], vE * dF - rd * dFp);
            else atomicAdd(&gemb[4 * (int64_t)k + p], vE * dF - rd * dFp);
        }
    }
    __syncthreads();
    for (int32_t t = threadIdx.x; t < 4 * wf; t += blockDim.x)
        if (lemb[t] != 0.0) atomicAdd(&gemb[t], lemb[t]);
}

} // namespace

// The staged-cotangent variants need 24 (LJ, pass A) or 40 (pass B) more bytes of
// LDS per candidate; they run when that stage fits one workgroup's LDS (with
// room for the kernel's static LDS) and v.stage_u allows it.
// workgroups of `threads` that one CU holds with `lds` bytes each
inline int per_cu(const void *kernel, int threads, size_t lds)
{
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, lds) != hipSuccess) return 0;
    return occ;
}

void launch_lj_vjp(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max)
{
    const size_t lds_u = stage_bytes(a.f.cap, 3, false, a.f.bd.stride);
    const size_t lds_g = stage_bytes(a.f.cap, 0, true, a.f.bd.stride);
    if (a.stage_u && lds_u + 256 <= (size_t)lds_max) allow_lds(k_lj_vjp<true>, lds_u);
    if (a.stage_u && lds_u + 256 <= (size_t)lds_max &&
        per_cu(reinterpret_cast<const void *>(k_lj_vjp<true>), threads, lds_u) >=
            per_cu(reinterpret_cast<const void *>(k_lj_vjp<false>), threads, lds_g)) {
        allow_lds(k_lj_vjp<true>, lds_u);
        const int used = resident_grid(k_lj_vjp<true>, grid, threads, lds_u);
        hipLaunchKernelGGL(k_lj_vjp<true>, dim3(used), dim3(threads), lds_u, s, a);
        if (a.gout != nullptr)
            launch_sum_partials(s, a.gpart, used, threads, SumOut{{a.gout, a.gout + 1, nullptr, nullptr}, {1.0, 1.0, 0.0, 0.0}});
        return;
    }
    const size_t lds = stage_bytes(a.f.cap, 0, true, a.f.bd.stride);
    allow_lds(k_lj_vjp<false>, lds);
    const int used = resident_grid(k_lj_vjp<false>, grid, threads, lds);
    hipLaunchKernelGGL(k_lj_vjp<false>, dim3(used), dim3(threads), lds, s, a);
    if (a.gout != nullptr)
        launch_sum_partials(s, a.gpart, used, threads, SumOut{{a.gout, a.gout + 1, nullptr, nullptr}, {1.0, 1.0, 0.0, 0.0}});
}

void launch_eam_vjp_a(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max)
{
    const size_t lds_u = stage_bytes(a.f.cap, 3, false, a.f.bd.stride);
    const size_t lds_g = stage_bytes(a.f.cap, 0, true, a.f.bd.stride);
    if (a.stage_u && lds_u + 256 <= (size_t)lds_max) allow_lds(k_eam_vjp_a<true>, lds_u);
    if (a.stage_u && lds_u + 256 <= (size_t)lds_max &&
        per_cu(reinterpret_cast<const void *>(k_eam_vjp_a<true>), threads, lds_u) >=
            per_cu(reinterpret_cast<const void *>(k_eam_vjp_a<false>), threads, lds_g)) {
        allow_lds(k_eam_vjp_a<true>, lds_u);
        hipLaunchKernelGGL(k_eam_vjp_a<true>, dim3(resident_grid(k_eam_vjp_a<true>, grid, threads, lds_u)),
                           dim3(threads), lds_u, s, a);
        return;
    }
    const size_t lds = stage_bytes(a.f.cap, 0, true, a.f.bd.stride);
    allow_lds(k_eam_vjp_a<false>, lds);
    hipLaunchKernelGGL(k_eam_vjp_a<false>, dim3(resident_grid(k_eam_vjp_a<false>, grid, threads, lds)),
                       dim3(threads), lds, s, a);
}

// The parameter-gradient sums in LDS take what the workgroups that fit on a CU
// leave of its LDS (lds_max, the LDS of one CU; the kernel's registers allow one
// 512-thread workgroup per CU): as many trailing intervals of each pair table
// as fit, none when the stage alone fills it.  Smaller workgroups would fit
// several per CU; then the LDS request may leave fewer of them resident.
template <bool STAGE_U>
void launch_eam_vjp_b_t(hipStream_t s, int grid, int threads, const VjpArgs &a0, int32_t lds_max, int32_t limit)
{
    auto kernel = k_eam_vjp_b<STAGE_U>;
    VjpArgs a = a0;
    const size_t stage = (stage_bytes(a.f.cap, STAGE_U ? 5 : 0, true, a.f.bd.stride) + 15) & ~(size_t)15;
    size_t lds = stage;
    a.gw_p = a.gw_r = 0;
    a.gw_off = (int32_t)stage;
    if (a.gtab != nullptr) {
        allow_lds(kernel, stage);
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, stage) != hipSuccess || occ < 1) occ = 1;
        // fewer workgroups per CU when that is what it takes to hold the upper
        // half of the larger pair table (global atomics on the hot intervals
        // cost far more than the lost occupancy); 256 bytes stay free for the
        // kernel's static LDS; 32 bytes per interval and table
        const int64_t want = (std::max(a.f.nk[0], a.f.nk[1]) - 1) / 2;
        int64_t w = 0;
        for (; occ >= 1; occ--) {
            const int64_t room = (int64_t)lds_max / occ - 256 - (int64_t)stage;
            w = room > 0 ? room / 64 : 0;
            if (w >= want) break;
        }
        if (limit >= 0) w = std::min<int64_t>(w, limit);
        a.gw_p = (int32_t)std::min<int64_t>(w, a.f.nk[0] - 1);
        a.gw_r = (int32_t)std::min<int64_t>(w, a.f.nk[1] - 1);
        lds = stage + 32 * (size_t)(a.gw_p + a.gw_r);
    }
    allow_lds(kernel, lds);
    hipLaunchKernelGGL(kernel, dim3(resident_grid(kernel, grid, threads, lds)), dim3(threads), lds, s, a);
}

// The staged variant only where its larger stage still leaves the parameter
// sums as many table intervals in LDS as the gathering one gets (or half the
// larger table): losing them to global atomics costs far more than the
// gathers it saves.
void launch_eam_vjp_b(hipStream_t s, int grid, int threads, const VjpArgs &a, int32_t lds_max, int32_t limit)
{
    auto window = [&](int nextra) {
        const int64_t stage = (int64_t)((stage_bytes(a.f.cap, nextra, true, a.f.bd.stride) + 15) & ~(size_t)15);
        const int64_t room = (int64_t)lds_max - 256 - stage;
        return room > 0 ? room / 64 : (int64_t)-1;
    };
    const int64_t want = (std::max(a.f.nk[0], a.f.nk[1]) - 1) / 2;
    const int64_t wu = window(5), wg = window(0);
    const bool fits = a.gtab == nullptr ? wu >= 0 : wu >= std::min(want, wg);
    if (a.stage_u && fits)
        launch_eam_vjp_b_t<true>(s, grid, threads, a, lds_max, limit);
    else
        launch_eam_vjp_b_t<false>(s, grid, threads, a, lds_max, limit);
}

// The whole embedding table's gradient goes to LDS when it fits two 256-thread
// workgroups per CU and the limit allows the whole table (then the grid is the
// resident one, each workgroup striding over many atoms); otherwise every term
// is a global atomic.
void launch_eam_vjp_embed(hipStream_t s, int grid, const VjpArgs &a0, int32_t lds_max, int32_t limit)
{
    VjpArgs a = a0;
    a.gw_p = 0;
    const int32_t nk = a.f.nk[2];
    const size_t lds = 32 * (size_t)(nk - 1);
    if ((int64_t)lds <= (int64_t)lds_max / 2 - 256 && (limit < 0 || limit >= nk - 1)) {
        a.gw_p = nk - 1;
        allow_lds(k_eam_vjp_embed, lds);
        hipLaunchKernelGGL(k_eam_vjp_embed, dim3(resident_grid(k_eam_vjp_embed, grid, 256, lds)), dim3(256), lds, s, a);
        return;
    }
    hipLaunchKernelGGL(k_eam_vjp_embed, dim3(grid), dim3(256), 0, s, a);
}
