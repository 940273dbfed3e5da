// cvo_reduce.hip -- per-pair reduction of the pair-pass moments and the
// FP64 ascent step (Problem 1 solved by gradient ascent on SE(3), with the
// lengthscale annealed as in Sec. IV).
//
// From the per-query moments W_j = sum_i w_ij, D_j = sum_i w_ij d_ij and
// S_j = sum_i w_ij d_ij d_ij^T (d = x - z'), held as partial moments per
// piece of the query's candidate list, one O(M) pass gives
//   F        = sum_j W_j                                       (eq. (7))
//   omega    = ell^-2 sum_j z'_j x D_j,  v = ell^-2 sum_j D_j   (gradient)
//   H        = sum_j H_j, the 6x6 matrix with xi^T H xi equal to the second
//              derivative of F(Exp(tau xi) T) at tau = 0 for any xi:
//              with A = S/ell^4 - W I/ell^2 and Z = [z']_x,
//              H_ww = -Z A Z + (D z'^T + z' D^T)/(2 ell^2) - (D.z') I/ell^2
//              H_wv =  Z A - [D]_x /(2 ell^2),   H_vv = A
//   tr S / ell^3 = dF/dell (cutoff held fixed), |P| = sum n_j,
//   r_max = max_j |z'_j|,
// and, for the adaptive lengthscale (Sec. VI), over the targets with W_j > 0:
//   sum log W_j, sum r_j with r_j = tr S_j / W_j (the target's weighted mean
//   squared residual), and their number |Z+|.
// The curvature along a direction d is d^T H d.  Each block reduces a fixed
// slice of the queries in a fixed tree order; a second launch, one workgroup
// per pair, combines the block partials in a fixed order and, in step mode,
// takes the ascent step -- so results are bitwise reproducible.
#include "cvo_launch.hpp"

namespace cvo {

// accumulator slots (R_LOGW .. R_ZP: the lengthscale objective's sums over
// the targets with W_j > 0, reduced only when asked for; 43 .. 47 unused)
enum {
    R_F = 0, R_OM = 1, R_V = 4, R_HWW = 7, R_HWV = 13, R_HVV = 22, R_TRS = 28, R_N = 29, R_RMAX = 30,
    R_ZS = 31, R_ZZ = 34, R_LOGW = 40, R_RSUM = 41, R_ZP = 42, R_END = 48
};

// Solve G d = g for a symmetric positive definite 6x6 G by Cholesky
// (G = L L^T), fully unrolled so everything stays in registers; false if a
// pivot is not positive.  Each pivot is inverted once and the solves
// multiply by the inverse (6 divisions on the serial chain instead of 27).
__device__ bool chol_solve6(const double G[36], const double g[6], double d[6])
{
    double L[6][6], inv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = G[6 * i + j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i][i] = sqrt(s);
                inv[i] = 1.0 / L[i][i];
            } else {
                L[i][j] = s * inv[j];
            }
        }
    }
    double y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double s = g[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[k][i] * d[k];
        d[i] = s * inv[i];
    }
    return true;
}

// xi^T H xi for the reduced 6x6 curvature matrix
__device__ double quad_form(const double *tot, const double xi[6])
{
    const double Hww[3][3] = {{tot[R_HWW + 0], tot[R_HWW + 1], tot[R_HWW + 2]},
                              {tot[R_HWW + 1], tot[R_HWW + 3], tot[R_HWW + 4]},
                              {tot[R_HWW + 2], tot[R_HWW + 4], tot[R_HWW + 5]}};
    const double Hvv[3][3] = {{tot[R_HVV + 0], tot[R_HVV + 1], tot[R_HVV + 2]},
                              {tot[R_HVV + 1], tot[R_HVV + 3], tot[R_HVV + 4]},
                              {tot[R_HVV + 2], tot[R_HVV + 4], tot[R_HVV + 5]}};
    double q = 0.0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            q += xi[r] * Hww[r][k] * xi[k] + 2.0 * xi[r] * tot[R_HWV + 3 * r + k] * xi[3 + k] +
                 xi[3 + r] * Hvv[r][k] * xi[3 + k];
    return q;
}

// SE(3) exponential of xi = (omega, v): R = I + a W + b W^2, V = I + b W + c W^2,
// p = V v with a = sin th / th, b = (1 - cos th) / th^2, c = (th - sin th) / th^3,
// th = |omega|; below th = 1e-2 the three coefficients are their Taylor
// series through th^6, above it b is written 2 sin^2(th/2) / th^2.
__device__ void exp_se3(const double xi[6], double E[12])
{
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double th = sqrt(th2);
    double ca, cb, cc;
    if (th < 1e-2) {
        const double th4 = th2 * th2, th6 = th4 * th2;
        // (reciprocal factorials as constants: multiplications, not divisions)
        ca = 1.0 - th2 * (1.0 / 6.0) + th4 * (1.0 / 120.0) - th6 * (1.0 / 5040.0);
        cb = 0.5 - th2 * (1.0 / 24.0) + th4 * (1.0 / 720.0) - th6 * (1.0 / 40320.0);
        cc = 1.0 / 6.0 - th2 * (1.0 / 120.0) + th4 * (1.0 / 5040.0) - th6 * (1.0 / 362880.0);
    } else {
        const double sh = sin(0.5 * th);
        ca = sin(th) / th;
        cb = 2.0 * sh * sh / th2;
        cc = (th - sin(th)) / (th2 * th);
    }
    const double Wm[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double W2[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) W2[r][k] = Wm[r][0] * Wm[0][k] + Wm[r][1] * Wm[1][k] + Wm[r][2] * Wm[2][k];
    double V[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double I = (r == k) ? 1.0 : 0.0;
            E[4 * r + k] = I + ca * Wm[r][k] + cb * W2[r][k];
            V[r][k] = I + cb * Wm[r][k] + cc * W2[r][k];
        }
#pragma unroll
    for (int r = 0; r < 3; ++r) E[4 * r + 3] = V[r][0] * xi[3] + V[r][1] * xi[4] + V[r][2] * xi[5];
}

__device__ void compose_left(const double E[12], double T[12])
{
    double O[12];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int k = 0; k < 3; ++k) O[4 * r + k] = E[4 * r] * T[k] + E[4 * r + 1] * T[4 + k] + E[4 * r + 2] * T[8 + k];
        O[4 * r + 3] = E[4 * r] * T[3] + E[4 * r + 1] * T[7] + E[4 * r + 2] * T[11] + E[4 * r + 3];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = O[k];
}

__device__ void invert_pose(const double T[12], double Ti[12])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int k = 0; k < 3; ++k) Ti[4 * r + k] = T[4 * k + r];
        Ti[4 * r + 3] = -(T[r] * T[3] + T[4 + r] * T[7] + T[8 + r] * T[11]);
    }
}

// Finish one pair: publish the evaluation, and in step mode take the step.
// Works on register copies of the state and constants (one batch of loads,
// one batch of stores) rather than on global memory field by field.
__device__ __forceinline__ void finalize_local(PairState &st, const AlignConst &ac, const double *tot,
                                               double *trace, long long trace_rows, int mode)
{
    const double ell = st.ell;
    const double il1 = 1.0 / ell;
    const double il2 = il1 * il1;
    double g[6];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        g[k] = tot[R_OM + k] * il2;
        g[3 + k] = tot[R_V + k] * il2;
    }
    const double curv = quad_form(tot, g);
    const double F = tot[R_F];
    const double np = tot[R_N];
    const double ind = (ac.sqrt_nm > 0.0) ? F / ac.sqrt_nm : 0.0;
    st.F = F;
    st.i_theta = ind;
    st.curv = curv;
    st.r_max = tot[R_RMAX];
    st.dF_dell = tot[R_TRS] * il2 * il1;
    st.n_pairs = np;
    {
        // lengthscale objective J = sum log W_j - 3 |Z+| log ell (all zero
        // unless its sums were reduced)
        const double mp = tot[R_ZP];
        st.J = 0.0;
        st.dJ_dell = 0.0;
        st.ell_ml = 0.0;
        if (mp > 0.0) {
            st.J = tot[R_LOGW] - 3.0 * mp * log(ell);
            st.dJ_dell = tot[R_RSUM] * il2 * il1 - 3.0 * mp * il1;
            st.ell_ml = sqrt(tot[R_RSUM] / (3.0 * mp));
        }
        st.zplus = mp;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) st.grad[k] = g[k];
    const double gn2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3] + g[4] * g[4] + g[5] * g[5];
    st.gnorm = sqrt(gn2);
    if (mode == 0) return;

    // ---- ascent step (same decision sequence as the definition it follows)
    if (np == 0.0) { st.status = ST_NO_OVERLAP; st.done = 1; return; }
    if (gn2 == 0.0) { st.status = ST_STATIONARY; st.done = 1; return; }
    // direction: the Riemannian gradient G^-1 g.  Kinetic-energy metric of
    // the moving cloud: G = [[tr(S) I - S + mu I, [c]_x], [[c]_x^T, I]] with
    // c = mean z', S = mean z' z'^T, mu = 1e-6 (tr S + 1e-12).
    double d[6];
    if (ac.metric == 0) {
        const double im = ac.inv_m;
        const double c[3] = {tot[R_ZS] * im, tot[R_ZS + 1] * im, tot[R_ZS + 2] * im};
        const double S[3][3] = {{tot[R_ZZ + 0] * im, tot[R_ZZ + 1] * im, tot[R_ZZ + 2] * im},
                                {tot[R_ZZ + 1] * im, tot[R_ZZ + 3] * im, tot[R_ZZ + 4] * im},
                                {tot[R_ZZ + 2] * im, tot[R_ZZ + 4] * im, tot[R_ZZ + 5] * im}};
        const double trs = S[0][0] + S[1][1] + S[2][2];
        const double mu = 1e-6 * (trs + 1e-12);
        const double Cx[3][3] = {{0.0, -c[2], c[1]}, {c[2], 0.0, -c[0]}, {-c[1], c[0], 0.0}};
        double G[36];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                G[6 * r + k] = (r == k ? trs + mu : 0.0) - S[r][k];
                G[6 * r + 3 + k] = Cx[r][k];
                G[6 * (3 + r) + k] = Cx[k][r];
                G[6 * (3 + r) + 3 + k] = (r == k) ? 1.0 : 0.0;
            }
        if (!chol_solve6(G, g, d)) { st.status = ST_STATIONARY; st.done = 1; return; }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) d[k] = g[k];
    }
    const double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2] + g[3] * d[3] + g[4] * d[4] + g[5] * d[5];
    const double curv_d = quad_form(tot, d);
    const double tauN = (curv_d < 0.0) ? slope / (-curv_d) : INFINITY;
    const double nw = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double nv = sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
    const double tauC = ac.step_lambda * ell / (nw * tot[R_RMAX] + nv);
    const double tau = tauN < tauC ? tauN : tauC;
    double xi[6], E[12];
#pragma unroll
    for (int k = 0; k < 6; ++k) xi[k] = tau * d[k];
    exp_se3(xi, E);
    compose_left(E, st.T);
    invert_pose(st.T, st.Tinv);
    st.tau = tau;
    const long long it = st.it;
    if (trace && it < trace_rows) {
        double *tr = trace + it * kTraceLen;
        tr[0] = (double)it;
        tr[1] = ell;
        tr[2] = F;
        tr[3] = sqrt(gn2);
        tr[4] = tau;
        tr[5] = ind;
        tr[6] = np;
        tr[7] = curv_d;
    }
    st.it = it + 1;
    st.total_pairs += np;
    if (ac.ell_sched) {
        // replay of a given lengthscale sequence: no annealing or convergence decisions
        if (it + 1 >= ac.n_sched) {
            st.status = ST_MAX_ITER;
            st.done = 1;
            return;
        }
        st.ell = ac.ell_sched[it + 1];
    } else if (ac.ell_mode == 1 && !ac.fixed_iters) {
        // adaptive lengthscale: the objective's maximiser at this iteration's
        // (T, ell), clamped to [ell_min, ell_init] and to one factor `decay`
        double next = ell;
        if (st.ell_ml > 0.0) {
            double lo = ac.decay * ell, hi = ell / ac.decay;
            if (lo < ac.ell_min) lo = ac.ell_min;
            if (hi > ac.ell_init) hi = ac.ell_init;
            next = st.ell_ml < lo ? lo : (st.ell_ml > hi ? hi : st.ell_ml);
        }
        const bool still = fabs(next - ell) <= ac.ind_rel_tol * ell;
        st.ell = next;
        if (still && tau * nw < ac.eps_rot && tau * nv < ac.eps_trans) {
            st.status = ST_CONVERGED;
            st.done = 1;
            return;
        }
    } else if (!ac.fixed_iters) {
        const double ip = st.i_prev;
        if (isfinite(ip) && fabs(ind - ip) <= ac.ind_rel_tol * fabs(ind) && ell > ac.ell_min) {
            const double e2 = ac.decay * ell;
            st.ell = e2 > ac.ell_min ? e2 : ac.ell_min;
            st.i_prev = NAN;
        } else {
            st.i_prev = ind;
        }
        if (st.ell == ac.ell_min && tau * nw < ac.eps_rot && tau * nv < ac.eps_trans) {
            st.status = ST_CONVERGED;
            st.done = 1;
            return;
        }
    }
    if (it + 1 >= ac.max_iter) {
        st.status = ST_MAX_ITER;
        st.done = 1;
        return;
    }
    // the views no longer fit: the cutoff shrank past the rebuild ratio, or
    // the pair density fell to a lower class.  Decided from the iterates
    // alone, so where views change does not depend on how many iterations
    // are enqueued between host checks.
    if (isfinite(ac.kappa) && ac.kappa * st.ell < ac.rebuild_ratio * st.rc_build) st.pause = 1;
    // (an adaptive lengthscale may also grow: rebuild once the cutoff has
    // grown by the same ratio)
    if (isfinite(ac.kappa) && ac.rebuild_ratio < 1.0 && ac.kappa * st.ell * ac.rebuild_ratio > st.rc_build)
        st.pause = 1;
    if (ac.adaptive && st.cls_built >= 0 && density_class(np * ac.inv_m, ac.cls_t) < st.cls_built) st.pause = 1;
}

static_assert(kRedThreads == 256 && R_END == 48 && R_END <= kRedVals, "reduction layout");

// ONE: every thread has at most one query (nblk * kRedThreads covers the
// largest cloud), so there is no loop over queries around the 48 sums.
template <bool ONE>
__global__ __launch_bounds__(kRedThreads) void reduce_kernel(const ReduceArgs a)
{
    const int b = blockIdx.y;
    const PairState *st = a.state + b;
    // the skip flags, the pose and the cloud range are loaded together (one
    // round trip) before the skip test
    const ClusterDesc cd = a.cdesc[b];
    double T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = st->T[k];
    const double ell = st->ell;
    if (st->done | st->pause) return;
    const double ascale = 1.4426950408889634 / (2.0 * ell * ell);
    const double isc = 1.0 / sqrt(ascale), ia = 1.0 / ascale;
    const double il2 = 1.0 / (ell * ell), il4 = il2 * il2;

    // every accumulator index below is a compile-time constant, so the 48
    // values stay in registers
    double acc[R_END];
#pragma unroll
    for (int k = 0; k < R_END; ++k) acc[k] = 0.0;
    const long long end = (long long)cd.pt_base + cd.n;
    auto add_query = [&](long long j) {
        const float4 zq = a.qpts[j];
        const int4 qm = a.map.qmap[j];  // (t, cluster size, pieces, first slot)
        const double z[3] = {T[0] * zq.x + T[1] * zq.y + T[2] * zq.z + T[3],
                             T[4] * zq.x + T[5] * zq.y + T[6] * zq.z + T[7],
                             T[8] * zq.x + T[9] * zq.y + T[10] * zq.z + T[11]};
        acc[R_RMAX] = fmax(acc[R_RMAX], sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]));
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[R_ZS + k] += z[k];
        acc[R_ZZ + 0] += z[0] * z[0];
        acc[R_ZZ + 1] += z[0] * z[1];
        acc[R_ZZ + 2] += z[0] * z[2];
        acc[R_ZZ + 3] += z[1] * z[1];
        acc[R_ZZ + 4] += z[1] * z[2];
        acc[R_ZZ + 5] += z[2] * z[2];
        // the query's partial moments of its cluster's pieces, in piece
        // order: piece k's is at slot first + k n.  One piece per loop trip:
        // the other queries' threads keep the memory system busy, and
        // unrolling the loop with predicated loads (2, 4, ... pieces in
        // flight) was slower at every density
        int nj = 0;
        double Wt = 0.0, D0 = 0.0, D1 = 0.0, D2 = 0.0;
        double S0 = 0.0, S1 = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, S5 = 0.0;
        for (int k = 0; k < qm.z; ++k) {
            const long long o = (long long)qm.w + (long long)k * qm.y;
            nj += a.cnt[o];
            Wt += a.W[o];
            D0 += a.D[3 * o + 0];
            D1 += a.D[3 * o + 1];
            D2 += a.D[3 * o + 2];
            S0 += (double)a.S[6 * o + 0];
            S1 += (double)a.S[6 * o + 1];
            S2 += (double)a.S[6 * o + 2];
            S3 += (double)a.S[6 * o + 3];
            S4 += (double)a.S[6 * o + 4];
            S5 += (double)a.S[6 * o + 5];
        }
        if (nj == 0) return;
        const double Dt[3] = {D0 * isc, D1 * isc, D2 * isc};
        const double S6[6] = {S0 * ia, S1 * ia, S2 * ia, S3 * ia, S4 * ia, S5 * ia};
        acc[R_F] += Wt;
        acc[R_OM + 0] += z[1] * Dt[2] - z[2] * Dt[1];
        acc[R_OM + 1] += z[2] * Dt[0] - z[0] * Dt[2];
        acc[R_OM + 2] += z[0] * Dt[1] - z[1] * Dt[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[R_V + k] += Dt[k];
        const double trs = S6[0] + S6[3] + S6[5];
        acc[R_TRS] += trs;
        acc[R_N] += (double)nj;
        if (a.ellobj && Wt > 0.0) {
            acc[R_LOGW] += log(Wt);
            acc[R_RSUM] += trs / Wt;
            acc[R_ZP] += 1.0;
        }
        // A = S/ell^4 - W I/ell^2
        const double A[3][3] = {{S6[0] * il4 - Wt * il2, S6[1] * il4, S6[2] * il4},
                                {S6[1] * il4, S6[3] * il4 - Wt * il2, S6[4] * il4},
                                {S6[2] * il4, S6[4] * il4, S6[5] * il4 - Wt * il2}};
        const double Zm[3][3] = {{0.0, -z[2], z[1]}, {z[2], 0.0, -z[0]}, {-z[1], z[0], 0.0}};
        double ZA[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) ZA[r][k] = Zm[r][0] * A[0][k] + Zm[r][1] * A[1][k] + Zm[r][2] * A[2][k];
        const double dz = Dt[0] * z[0] + Dt[1] * z[1] + Dt[2] * z[2];
        // upper triangle (r, k) of the symmetric 3x3 blocks, slot q
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const int r = (q < 3) ? 0 : (q < 5 ? 1 : 2);
            const int k = (q < 3) ? q : (q < 5 ? q - 2 : 2);
            const double zaz = ZA[r][0] * Zm[0][k] + ZA[r][1] * Zm[1][k] + ZA[r][2] * Zm[2][k];
            const double m3 = 0.5 * (Dt[r] * z[k] + z[r] * Dt[k]) - (r == k ? dz : 0.0);
            acc[R_HWW + q] += -zaz + m3 * il2;
            acc[R_HVV + q] += A[r][k];
        }
        const double Dx[3][3] = {{0.0, -Dt[2], Dt[1]}, {Dt[2], 0.0, -Dt[0]}, {-Dt[1], Dt[0], 0.0}};
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int k = 0; k < 3; ++k) acc[R_HWV + 3 * r + k] += ZA[r][k] - 0.5 * Dx[r][k] * il2;
    };
    const long long j0 = (long long)cd.pt_base + (long long)blockIdx.x * kRedThreads + threadIdx.x;
    if (ONE) {
        if (j0 < end) add_query(j0);
    } else {
        for (long long j = j0; j < end; j += (long long)a.nblk * kRedThreads) add_query(j);
    }


    // block reduction, 24 values at a time through LDS: every thread stores
    // its 24 values; thread (value kv = t / 8, stripe s = t % 8), t < 192,
    // adds the entries s, s + 8, ... of its value, and an 8-lane shuffle tree
    // finishes.  Fixed order throughout.
    constexpr int kChunk = 24, kStripes = 8;
    __shared__ double red[kChunk][kRedThreads];
    const int tid = threadIdx.x;
    double *part = a.partials + (long long)b * a.nblk * kRedVals + blockIdx.x;  // value-major
    {
        const int kv = tid / kStripes, sl = tid % kStripes;
#pragma unroll
        for (int c = 0; c < R_END / kChunk; ++c) {
#pragma unroll
            for (int k = 0; k < kChunk; ++k) red[k][tid] = acc[kChunk * c + k];
            __syncthreads();
            if (kv < kChunk) {
                const bool mx = (kChunk * c + kv) == R_RMAX;
                double v = red[kv][sl];
#pragma unroll
                for (int m = 1; m < kRedThreads / kStripes; ++m) {
                    const double o = red[kv][sl + kStripes * m];
                    v = mx ? fmax(v, o) : v + o;
                }
#pragma unroll
                for (int off = kStripes / 2; off > 0; off >>= 1) {
                    const double o = __shfl_xor(v, off);
                    v = mx ? fmax(v, o) : v + o;
                }
                if (sl == 0) part[(long long)(kChunk * c + kv) * a.nblk] = v;
            }
            __syncthreads();
        }
    }
}

// Second stage, one workgroup per pair: thread (kv = t / 32, stripe sl =
// t % 32) adds blocks sl, sl + 32, ... of the values kv + 8 c (value-major
// partials: a wave's loads are two runs of 32 consecutive doubles), four
// stripes' loads in flight at once; a 32-lane shuffle tree finishes, and one thread
// finishes the pair.  Fixed order throughout.  A separate launch rather than
// a last-block ticket: the kernel boundary makes the partials visible to
// every XCD without a device-scope fence in each block of the first stage.
__global__ __launch_bounds__(kRedThreads) void reduce_finish_kernel(const ReduceArgs a)
{
    const int b = blockIdx.x;
    PairState *st = a.state + b;
    __shared__ double tot[R_END];
    const int tid = threadIdx.x;
    // thread 0 holds the pair's state and constants in registers from the
    // start, so their loads overlap those of the partials; a skipped pair's
    // partials are read but not used
    PairState s;
    AlignConst ac;
    if (tid == 0) {
        s = *st;
        ac = a.ac[b];
    }
    const int kv = tid >> 5, sl = tid & 31;
    const double *pb = a.partials + (long long)b * a.nblk * kRedVals;
    double v[R_END / 8];
#pragma unroll
    for (int c = 0; c < R_END / 8; ++c) v[c] = 0.0;
    for (int q0 = sl; q0 < a.nblk; q0 += 4 * 32) {
        double p[4][R_END / 8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = q0 + 32 * u;
#pragma unroll
            for (int c = 0; c < R_END / 8; ++c) p[u][c] = (q < a.nblk) ? pb[(long long)(8 * c + kv) * a.nblk + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < R_END / 8; ++c)
                v[c] = ((8 * c + kv) == R_RMAX) ? fmax(v[c], p[u][c]) : v[c] + p[u][c];
    }
#pragma unroll
    for (int c = 0; c < R_END / 8; ++c) {
        const bool mx = (8 * c + kv) == R_RMAX;
        double x = v[c];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
            const double o = __shfl_xor(x, off);
            x = mx ? fmax(x, o) : x + o;
        }
        if (sl == 0) tot[8 * c + kv] = x;
    }
    __syncthreads();
    if (tid == 0 && !(s.done | s.pause)) {
        finalize_local(s, ac, tot, a.trace ? a.trace + (long long)b * a.trace_rows * kTraceLen : nullptr,
                       a.trace_rows, a.mode);
        *st = s;
    }
}

void launch_reduce(const ReduceArgs &a, int B, hipStream_t s)
{
    if (a.one_query)
        hipLaunchKernelGGL(reduce_kernel<true>, dim3(a.nblk, B), dim3(kRedThreads), 0, s, a);
    else
        hipLaunchKernelGGL(reduce_kernel<false>, dim3(a.nblk, B), dim3(kRedThreads), 0, s, a);
    hipLaunchKernelGGL(reduce_finish_kernel, dim3(B), dim3(kRedThreads), 0, s, a);
}

// ---------------------------------------------------------------- backward
// d(gF F)/d(query point) = gF * R_P^T D / ell^2, with R_P the rotation of
// the pose that mapped queries into the reference frame (T for Z, T^-1 for
// X), and feature gradients scaled back from pre-scaled columns.
__global__ void backward_finish(const BackwardArgs a)
{
    const PairState *st = a.state;
    const double *P = a.pose_is_inverse ? st->Tinv : st->T;
    const double ell = st->ell;
    const double ascale = 1.4426950408889634 / (2.0 * ell * ell);
    const double f = a.gF / (sqrt(ascale) * ell * ell);
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < a.n;
         p += (long long)gridDim.x * blockDim.x) {
        const long long o = a.qperm[p];
        const int4 qm = a.map.qmap[p];  // (t, cluster size, pieces, first slot)
        if (a.dxyz) {
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            for (int k = 0; k < qm.z; ++k) {
                const long long s = (long long)qm.w + (long long)k * qm.y;
                d0 += a.D[3 * s];
                d1 += a.D[3 * s + 1];
                d2 += a.D[3 * s + 2];
            }
            for (int k = 0; k < 3; ++k)
                a.dxyz[3 * o + k] = (float)(f * (P[k] * d0 + P[4 + k] * d1 + P[8 + k] * d2));
        }
        if (a.dfeat) {
            // folded LIN blocks: the gradient of a tensor-product column c
            // reaches u_b[digit_b(c)] times the other blocks' factors of c
            double gl[64];
            if (a.lay.nlin > 0)
                for (int k = 0; k < 64; ++k) gl[k] = 0.0;
            const float *f = a.lay.nlin > 0 ? a.src_feat + o * a.lay.src_dim : nullptr;
            for (int k = 0; k < a.lay.d4; ++k) {
                const int col = a.lay.col[k];
                if (col == -1) continue;
                double gk = 0.0;
                for (int i = 0; i < qm.z; ++i)
                    gk += a.G[((long long)qm.w + (long long)i * qm.y) * a.lay.d4 + k];
                if (col >= 0) {
                    a.dfeat[o * a.lay.src_dim + col] = (float)(a.gF * gk * a.lay.gscale[k]);
                } else {
                    int dig[8];
                    int cc = k - a.lay.sed;
                    for (int b = a.lay.nlin - 1; b >= 0; --b) {
                        dig[b] = cc % a.lay.lin_dim[b];
                        cc /= a.lay.lin_dim[b];
                    }
                    for (int b = 0; b < a.lay.nlin; ++b) {
                        double other = 1.0;
                        for (int b2 = 0; b2 < a.lay.nlin; ++b2)
                            if (b2 != b) other *= (double)f[a.lay.lin_src[b2] + dig[b2]];
                        gl[a.lay.lin_src[b] + dig[b]] += gk * other;
                    }
                }
            }
            if (a.lay.nlin > 0)
                for (int b = 0; b < a.lay.nlin; ++b)
                    for (int j = 0; j < a.lay.lin_dim[b]; ++j) {
                        const int col = a.lay.lin_src[b] + j;
                        a.dfeat[o * a.lay.src_dim + col] = (float)(a.gF * gl[col]);
                    }
        }
    }
}

void launch_backward_finish(const BackwardArgs &a, hipStream_t s)
{
    long long nb = (a.n + 255) / 256;
    if (nb < 1) nb = 1;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(backward_finish, dim3((unsigned)nb), dim3(256), 0, s, a);
}

__global__ __launch_bounds__(256) void sum_doubles(const double *in, long long n, double *out)
{
    double v = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) v += in[i];
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

void launch_sum_doubles(const double *in, long long n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_doubles, dim3(1), dim3(256), 0, s, in, n, out);
}

}  // namespace cvo
