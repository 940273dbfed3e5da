// cvo_reduce.hip -- per-pair reduction of the pair-pass moments and the
// FP64 ascent step (Problem 1 solved by gradient ascent on SE(3), with the
// lengthscale annealed as in Sec. IV).
//
// From the per-query moments W_j = sum_i w_ij, D_j = sum_i w_ij d_ij and
// S_j = sum_i w_ij d_ij d_ij^T (d = x - z'), one O(M) pass gives
//   F        = sum_j W_j                                       (eq. (7))
//   omega    = ell^-2 sum_j z'_j x D_j,  v = ell^-2 sum_j D_j   (gradient)
//   H        = sum_j H_j, the 6x6 matrix with xi^T H xi equal to the second
//              derivative of F(Exp(tau xi) T) at tau = 0 for any xi:
//              with A = S/ell^4 - W I/ell^2 and Z = [z']_x,
//              H_ww = -Z A Z + (D z'^T + z' D^T)/(2 ell^2) - (D.z') I/ell^2
//              H_wv =  Z A - [D]_x /(2 ell^2),   H_vv = A
//   tr S / ell^3 = dF/dell (cutoff held fixed), |P| = sum n_j,
//   r_max = max_j |z'_j|.
// The curvature along the gradient is grad^T H grad.  Each block reduces a
// fixed slice of the queries in a fixed tree order; the last block of a pair
// (atomic ticket) combines the block partials in block order and, in step
// mode, takes the ascent step -- so results are bitwise reproducible.
#include "cvo_launch.hpp"

namespace cvo {

// accumulator slots
enum {
    R_F = 0, R_OM = 1, R_V = 4, R_HWW = 7, R_HWV = 13, R_HVV = 22, R_TRS = 28, R_N = 29, R_RMAX = 30,
    R_ZS = 31, R_ZZ = 34, R_END = 40
};

// Solve A x = b for the 6x6 system (Gaussian elimination, partial pivoting).
__device__ bool solve6(const double A_in[36], const double b[6], double x[6])
{
    double A[6][7];
    for (int r = 0; r < 6; ++r) {
        for (int c = 0; c < 6; ++c) A[r][c] = A_in[6 * r + c];
        A[r][6] = b[r];
    }
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return false;
        if (piv != c)
            for (int k = 0; k < 7; ++k) {
                const double t = A[c][k];
                A[c][k] = A[piv][k];
                A[piv][k] = t;
            }
        for (int r = c + 1; r < 6; ++r) {
            const double f = A[r][c] / A[c][c];
            for (int k = c; k < 7; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int r = 5; r >= 0; --r) {
        double s = A[r][6];
        for (int k = r + 1; k < 6; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
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
    for (int r = 0; r < 3; ++r)
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
        ca = 1.0 - th2 / 6.0 + th4 / 120.0 - th6 / 5040.0;
        cb = 0.5 - th2 / 24.0 + th4 / 720.0 - th6 / 40320.0;
        cc = 1.0 / 6.0 - th2 / 120.0 + th4 / 5040.0 - th6 / 362880.0;
    } else {
        const double sh = sin(0.5 * th);
        ca = sin(th) / th;
        cb = 2.0 * sh * sh / th2;
        cc = (th - sin(th)) / (th2 * th);
    }
    const double Wm[3][3] = {{0.0, -w2, w1}, {w2, 0.0, -w0}, {-w1, w0, 0.0}};
    double W2[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) W2[r][k] = Wm[r][0] * Wm[0][k] + Wm[r][1] * Wm[1][k] + Wm[r][2] * Wm[2][k];
    double V[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            const double I = (r == k) ? 1.0 : 0.0;
            E[4 * r + k] = I + ca * Wm[r][k] + cb * W2[r][k];
            V[r][k] = I + cb * Wm[r][k] + cc * W2[r][k];
        }
    for (int r = 0; r < 3; ++r) E[4 * r + 3] = V[r][0] * xi[3] + V[r][1] * xi[4] + V[r][2] * xi[5];
}

__device__ void compose_left(const double E[12], double T[12])
{
    double O[12];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) O[4 * r + k] = E[4 * r] * T[k] + E[4 * r + 1] * T[4 + k] + E[4 * r + 2] * T[8 + k];
        O[4 * r + 3] = E[4 * r] * T[3] + E[4 * r + 1] * T[7] + E[4 * r + 2] * T[11] + E[4 * r + 3];
    }
    for (int k = 0; k < 12; ++k) T[k] = O[k];
}

__device__ void invert_pose(const double T[12], double Ti[12])
{
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) Ti[4 * r + k] = T[4 * k + r];
        Ti[4 * r + 3] = -(T[r] * T[3] + T[4 + r] * T[7] + T[8 + r] * T[11]);
    }
}

// Finish one pair: publish the evaluation, and in step mode take the step.
__device__ void finalize_pair(PairState *st, const AlignConst *ac, const double *tot, double *trace,
                              long long trace_rows, int mode)
{
    const double ell = st->ell;
    const double il2 = 1.0 / (ell * ell);
    double g[6];
    for (int k = 0; k < 3; ++k) {
        g[k] = tot[R_OM + k] * il2;
        g[3 + k] = tot[R_V + k] * il2;
    }
    const double curv = quad_form(tot, g);
    const double F = tot[R_F];
    const double np = tot[R_N];
    const double ind = (ac->sqrt_nm > 0.0) ? F / ac->sqrt_nm : 0.0;
    st->F = F;
    st->i_theta = ind;
    st->curv = curv;
    st->r_max = tot[R_RMAX];
    st->dF_dell = tot[R_TRS] / (ell * ell * ell);
    st->n_pairs = np;
    for (int k = 0; k < 6; ++k) st->grad[k] = g[k];
    const double gn2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + g[3] * g[3] + g[4] * g[4] + g[5] * g[5];
    st->gnorm = sqrt(gn2);
    if (mode == 0) return;

    // ---- ascent step (same decision sequence as the definition it follows)
    if (np == 0.0) { st->status = ST_NO_OVERLAP; st->done = 1; return; }
    if (gn2 == 0.0) { st->status = ST_STATIONARY; st->done = 1; return; }
    // direction: the Riemannian gradient G^-1 g.  Kinetic-energy metric of
    // the moving cloud: G = [[tr(S) I - S + mu I, [c]_x], [[c]_x^T, I]] with
    // c = mean z', S = mean z' z'^T, mu = 1e-6 (tr S + 1e-12).
    double d[6];
    if (ac->metric == 0) {
        const double im = ac->inv_m;
        const double c[3] = {tot[R_ZS] * im, tot[R_ZS + 1] * im, tot[R_ZS + 2] * im};
        const double S[3][3] = {{tot[R_ZZ + 0] * im, tot[R_ZZ + 1] * im, tot[R_ZZ + 2] * im},
                                {tot[R_ZZ + 1] * im, tot[R_ZZ + 3] * im, tot[R_ZZ + 4] * im},
                                {tot[R_ZZ + 2] * im, tot[R_ZZ + 4] * im, tot[R_ZZ + 5] * im}};
        const double trs = S[0][0] + S[1][1] + S[2][2];
        const double mu = 1e-6 * (trs + 1e-12);
        const double Cx[3][3] = {{0.0, -c[2], c[1]}, {c[2], 0.0, -c[0]}, {-c[1], c[0], 0.0}};
        double G[36];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) {
                G[6 * r + k] = (r == k ? trs + mu : 0.0) - S[r][k];
                G[6 * r + 3 + k] = Cx[r][k];
                G[6 * (3 + r) + k] = Cx[k][r];
                G[6 * (3 + r) + 3 + k] = (r == k) ? 1.0 : 0.0;
            }
        if (!solve6(G, g, d)) { st->status = ST_STATIONARY; st->done = 1; return; }
    } else {
        for (int k = 0; k < 6; ++k) d[k] = g[k];
    }
    const double slope = g[0] * d[0] + g[1] * d[1] + g[2] * d[2] + g[3] * d[3] + g[4] * d[4] + g[5] * d[5];
    const double curv_d = quad_form(tot, d);
    const double tauN = (curv_d < 0.0) ? slope / (-curv_d) : INFINITY;
    const double nw = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double nv = sqrt(d[3] * d[3] + d[4] * d[4] + d[5] * d[5]);
    const double tauC = ac->step_lambda * ell / (nw * tot[R_RMAX] + nv);
    const double tau = tauN < tauC ? tauN : tauC;
    double xi[6], E[12];
    for (int k = 0; k < 6; ++k) xi[k] = tau * d[k];
    exp_se3(xi, E);
    compose_left(E, st->T);
    invert_pose(st->T, st->Tinv);
    st->tau = tau;
    const long long it = st->it;
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
    st->it = it + 1;
    st->total_pairs += np;
    if (!ac->fixed_iters) {
        const double ip = st->i_prev;
        if (isfinite(ip) && fabs(ind - ip) <= ac->ind_rel_tol * fabs(ind) && ell > ac->ell_min) {
            const double e2 = ac->decay * ell;
            st->ell = e2 > ac->ell_min ? e2 : ac->ell_min;
            st->i_prev = NAN;
        } else {
            st->i_prev = ind;
        }
        if (st->ell == ac->ell_min && tau * nw < ac->eps_rot && tau * nv < ac->eps_trans) {
            st->status = ST_CONVERGED;
            st->done = 1;
            return;
        }
    }
    if (it + 1 >= ac->max_iter) {
        st->status = ST_MAX_ITER;
        st->done = 1;
    }
}

__global__ __launch_bounds__(kRedThreads) void reduce_kernel(const ReduceArgs a)
{
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0 && a.ticket) *a.ticket = 0u;
    const int b = blockIdx.y;
    PairState *st = a.state + b;
    if (st->done) return;
    const ClusterDesc cd = a.cdesc[b];
    double T[12];
    for (int k = 0; k < 12; ++k) T[k] = st->T[k];
    const double ell = st->ell;
    const double ascale = 1.4426950408889634 / (2.0 * ell * ell);
    const double isc = 1.0 / sqrt(ascale), ia = 1.0 / ascale;
    const double il2 = 1.0 / (ell * ell), il4 = il2 * il2;

    double acc[kRedVals];
    for (int k = 0; k < kRedVals; ++k) acc[k] = 0.0;
    const long long end = (long long)cd.pt_base + cd.n;
    for (long long j = (long long)cd.pt_base + (long long)blockIdx.x * kRedThreads + threadIdx.x; j < end;
         j += (long long)a.nblk * kRedThreads) {
        const float4 zq = a.qpts[j];
        const double z[3] = {T[0] * zq.x + T[1] * zq.y + T[2] * zq.z + T[3],
                             T[4] * zq.x + T[5] * zq.y + T[6] * zq.z + T[7],
                             T[8] * zq.x + T[9] * zq.y + T[10] * zq.z + T[11]};
        acc[R_RMAX] = fmax(acc[R_RMAX], sqrt(z[0] * z[0] + z[1] * z[1] + z[2] * z[2]));
        for (int k = 0; k < 3; ++k) acc[R_ZS + k] += z[k];
        acc[R_ZZ + 0] += z[0] * z[0];
        acc[R_ZZ + 1] += z[0] * z[1];
        acc[R_ZZ + 2] += z[0] * z[2];
        acc[R_ZZ + 3] += z[1] * z[1];
        acc[R_ZZ + 4] += z[1] * z[2];
        acc[R_ZZ + 5] += z[2] * z[2];
        // combine this query's partial moments over its cluster's pieces
        const int c = a.map.tclus[j];
        const int t = (int)(j - a.map.clus[c].x);
        const int2 cp = a.map.cpieces[c];
        int nj = 0;
        double Wt = 0.0, Dsum[3] = {0.0, 0.0, 0.0}, Ssum[6] = {0, 0, 0, 0, 0, 0};
        for (int i = cp.x; i < cp.x + cp.y; ++i) {
            const long long o = (long long)a.map.pieces[i].w + t;
            nj += a.cnt[o];
            Wt += a.W[o];
            for (int k = 0; k < 3; ++k) Dsum[k] += a.D[3 * o + k];
            for (int k = 0; k < 6; ++k) Ssum[k] += (double)a.S[6 * o + k];
        }
        if (nj == 0) continue;
        const double Dt[3] = {Dsum[0] * isc, Dsum[1] * isc, Dsum[2] * isc};
        const double S6[6] = {Ssum[0] * ia, Ssum[1] * ia, Ssum[2] * ia, Ssum[3] * ia, Ssum[4] * ia, Ssum[5] * ia};
        acc[R_F] += Wt;
        acc[R_OM + 0] += z[1] * Dt[2] - z[2] * Dt[1];
        acc[R_OM + 1] += z[2] * Dt[0] - z[0] * Dt[2];
        acc[R_OM + 2] += z[0] * Dt[1] - z[1] * Dt[0];
        for (int k = 0; k < 3; ++k) acc[R_V + k] += Dt[k];
        acc[R_TRS] += S6[0] + S6[3] + S6[5];
        acc[R_N] += (double)nj;
        // A = S/ell^4 - W I/ell^2
        const double A[3][3] = {{S6[0] * il4 - Wt * il2, S6[1] * il4, S6[2] * il4},
                                {S6[1] * il4, S6[3] * il4 - Wt * il2, S6[4] * il4},
                                {S6[2] * il4, S6[4] * il4, S6[5] * il4 - Wt * il2}};
        const double Zm[3][3] = {{0.0, -z[2], z[1]}, {z[2], 0.0, -z[0]}, {-z[1], z[0], 0.0}};
        double ZA[3][3];
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) ZA[r][k] = Zm[r][0] * A[0][k] + Zm[r][1] * A[1][k] + Zm[r][2] * A[2][k];
        const double dz = Dt[0] * z[0] + Dt[1] * z[1] + Dt[2] * z[2];
        const int ur[6] = {0, 0, 0, 1, 1, 2}, uc[6] = {0, 1, 2, 1, 2, 2};
        for (int q = 0; q < 6; ++q) {
            const int r = ur[q], k = uc[q];
            const double zaz = ZA[r][0] * Zm[0][k] + ZA[r][1] * Zm[1][k] + ZA[r][2] * Zm[2][k];
            const double m3 = 0.5 * (Dt[r] * z[k] + z[r] * Dt[k]) - (r == k ? dz : 0.0);
            acc[R_HWW + q] += -zaz + m3 * il2;
            acc[R_HVV + q] += A[r][k];
        }
        const double Dx[3][3] = {{0.0, -Dt[2], Dt[1]}, {Dt[2], 0.0, -Dt[0]}, {-Dt[1], Dt[0], 0.0}};
        for (int r = 0; r < 3; ++r)
            for (int k = 0; k < 3; ++k) acc[R_HWV + 3 * r + k] += ZA[r][k] - 0.5 * Dx[r][k] * il2;
    }

    // block reduction: lanes (xor tree), then waves in order
    for (int k = 0; k < R_END; ++k) {
        double v = acc[k];
        for (int off = kWave / 2; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = (k == R_RMAX) ? fmax(v, o) : v + o;
        }
        acc[k] = v;
    }
    __shared__ double red[kRedThreads / kWave][kRedVals];
    __shared__ int s_last;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    if (lane == 0)
        for (int k = 0; k < R_END; ++k) red[wv][k] = acc[k];
    __syncthreads();
    double *part = a.partials + ((long long)b * a.nblk + blockIdx.x) * kRedVals;
    if (threadIdx.x < R_END) {
        double v = red[0][threadIdx.x];
        for (int w = 1; w < kRedThreads / kWave; ++w)
            v = (threadIdx.x == R_RMAX) ? fmax(v, red[w][threadIdx.x]) : v + red[w][threadIdx.x];
        part[threadIdx.x] = v;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int ticket = atomicAdd(&a.counters[b], 1u);
        s_last = (ticket == (unsigned int)(a.nblk - 1));
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    // gather every block partial of this pair at once (one round of loads),
    // then combine each value over the blocks in block order
    __shared__ double tot[kRedVals];
    __shared__ double parts[64 * kRedVals];
    const double *pb = a.partials + (long long)b * a.nblk * kRedVals;
    for (int k = threadIdx.x; k < a.nblk * kRedVals; k += kRedThreads) parts[k] = pb[k];
    __syncthreads();
    if (threadIdx.x < R_END) {
        double v = 0.0;
        for (int k = 0; k < a.nblk; ++k) {
            const double p = parts[k * kRedVals + threadIdx.x];
            v = (threadIdx.x == R_RMAX) ? fmax(v, p) : v + p;
        }
        tot[threadIdx.x] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.counters[b] = 0u;
        finalize_pair(st, a.ac + b, tot, a.trace ? a.trace + (long long)b * a.trace_rows * kTraceLen : nullptr,
                      a.trace_rows, a.mode);
    }
}

void launch_reduce(const ReduceArgs &a, int B, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_kernel, dim3(a.nblk, B), dim3(kRedThreads), 0, s, a);
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
        const int c = a.map.tclus[p];
        const int t = (int)(p - a.map.clus[c].x);
        const int2 cp = a.map.cpieces[c];
        if (a.dxyz) {
            double d0 = 0.0, d1 = 0.0, d2 = 0.0;
            for (int i = cp.x; i < cp.x + cp.y; ++i) {
                const long long s = (long long)a.map.pieces[i].w + t;
                d0 += a.D[3 * s];
                d1 += a.D[3 * s + 1];
                d2 += a.D[3 * s + 2];
            }
            for (int k = 0; k < 3; ++k)
                a.dxyz[3 * o + k] = (float)(f * (P[k] * d0 + P[4 + k] * d1 + P[8 + k] * d2));
        }
        if (a.dfeat) {
            for (int k = 0; k < a.lay.d4; ++k) {
                const int col = a.lay.col[k];
                if (col < 0) continue;
                double gk = 0.0;
                for (int i = cp.x; i < cp.x + cp.y; ++i)
                    gk += a.G[((long long)a.map.pieces[i].w + t) * a.lay.d4 + k];
                a.dfeat[o * a.lay.src_dim + col] = (float)(a.gF * gk * a.lay.gscale[k]);
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
