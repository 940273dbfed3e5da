/*
 * cvo_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct FP64 CPU implementation of what the
 * continuous RKHS registration ("CVO") hot path computes.  It exists to check
 * the HIP implementation and is never part of the product path: only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant generator with the HIP path.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 * (no fused multiply-add anywhere: every * and + is a separately rounded
 * IEEE double operation, so the pair predicate below is reproducible).
 *
 * Paper: "A New Framework for Registration of Semantic Point Clouds from
 * Stereo and RGB-D Cameras" (arXiv 2012.03683).
 *
 * What each function follows
 *   canonical_transform  Sec. III (Problem 1): the action of the pose on the
 *                        second cloud, written T z = R z + t (T plays h^-1).
 *   feature_kernel       Sec. III-A eq. (2) geometric kernel; eq. (5) SE
 *                        appearance kernel; Sec. III-B eq. (6)-(7) product of
 *                        per-block kernels (c_ij); eq. (8) no blocks => c = 1.
 *   oracle_evaluate      eq. (7) double sum F, restricted to the pair set
 *                        within the cutoff (Sec. III-B notes the sum is
 *                        sparse); its gradient on se(3) and the curvature
 *                        along the gradient, with c_ij held constant
 *                        (Sec. III-B, the sentence after eq. (7)).  The paper
 *                        gives no gradient formula: the left-perturbation
 *                        derivative written below is derived from eq. (2).
 *   oracle_exp_se3       the SE(3) exponential used by the Lie-group ascent
 *                        (Sec. I cites gradient ascent on Riemannian
 *                        manifolds); closed form, textbook.
 *   oracle_align         Problem 1 solved by gradient ascent, with the
 *                        lengthscale decayed by 2 % whenever the alignment
 *                        indicator stabilises (Sec. IV) and the indicator of
 *                        eq. (10) (Sec. III-C).
 *   oracle_backward      derivatives of eq. (7) with respect to positions,
 *                        features and the lengthscale on the frozen pair set.
 *
 * Readings where the paper is silent (the same readings bind the HIP path):
 *   - pair set P = { (i,j) : s_ij <= (kappa*ell)^2 }, s_ij the squared
 *     distance evaluated in the exact operation order of canonical_distance;
 *     kappa = +inf means all pairs;
 *   - step size: one-dimensional Newton step along the gradient, clamped so
 *     that no point moves by more than lambda*ell;
 *   - "indicator stabilises": |i - i_prev| <= eps_ind * |i| at one lengthscale.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "cvo_oracle.h"

/* ------------------------------------------------------------------ */
/* Pose action (Problem 1): z' = R z + t, each product and sum rounded
 * separately, left to right.                                          */
static void canonical_transform(const double T[12], const float *z, double out[3])
{
    const double z0 = (double)z[0], z1 = (double)z[1], z2 = (double)z[2];
    for (int r = 0; r < 3; ++r) {
        double a = T[4 * r + 0] * z0;
        double b = T[4 * r + 1] * z1;
        double c = T[4 * r + 2] * z2;
        out[r] = ((a + b) + c) + T[4 * r + 3];
    }
}

/* Squared distance between x and z' in the fixed order (dx^2 + dy^2) + dz^2. */
static double canonical_distance(const float *x, const double zt[3], double d[3])
{
    d[0] = (double)x[0] - zt[0];
    d[1] = (double)x[1] - zt[1];
    d[2] = (double)x[2] - zt[2];
    double a = d[0] * d[0];
    double b = d[1] * d[1];
    double c = d[2] * d[2];
    return (a + b) + c;
}

static double cutoff_sq(double ell, double kappa)
{
    if (isinf(kappa)) return INFINITY;
    double r = kappa * ell;
    return r * r;
}

/* Feature kernel c_ij = prod_b k_b(u_b, v_b)  (eq. (6)-(7)).
 * SE block: sigma_b^2 exp(-|u_b - v_b|^2 / (2 ell_b^2))   (eq. (5))
 * LIN block: <u_b, v_b>                                    (eq. (4), (6))
 * cb[] receives the individual block values (needed by the backward). */
static double feature_kernel(const oracle_spec *sp, const float *u, const float *v, double *cb)
{
    double c = 1.0;
    int off = 0;
    for (int b = 0; b < sp->nblocks; ++b) {
        const int n = sp->dim[b];
        double val;
        if (sp->kind[b] == ORACLE_SE) {
            double ss = 0.0;
            for (int k = 0; k < n; ++k) {
                double e = (double)u[off + k] - (double)v[off + k];
                ss += e * e;
            }
            double sb = sp->sigma[b];
            val = sb * sb * exp(-ss / (2.0 * sp->ell[b] * sp->ell[b]));
        } else {
            double dot = 0.0;
            for (int k = 0; k < n; ++k) dot += (double)u[off + k] * (double)v[off + k];
            val = dot;
        }
        if (cb) cb[b] = val;
        c *= val;
        off += n;
    }
    return c;
}

static int spec_dim(const oracle_spec *sp)
{
    int D = 0;
    for (int b = 0; b < sp->nblocks; ++b) D += sp->dim[b];
    return D;
}

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static int nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

int oracle_num_threads(void) { return nthreads(); }

void oracle_transform(const double T[12], const float *z, int64_t M, double *zt)
{
    for (int64_t j = 0; j < M; ++j) canonical_transform(T, z + 3 * j, zt + 3 * j);
}

/* ------------------------------------------------------------------ */
/* F, gradient, curvature along a direction, dF/dell (eq. (7)).
 *
 * With z'_j = T z_j, d_ij = x_i - z'_j, s_ij = |d_ij|^2,
 *   w_ij   = c_ij * sigma^2 * exp(-s_ij / (2 ell^2))
 *   F      = sum_P w_ij
 * Left perturbation T <- Exp(eps xi) T, xi = (omega, v):
 *   dz'/deps = omega x z' + v = q ,  d2z'/deps2 = omega x q
 *   dF/domega = ell^-2 sum w (z' x d) ,  dF/dv = ell^-2 sum w d
 *   d2F/deps2 = sum w [ (d.q)^2/ell^4 - |q|^2/ell^2 + d.(omega x q)/ell^2 ]
 *   dF/dell   = sum w s / ell^3     (cutoff radius held fixed)
 * Pass 1 gives F and the gradient; pass 2 the curvature along a direction
 * (the gradient unless one is given).                                     */
typedef struct {
    double acc[16];
    int64_t np;
    double rmax;
} pass1_out;

static int eval_pass1(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp, double ell,
                      double sigma, double kappa, const double *zt, pass1_out *res)
{
    enum { NACC = 16 };
    const int D = spec_dim(sp);
    const int64_t N = X->n, M = Z->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double il2 = 1.0 / (ell * ell);
    const double s2 = sigma * sigma;
    const int nt = nthreads();
    double *part = (double *)calloc((size_t)nt * NACC, sizeof(double));
    int64_t *pcount = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    if (!part || !pcount) { free(part); free(pcount); return -2; }
#pragma omp parallel
    {
        double *a = part + (size_t)thread_id() * NACC;
        int64_t cnt = 0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const float *xi = X->xyz + 3 * i;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            for (int64_t j = 0; j < M; ++j) {
                double d[3];
                double s = canonical_distance(xi, zt + 3 * j, d);
                if (!(s <= rc2)) continue;
                const float *vj = D ? Z->feat + (size_t)D * j : NULL;
                double c = feature_kernel(sp, ui, vj, NULL);
                double w = c * (s2 * exp(-s / (2.0 * ell * ell)));
                double zxd[3];
                cross3(zt + 3 * j, d, zxd);
                a[0] += w;
                for (int k = 0; k < 3; ++k) a[1 + k] += w * zxd[k] * il2;
                for (int k = 0; k < 3; ++k) a[4 + k] += w * d[k] * il2;
                a[7] += w * s / (ell * ell * ell);
                a[8] += fabs(w);
                for (int k = 0; k < 3; ++k) a[9 + k] += fabs(w) * fabs(zxd[k]) * il2;
                for (int k = 0; k < 3; ++k) a[12 + k] += fabs(w) * fabs(d[k]) * il2;
                cnt += 1;
            }
        }
        pcount[thread_id()] = cnt;
    }
    memset(res, 0, sizeof(*res));
    for (int t = 0; t < nt; ++t) {
        for (int k = 0; k < NACC; ++k) res->acc[k] += part[(size_t)t * NACC + k];
        res->np += pcount[t];
    }
    for (int64_t j = 0; j < M; ++j) {
        double r = sqrt(dot3(zt + 3 * j, zt + 3 * j));
        if (r > res->rmax) res->rmax = r;
    }
    free(part);
    free(pcount);
    return 0;
}

static double eval_curvature(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp, double ell,
                             double sigma, double kappa, const double *zt, const double xi[6])
{
    const int D = spec_dim(sp);
    const int64_t N = X->n, M = Z->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double il2 = 1.0 / (ell * ell);
    const double s2 = sigma * sigma;
    const double om[3] = {xi[0], xi[1], xi[2]};
    const double vv[3] = {xi[3], xi[4], xi[5]};
    const int nt = nthreads();
    double *cpart = (double *)calloc((size_t)nt, sizeof(double));
#pragma omp parallel
    {
        double a = 0.0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const float *xi_ = X->xyz + 3 * i;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            for (int64_t j = 0; j < M; ++j) {
                double d[3];
                double s = canonical_distance(xi_, zt + 3 * j, d);
                if (!(s <= rc2)) continue;
                const float *vj = D ? Z->feat + (size_t)D * j : NULL;
                double c = feature_kernel(sp, ui, vj, NULL);
                double w = c * (s2 * exp(-s / (2.0 * ell * ell)));
                double q[3], oq[3];
                cross3(om, zt + 3 * j, q);
                for (int k = 0; k < 3; ++k) q[k] += vv[k];
                cross3(om, q, oq);
                double dq = dot3(d, q);
                a += w * (dq * dq * il2 * il2 - dot3(q, q) * il2 + dot3(d, oq) * il2);
            }
        }
        cpart[thread_id()] = a;
    }
    double phi2 = 0.0;
    for (int t = 0; t < nt; ++t) phi2 += cpart[t];
    free(cpart);
    return phi2;
}

int oracle_evaluate(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                    double ell, double sigma, double kappa, const double T[12],
                    double out[ORACLE_EVAL_LEN], int64_t *n_pairs)
{
    return oracle_evaluate_dir(X, Z, sp, ell, sigma, kappa, T, NULL, out, n_pairs);
}

/* As oracle_evaluate, with the curvature taken along `dir` (6 doubles,
 * omega then v) instead of along the gradient when dir is not NULL. */
int oracle_evaluate_dir(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                        double ell, double sigma, double kappa, const double T[12],
                        const double *dir, double out[ORACLE_EVAL_LEN], int64_t *n_pairs)
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int64_t N = X->n, M = Z->n;
    double *zt = (double *)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    if (!zt) return -2;
    oracle_transform(T, Z->xyz, M, zt);
    pass1_out p;
    int rc = eval_pass1(X, Z, sp, ell, sigma, kappa, zt, &p);
    if (rc) { free(zt); return rc; }
    double xi[6];
    for (int k = 0; k < 6; ++k) xi[k] = dir ? dir[k] : p.acc[1 + k];
    const double phi2 = eval_curvature(X, Z, sp, ell, sigma, kappa, zt, xi);

    out[ORACLE_F] = p.acc[0];
    for (int k = 0; k < 6; ++k) out[ORACLE_G + k] = p.acc[1 + k];
    out[ORACLE_PHI2] = phi2;
    out[ORACLE_DELL] = p.acc[7];
    out[ORACLE_ABSF] = p.acc[8];
    for (int k = 0; k < 6; ++k) out[ORACLE_ABSG + k] = p.acc[9 + k];
    out[ORACLE_RMAX] = p.rmax;
    out[ORACLE_ITHETA] = (N > 0 && M > 0) ? p.acc[0] / sqrt((double)N * (double)M) : 0.0;
    *n_pairs = p.np;
    free(zt);
    return 0;
}

/* Per-target sums for a subset of targets j (for sampled checks at sizes
 * where the full double loop is too slow):
 *   W_j = sum_i w_ij, D_j = sum_i w_ij d_ij, S_j = sum_i w_ij d_ij d_ij^T
 *   (upper triangle xx,xy,xz,yy,yz,zz), n_j = #{i : (i,j) in P}.          */
int oracle_target_moments(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                          double ell, double sigma, double kappa, const double T[12],
                          const int64_t *idx, int64_t nidx, double *W, double *Dm, double *S,
                          int64_t *cnt)
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int D = spec_dim(sp);
    const double rc2 = cutoff_sq(ell, kappa);
    const double s2 = sigma * sigma;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nidx; ++q) {
        const int64_t j = idx[q];
        double zt[3];
        canonical_transform(T, Z->xyz + 3 * j, zt);
        const float *vj = D ? Z->feat + (size_t)D * j : NULL;
        double w_ = 0.0, d_[3] = {0, 0, 0}, s_[6] = {0, 0, 0, 0, 0, 0};
        int64_t c_ = 0;
        for (int64_t i = 0; i < X->n; ++i) {
            double d[3];
            double s = canonical_distance(X->xyz + 3 * i, zt, d);
            if (!(s <= rc2)) continue;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            double w = feature_kernel(sp, ui, vj, NULL) * (s2 * exp(-s / (2.0 * ell * ell)));
            w_ += w;
            for (int k = 0; k < 3; ++k) d_[k] += w * d[k];
            s_[0] += w * d[0] * d[0];
            s_[1] += w * d[0] * d[1];
            s_[2] += w * d[0] * d[2];
            s_[3] += w * d[1] * d[1];
            s_[4] += w * d[1] * d[2];
            s_[5] += w * d[2] * d[2];
            c_ += 1;
        }
        W[q] = w_;
        for (int k = 0; k < 3; ++k) Dm[3 * q + k] = d_[k];
        for (int k = 0; k < 6; ++k) S[6 * q + k] = s_[k];
        cnt[q] = c_;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* The lengthscale as an optimisation variable (Sec. VI names Adaptive CVO,
 * which makes the lengthscale part of what is optimised, without a formula).
 * F of eq. (7) grows with ell, so F itself cannot choose it.  Reading: ell
 * maximises the log-likelihood of the moved cloud under the kernel mixture
 * centred on X, the kernel of eq. (2) normalised as a density over R^3:
 *   J(T, ell) = sum_{j in Z+} log W_j(T, ell) - 3 |Z+| log ell,
 *   W_j = sum_{i : (i,j) in P} w_ij,   Z+ = {j : W_j > 0},
 * on the pair set frozen at (T, ell), as for dF/dell.  With
 *   r_j = (sum_i w_ij s_ij) / W_j   (target j's weighted mean squared residual)
 *   dJ/dell = sum_{j in Z+} r_j / ell^3 - 3 |Z+| / ell,
 * which is zero at ell^2 = sum_{j in Z+} r_j / (3 |Z+|) when the r_j are held
 * fixed (the variance update of EM for a Gaussian mixture).
 * zt: the moved targets (3 M doubles).  out as ORACLE_ELLOBJ_LEN.        */
static int ell_objective_zt(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp, double ell,
                            double sigma, double kappa, const double *zt, double out[ORACLE_ELLOBJ_LEN])
{
    const int D = spec_dim(sp);
    const int64_t N = X->n, M = Z->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double s2 = sigma * sigma;
    double *Wj = (double *)calloc((size_t)(M > 0 ? M : 1), sizeof(double));
    double *Ws = (double *)calloc((size_t)(M > 0 ? M : 1), sizeof(double));
    if (!Wj || !Ws) { free(Wj); free(Ws); return -2; }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < M; ++j) {
        const float *vj = D ? Z->feat + (size_t)D * j : NULL;
        double w_ = 0.0, ws_ = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double d[3];
            const double s = canonical_distance(X->xyz + 3 * i, zt + 3 * j, d);
            if (!(s <= rc2)) continue;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            const double w = feature_kernel(sp, ui, vj, NULL) * (s2 * exp(-s / (2.0 * ell * ell)));
            w_ += w;
            ws_ += w * s;
        }
        Wj[j] = w_;
        Ws[j] = ws_;
    }
    double J = 0.0, rsum = 0.0;
    int64_t mp = 0;
    for (int64_t j = 0; j < M; ++j) {
        if (!(Wj[j] > 0.0)) continue;
        J += log(Wj[j]);
        rsum += Ws[j] / Wj[j];
        mp += 1;
    }
    free(Wj);
    free(Ws);
    out[ORACLE_J] = J - 3.0 * (double)mp * log(ell);
    out[ORACLE_DJ] = rsum / (ell * ell * ell) - 3.0 * (double)mp / ell;
    out[ORACLE_ELL_ML] = mp > 0 ? sqrt(rsum / (3.0 * (double)mp)) : 0.0;
    out[ORACLE_ZPLUS] = (double)mp;
    return 0;
}

int oracle_ell_objective(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                         double ell, double sigma, double kappa, const double T[12],
                         double out[ORACLE_ELLOBJ_LEN])
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int64_t M = Z->n;
    double *zt = (double *)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    if (!zt) return -2;
    oracle_transform(T, Z->xyz, M, zt);
    const int rc = ell_objective_zt(X, Z, sp, ell, sigma, kappa, zt, out);
    free(zt);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Metric on se(3) used for the ascent direction: the kinetic energy of the
 * moving cloud as a rigid body with unit masses,
 *   xi^T G xi = (1/M) sum_j |omega x z'_j + v|^2,  G = (1/M) sum_j J_j^T J_j,
 *   J_j = [ -[z'_j]_x  I ],
 * plus mu = 1e-6 (mean |z'|^2 + 1e-12) on the rotation block, which keeps G
 * positive definite for collinear or single-point clouds.  The Riemannian
 * gradient is G^-1 grad.                                                  */
void oracle_metric_tensor(const double T[12], const float *z, int64_t M, double G[36])
{
    for (int k = 0; k < 36; ++k) G[k] = 0.0;
    double r2 = 0.0;
    for (int64_t j = 0; j < M; ++j) {
        double zt[3];
        canonical_transform(T, z + 3 * j, zt);
        double J[3][6];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 6; ++c) J[r][c] = 0.0;
        /* -[z]_x */
        J[0][1] = zt[2];  J[0][2] = -zt[1];
        J[1][0] = -zt[2]; J[1][2] = zt[0];
        J[2][0] = zt[1];  J[2][1] = -zt[0];
        J[0][3] = 1.0; J[1][4] = 1.0; J[2][5] = 1.0;
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 6; ++b) G[6 * a + b] += J[0][a] * J[0][b] + J[1][a] * J[1][b] + J[2][a] * J[2][b];
        r2 += dot3(zt, zt);
    }
    const double inv = M > 0 ? 1.0 / (double)M : 0.0;
    for (int k = 0; k < 36; ++k) G[k] *= inv;
    const double mu = 1e-6 * (r2 * inv + 1e-12);
    for (int a = 0; a < 3; ++a) G[7 * a] += mu;
}

/* Solve G d = g for a symmetric positive definite 6x6 G (Gaussian
 * elimination with partial pivoting).  Returns nonzero if G is singular. */
int oracle_solve6(const double G[36], const double g[6], double d[6])
{
    double A[6][7];
    for (int r = 0; r < 6; ++r) {
        for (int c = 0; c < 6; ++c) A[r][c] = G[6 * r + c];
        A[r][6] = g[r];
    }
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        for (int r = c + 1; r < 6; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c)
            for (int k = 0; k < 7; ++k) { double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
        for (int r = c + 1; r < 6; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 7; ++k) A[r][k] -= f * A[c][k];
        }
    }
    for (int r = 5; r >= 0; --r) {
        double s = A[r][6];
        for (int k = r + 1; k < 6; ++k) s -= A[r][k] * d[k];
        d[r] = s / A[r][r];
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* SE(3) exponential of xi = (omega, v):
 *   R = I + a W + b W^2,  V = I + b W + c W^2,  p = V v
 *   a = sin(th)/th, b = (1-cos th)/th^2, c = (th - sin th)/th^3,
 *   th = |omega|, W = [omega]_x.
 * Below th = 1e-2 the three coefficients are their Taylor series through the
 * th^6 term (truncation below 1e-19); above, b is written 2 sin^2(th/2)/th^2,
 * which avoids the cancellation in 1 - cos th.                           */
void oracle_exp_se3(const double xi[6], double T[12])
{
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double th = sqrt(th2);
    double a, b, c;
    if (th < 1e-2) {
        const double th4 = th2 * th2, th6 = th4 * th2;
        a = 1.0 - th2 / 6.0 + th4 / 120.0 - th6 / 5040.0;
        b = 0.5 - th2 / 24.0 + th4 / 720.0 - th6 / 40320.0;
        c = 1.0 / 6.0 - th2 / 120.0 + th4 / 5040.0 - th6 / 362880.0;
    } else {
        const double sh = sin(0.5 * th);
        a = sin(th) / th;
        b = 2.0 * sh * sh / th2;
        c = (th - sin(th)) / (th2 * th);
    }
    const double W[3][3] = {{0, -w2, w1}, {w2, 0, -w0}, {-w1, w0, 0}};
    double W2[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int m = 0; m < 3; ++m) s += W[r][m] * W[m][k];
            W2[r][k] = s;
        }
    double V[3][3];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            double I = (r == k) ? 1.0 : 0.0;
            T[4 * r + k] = I + a * W[r][k] + b * W2[r][k];
            V[r][k] = I + b * W[r][k] + c * W2[r][k];
        }
    for (int r = 0; r < 3; ++r) T[4 * r + 3] = V[r][0] * xi[3] + V[r][1] * xi[4] + V[r][2] * xi[5];
}

/* A <- B * A for 3x4 rigid transforms (rotation then translation). */
static void compose_left(const double B[12], double A[12])
{
    double O[12];
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k)
            O[4 * r + k] = B[4 * r + 0] * A[0 + k] + B[4 * r + 1] * A[4 + k] + B[4 * r + 2] * A[8 + k];
        O[4 * r + 3] = B[4 * r + 0] * A[3] + B[4 * r + 1] * A[7] + B[4 * r + 2] * A[11] + B[4 * r + 3];
    }
    memcpy(A, O, sizeof(O));
}

/* ------------------------------------------------------------------ */
/* Problem 1 by gradient ascent on SE(3) with lengthscale annealing.
 * Per iteration, at the current (T, ell):
 *   a. evaluate F, the gradient g = (omega, v) and |P|.
 *      |P| = 0 -> NO_OVERLAP; g = 0 -> STATIONARY (no step).
 *      A metric G that cannot be solved also ends as STATIONARY (no step).
 *   b. indicator i = F / sqrt(|X||Z|)                         (eq. (10))
 *   c. ascent direction d = G^-1 g, the Riemannian gradient for the metric G
 *      (kinetic-energy metric of the moving cloud, or the identity), and the
 *      curvature phi'' of F(Exp(tau d) T) at tau = 0;
 *      tau_N = (g.d) / (-phi'') if phi'' < 0, else +inf;
 *      tau_C = lambda * ell / (|d_omega| * r_max + |d_v|), r_max = max_j |z'_j|;
 *      tau = min(tau_N, tau_C)
 *   d. T <- Exp(tau d) T
 *   e. annealing (Sec. IV): when the indicator has stabilised at the current
 *      lengthscale, ell <- max(ell_min, decay * ell) and the reference
 *      indicator is cleared; otherwise it becomes the reference.
 *   f. converged when ell == ell_min and the step moved less than
 *      (eps_rot, eps_trans).
 *   g. stop at max_iter.
 * In fixed-iteration mode e. and f. are skipped.
 * Adaptive mode (ell_mode = ORACLE_ELL_ADAPTIVE) replaces e. and f.:
 *   e'. ell <- ell_ml of oracle_ell_objective at the iteration's (T, ell)
 *       (before the step), kept within [ell_min, ell_init] and within a
 *       factor `decay` of ell (at most one annealing decay per iteration,
 *       down or up); unchanged when Z+ is empty.
 *   f'. converged when the step moved less than (eps_rot, eps_trans) and
 *       ell changed by at most ind_rel_tol * ell.
 * trace (may be NULL): per iteration ORACLE_TRACE_LEN doubles.          */
int oracle_align(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                 const oracle_align_params *ap, const double T_init[12], double T_out[12],
                 double report[ORACLE_REPORT_LEN], double *trace)
{
    double T[12];
    memcpy(T, T_init, sizeof(T));
    double ell = ap->ell_init;
    double i_prev = NAN;
    int64_t it = 0;
    int status = ORACLE_MAX_ITER;
    int64_t np = 0;
    double last_F = 0.0, last_i = 0.0;
    const int64_t M = Z->n;
    if (X->n == 0 || M == 0) {
        memcpy(T_out, T_init, sizeof(double) * 12);
        report[0] = 0;
        report[1] = ell;
        report[2] = 0;
        report[3] = 0;
        report[4] = 0;
        report[5] = ORACLE_NO_OVERLAP;
        return 0;
    }
    double *zt = (double *)malloc(sizeof(double) * 3 * M);
    if (!zt) return -2;
    while (it < ap->max_iter) {
        oracle_transform(T, Z->xyz, M, zt);
        pass1_out p;
        int rc = eval_pass1(X, Z, sp, ell, ap->sigma, ap->kappa, zt, &p);
        if (rc) { free(zt); return rc; }
        np = p.np;
        last_F = p.acc[0];
        last_i = p.acc[0] / sqrt((double)X->n * (double)M);
        if (np == 0) { status = ORACLE_NO_OVERLAP; break; }
        const double *g = p.acc + 1;
        const double gn2 = dot3(g, g) + dot3(g + 3, g + 3);
        if (gn2 == 0.0) { status = ORACLE_STATIONARY; break; }
        const double ind = last_i;
        double d[6];
        if (ap->metric == ORACLE_METRIC_KINETIC) {
            double G[36];
            oracle_metric_tensor(T, Z->xyz, M, G);
            /* no direction solves G d = g: nothing defines an ascent step, so
             * the iterate is taken as stationary (no step is made) */
            if (oracle_solve6(G, g, d)) { status = ORACLE_STATIONARY; break; }
        } else {
            for (int k = 0; k < 6; ++k) d[k] = g[k];
        }
        const double slope = dot3(g, d) + dot3(g + 3, d + 3);
        const double phi2 = eval_curvature(X, Z, sp, ell, ap->sigma, ap->kappa, zt, d);
        double ell_ml = 0.0;
        const int adaptive = ap->ell_mode == ORACLE_ELL_ADAPTIVE && !ap->fixed_iters;
        if (adaptive) {
            double eo[ORACLE_ELLOBJ_LEN];
            rc = ell_objective_zt(X, Z, sp, ell, ap->sigma, ap->kappa, zt, eo);
            if (rc) { free(zt); return rc; }
            ell_ml = eo[ORACLE_ELL_ML];
        }
        const double tauN = (phi2 < 0.0) ? slope / (-phi2) : INFINITY;
        const double nw = sqrt(dot3(d, d)), nv = sqrt(dot3(d + 3, d + 3));
        const double tauC = ap->step_lambda * ell / (nw * p.rmax + nv);
        const double tau = tauN < tauC ? tauN : tauC;
        double xi[6], E[12];
        for (int k = 0; k < 6; ++k) xi[k] = tau * d[k];
        oracle_exp_se3(xi, E);
        compose_left(E, T);
        if (trace) {
            double *tr = trace + (size_t)it * ORACLE_TRACE_LEN;
            tr[0] = (double)it;
            tr[1] = ell;
            tr[2] = p.acc[0];
            tr[3] = sqrt(gn2);
            tr[4] = tau;
            tr[5] = ind;
            tr[6] = (double)np;
            tr[7] = phi2;
        }
        it += 1;
        if (adaptive) {
            double next = ell;
            if (ell_ml > 0.0) {
                double lo = ap->decay * ell, hi = ell / ap->decay;
                if (lo < ap->ell_min) lo = ap->ell_min;
                if (hi > ap->ell_init) hi = ap->ell_init;
                next = ell_ml < lo ? lo : (ell_ml > hi ? hi : ell_ml);
            }
            const int still = fabs(next - ell) <= ap->ind_rel_tol * ell;
            ell = next;
            if (still && tau * nw < ap->eps_rot && tau * nv < ap->eps_trans) {
                status = ORACLE_CONVERGED;
                break;
            }
        } else if (!ap->fixed_iters) {
            if (isfinite(i_prev) && fabs(ind - i_prev) <= ap->ind_rel_tol * fabs(ind) &&
                ell > ap->ell_min) {
                double e2 = ap->decay * ell;
                ell = e2 > ap->ell_min ? e2 : ap->ell_min;
                i_prev = NAN;
            } else {
                i_prev = ind;
            }
            if (ell == ap->ell_min && tau * nw < ap->eps_rot && tau * nv < ap->eps_trans) {
                status = ORACLE_CONVERGED;
                break;
            }
        }
    }
    free(zt);
    memcpy(T_out, T, sizeof(T));
    report[0] = (double)it;
    report[1] = ell;
    report[2] = last_F;
    report[3] = last_i;
    report[4] = (double)np;
    report[5] = (double)status;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Derivatives of F (eq. (7)) on the pair set P frozen at (T, ell):
 *   dF/dx_i = -ell^-2 sum_j w d_ij          dF/dz_j = R^T ell^-2 sum_i w d_ij
 *   SE block b:  dF/du_i = -sum_j w (u_i - v_j) / ell_b^2,  dF/dv_j = -dF/du-term
 *   LIN block b: dF/du_i = sum_j k_ij (prod_{b' != b} c_b') v_j   (and sym.)
 *   dF/dell = sum w s / ell^3
 * Any output pointer may be NULL. */
int oracle_backward(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                    double ell, double sigma, double kappa, const double T[12],
                    double *dx, double *dz, double *du, double *dv, double *dell)
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int D = spec_dim(sp);
    const int64_t N = X->n, M = Z->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double il2 = 1.0 / (ell * ell);
    const double s2 = sigma * sigma;
    double *zt = (double *)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    if (!zt) return -2;
    oracle_transform(T, Z->xyz, M, zt);
    /* target-side raw sums, accumulated per thread then combined in order */
    const int nt = nthreads();
    double *dzr = (double *)calloc((size_t)nt * 3 * (M > 0 ? M : 1), sizeof(double));
    double *dvr = D ? (double *)calloc((size_t)nt * D * (M > 0 ? M : 1), sizeof(double)) : NULL;
    double *dlp = (double *)calloc((size_t)nt, sizeof(double));

#pragma omp parallel
    {
        const int t = thread_id();
        double *myz = dzr + (size_t)t * 3 * M;
        double *myv = D ? dvr + (size_t)t * D * M : NULL;
        double cb[ORACLE_MAX_BLOCKS];
        double dl = 0.0;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < N; ++i) {
            const float *xi = X->xyz + 3 * i;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            double gx[3] = {0, 0, 0};
            if (dx) for (int k = 0; k < 3; ++k) dx[3 * i + k] = 0.0;
            if (du) for (int k = 0; k < D; ++k) du[(size_t)D * i + k] = 0.0;
            for (int64_t j = 0; j < M; ++j) {
                double d[3];
                double s = canonical_distance(xi, zt + 3 * j, d);
                if (!(s <= rc2)) continue;
                const float *vj = D ? Z->feat + (size_t)D * j : NULL;
                double c = feature_kernel(sp, ui, vj, cb);
                double kg = s2 * exp(-s / (2.0 * ell * ell));
                double w = c * kg;
                for (int k = 0; k < 3; ++k) {
                    gx[k] += w * d[k];
                    myz[3 * j + k] += w * d[k];
                }
                dl += w * s / (ell * ell * ell);
                int off = 0;
                for (int b = 0; b < sp->nblocks; ++b) {
                    const int n = sp->dim[b];
                    if (sp->kind[b] == ORACLE_SE) {
                        double ib = 1.0 / (sp->ell[b] * sp->ell[b]);
                        for (int k = 0; k < n; ++k) {
                            double e = (double)ui[off + k] - (double)vj[off + k];
                            if (du) du[(size_t)D * i + off + k] += -w * e * ib;
                            myv[(size_t)D * j + off + k] += w * e * ib;
                        }
                    } else {
                        double other = kg;
                        for (int b2 = 0; b2 < sp->nblocks; ++b2)
                            if (b2 != b) other *= cb[b2];
                        for (int k = 0; k < n; ++k) {
                            if (du) du[(size_t)D * i + off + k] += other * (double)vj[off + k];
                            myv[(size_t)D * j + off + k] += other * (double)ui[off + k];
                        }
                    }
                    off += n;
                }
            }
            if (dx) for (int k = 0; k < 3; ++k) dx[3 * i + k] = -gx[k] * il2;
        }
        dlp[t] = dl;
    }
    for (int64_t j = 0; j < M; ++j) {
        double r[3] = {0, 0, 0};
        for (int t = 0; t < nt; ++t)
            for (int k = 0; k < 3; ++k) r[k] += dzr[(size_t)t * 3 * M + 3 * j + k];
        if (dz)
            for (int k = 0; k < 3; ++k)
                dz[3 * j + k] = (T[0 + k] * r[0] + T[4 + k] * r[1] + T[8 + k] * r[2]) * il2;
        if (dv)
            for (int k = 0; k < D; ++k) {
                double a = 0.0;
                for (int t = 0; t < nt; ++t) a += dvr[(size_t)t * D * M + (size_t)D * j + k];
                dv[(size_t)D * j + k] = a;
            }
    }
    if (dell) {
        double a = 0.0;
        for (int t = 0; t < nt; ++t) a += dlp[t];
        *dell = a;
    }
    free(dlp);
    free(dvr);
    free(dzr);
    free(zt);
    return 0;
}

/* Source-side derivatives for a subset of source points only (for sampled
 * checks at full sizes): dF/dx_i and dF/du_i for i in idx.               */
int oracle_source_grad(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                       double ell, double sigma, double kappa, const double T[12],
                       const int64_t *idx, int64_t nidx, double *dx, double *du)
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int D = spec_dim(sp);
    const int64_t M = Z->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double il2 = 1.0 / (ell * ell);
    const double s2 = sigma * sigma;
    double *zt = (double *)malloc(sizeof(double) * 3 * (M > 0 ? M : 1));
    if (!zt) return -2;
    oracle_transform(T, Z->xyz, M, zt);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nidx; ++q) {
        const int64_t i = idx[q];
        const float *xi = X->xyz + 3 * i;
        const float *ui = D ? X->feat + (size_t)D * i : NULL;
        double cb[ORACLE_MAX_BLOCKS];
        double gx[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) du[(size_t)D * q + k] = 0.0;
        for (int64_t j = 0; j < M; ++j) {
            double d[3];
            double s = canonical_distance(xi, zt + 3 * j, d);
            if (!(s <= rc2)) continue;
            const float *vj = D ? Z->feat + (size_t)D * j : NULL;
            double c = feature_kernel(sp, ui, vj, cb);
            double kg = s2 * exp(-s / (2.0 * ell * ell));
            double w = c * kg;
            for (int k = 0; k < 3; ++k) gx[k] += w * d[k];
            int off = 0;
            for (int b = 0; b < sp->nblocks; ++b) {
                const int n = sp->dim[b];
                if (sp->kind[b] == ORACLE_SE) {
                    double ib = 1.0 / (sp->ell[b] * sp->ell[b]);
                    for (int k = 0; k < n; ++k)
                        du[(size_t)D * q + off + k] += -w * ((double)ui[off + k] - (double)vj[off + k]) * ib;
                } else {
                    double other = kg;
                    for (int b2 = 0; b2 < sp->nblocks; ++b2)
                        if (b2 != b) other *= cb[b2];
                    for (int k = 0; k < n; ++k) du[(size_t)D * q + off + k] += other * (double)vj[off + k];
                }
                off += n;
            }
        }
        for (int k = 0; k < 3; ++k) dx[3 * q + k] = -gx[k] * il2;
    }
    free(zt);
    return 0;
}

/* dF/dz_j and dF/dv_j for the targets j in idx only (the target side of
 * oracle_backward, restricted to a subset so large clouds can be sampled):
 *   dF/dz_j = R^T ell^-2 sum_i w_ij d_ij, d_ij = x_i - z'_j;
 *   SE block b: dF/dv_j = + sum_i w_ij (u_i - v_j) / ell_b^2;
 *   LIN block b: dF/dv_j = sum_i k_ij prod_{b' != b} c^(b') u_i.          */
int oracle_target_grad(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                       double ell, double sigma, double kappa, const double T[12],
                       const int64_t *idx, int64_t nidx, double *dz, double *dv)
{
    if (!(ell > 0.0) || !(sigma > 0.0) || !(kappa > 0.0)) return -1;
    const int D = spec_dim(sp);
    const int64_t N = X->n;
    const double rc2 = cutoff_sq(ell, kappa);
    const double il2 = 1.0 / (ell * ell);
    const double s2 = sigma * sigma;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nidx; ++q) {
        const int64_t j = idx[q];
        double zt[3];
        canonical_transform(T, Z->xyz + 3 * j, zt);
        const float *vj = D ? Z->feat + (size_t)D * j : NULL;
        double cb[ORACLE_MAX_BLOCKS];
        double gz[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) dv[(size_t)D * q + k] = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double d[3];
            double s = canonical_distance(X->xyz + 3 * i, zt, d);
            if (!(s <= rc2)) continue;
            const float *ui = D ? X->feat + (size_t)D * i : NULL;
            double c = feature_kernel(sp, ui, vj, cb);
            double kg = s2 * exp(-s / (2.0 * ell * ell));
            double w = c * kg;
            for (int k = 0; k < 3; ++k) gz[k] += w * d[k];
            int off = 0;
            for (int b = 0; b < sp->nblocks; ++b) {
                const int n = sp->dim[b];
                if (sp->kind[b] == ORACLE_SE) {
                    double ib = 1.0 / (sp->ell[b] * sp->ell[b]);
                    for (int k = 0; k < n; ++k)
                        dv[(size_t)D * q + off + k] += w * ((double)ui[off + k] - (double)vj[off + k]) * ib;
                } else {
                    double other = kg;
                    for (int b2 = 0; b2 < sp->nblocks; ++b2)
                        if (b2 != b) other *= cb[b2];
                    for (int k = 0; k < n; ++k) dv[(size_t)D * q + off + k] += other * (double)ui[off + k];
                }
                off += n;
            }
        }
        /* R^T (ell^-2 gz) */
        for (int k = 0; k < 3; ++k)
            dz[3 * q + k] = (T[k] * gz[0] + T[4 + k] * gz[1] + T[8 + k] * gz[2]) * il2;
    }
    return 0;
}
