/*
 * cvo_oracle.h -- TEST INFRASTRUCTURE ONLY: the FP64 CPU oracle's own
 * declarations.  Nothing in the product library includes this header.
 */
#ifndef CVO_ORACLE_H
#define CVO_ORACLE_H
#include <stdint.h>

#define ORACLE_MAX_BLOCKS 8
#define ORACLE_SE 0  /* squared-exponential block kernel (eq. (5)) */
#define ORACLE_LIN 1 /* linear (inner product) block kernel (eq. (4), (6)) */

/* status values of a registration (same numbering as the product ABI) */
#define ORACLE_CONVERGED 1
#define ORACLE_MAX_ITER 2
#define ORACLE_NO_OVERLAP 3
#define ORACLE_STATIONARY 4

/* metric on se(3) for the ascent direction */
#define ORACLE_METRIC_KINETIC 0  /* mean squared point velocity of the moving cloud */
#define ORACLE_METRIC_IDENTITY 1 /* plain coordinates (omega, v) */

/* layout of oracle_evaluate's output vector */
#define ORACLE_F 0
#define ORACLE_G 1      /* 6: omega xyz, v xyz */
#define ORACLE_PHI2 7   /* curvature of F(Exp(tau g) T) at tau = 0 */
#define ORACLE_DELL 8   /* dF/dell with the cutoff radius fixed */
#define ORACLE_ABSF 9   /* sum |w| */
#define ORACLE_ABSG 10  /* 6: sums of |w| |per-pair gradient term| */
#define ORACLE_RMAX 16  /* max_j |T z_j| */
#define ORACLE_ITHETA 17 /* F / sqrt(|X| |Z|) */
#define ORACLE_EVAL_LEN 18

#define ORACLE_TRACE_LEN 8  /* it, ell, F, |g|, tau, indicator, |P|, phi'' */
#define ORACLE_REPORT_LEN 6 /* iterations, final ell, F, indicator, |P|, status */

typedef struct {
    const float *xyz;  /* n x 3 */
    const float *feat; /* n x D, may be NULL when D = 0 */
    int64_t n;
} oracle_cloud;

typedef struct {
    int32_t nblocks;
    int32_t dim[ORACLE_MAX_BLOCKS];
    int32_t kind[ORACLE_MAX_BLOCKS];
    double ell[ORACLE_MAX_BLOCKS];
    double sigma[ORACLE_MAX_BLOCKS];
} oracle_spec;

/* how the lengthscale moves during a registration */
#define ORACLE_ELL_ANNEAL 0   /* Sec. IV: decay by `decay` when the indicator stabilises */
#define ORACLE_ELL_ADAPTIVE 1 /* Sec. VI: ell follows the maximiser of oracle_ell_objective's J */

/* layout of oracle_ell_objective's output vector */
#define ORACLE_J 0        /* J(T, ell) */
#define ORACLE_DJ 1       /* dJ/dell, pair set frozen */
#define ORACLE_ELL_ML 2   /* sqrt(sum_j r_j / (3 |Z+|)), 0 when Z+ is empty */
#define ORACLE_ZPLUS 3    /* |Z+| */
#define ORACLE_ELLOBJ_LEN 4

typedef struct {
    double ell_init, ell_min, decay, ind_rel_tol;
    double eps_rot, eps_trans, step_lambda;
    double sigma, kappa;
    int64_t max_iter;
    int32_t fixed_iters;
    int32_t metric;
    int32_t ell_mode;  /* ORACLE_ELL_ANNEAL or ORACLE_ELL_ADAPTIVE */
    int32_t reserved;
} oracle_align_params;

int oracle_num_threads(void);
void oracle_transform(const double T[12], const float *z, int64_t M, double *zt);
int oracle_evaluate(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                    double ell, double sigma, double kappa, const double T[12],
                    double out[ORACLE_EVAL_LEN], int64_t *n_pairs);
int oracle_evaluate_dir(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                        double ell, double sigma, double kappa, const double T[12],
                        const double *dir, double out[ORACLE_EVAL_LEN], int64_t *n_pairs);
void oracle_metric_tensor(const double T[12], const float *z, int64_t M, double G[36]);
int oracle_solve6(const double G[36], const double g[6], double d[6]);
int oracle_target_moments(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                          double ell, double sigma, double kappa, const double T[12],
                          const int64_t *idx, int64_t nidx, double *W, double *D, double *S,
                          int64_t *cnt);
void oracle_exp_se3(const double xi[6], double T[12]);
int oracle_ell_objective(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                         double ell, double sigma, double kappa, const double T[12],
                         double out[ORACLE_ELLOBJ_LEN]);
int oracle_align(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                 const oracle_align_params *ap, const double T_init[12], double T_out[12],
                 double report[ORACLE_REPORT_LEN], double *trace);
int oracle_backward(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                    double ell, double sigma, double kappa, const double T[12],
                    double *dx, double *dz, double *du, double *dv, double *dell);
int oracle_source_grad(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                       double ell, double sigma, double kappa, const double T[12],
                       const int64_t *idx, int64_t nidx, double *dx, double *du);
int oracle_target_grad(const oracle_cloud *X, const oracle_cloud *Z, const oracle_spec *sp,
                       double ell, double sigma, double kappa, const double T[12],
                       const int64_t *idx, int64_t nidx, double *dz, double *dv);
#endif
