// cvo_internal.hpp -- shared host/device definitions of the gfx950 CVO library.
//
// Data layout in HBM (all arrays live in the handle's arena):
//   A cloud is prepared in one of two views, both holding sorted float4 copies
//   of the raw float32 coordinates (w unused) and sorted, padded feature rows
//   (stride D4 floats; SE columns pre-multiplied by sqrt(log2(e) / (2 ell_b^2))
//   so one exp2 of a plain sum of squares gives every SE factor, LIN columns
//   unscaled; padding columns are zero):
//     grid view    (reference side of a pair pass): points sorted by the
//                  row-major index of a uniform cell grid; a dense table
//                  cell_start[k] = first sorted index with cell >= k, so a
//                  run of cells along x is one contiguous index range.
//     cluster view (query side): points sorted by a Morton code; a cluster is
//                  an aligned octree block holding at most cluster_max points,
//                  with its centre and radius in the cloud's own frame.  A
//                  rigid motion keeps clusters compact, so they are built once
//                  per lengthscale band, never per iteration.
//   Several clouds are prepared together by prefixing every sort key with the
//   cloud index; the plain path is the batch of one.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cvo {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 1;  // pair pass: one wave per workgroup, so a finished piece frees its slot at once
constexpr int kQueueCap = 80;    // LDS candidate queue per wave
constexpr int kQueueFlush = 16;  // process the queue once it holds this many (cap >= flush + 64)
constexpr int kTraceLen = 8;
constexpr int kRadixTile = 1024;  // keys per workgroup and pass of the radix sort
constexpr int kRedVals = 48;     // values reduced per pair by the reduction kernel
constexpr int kRedThreads = 256;

enum Status { ST_RUNNING = 0, ST_CONVERGED = 1, ST_MAX_ITER = 2, ST_NO_OVERLAP = 3, ST_STATIONARY = 4 };

// Holds a wave-uniform value in scalar registers at this point, so its load
// is issued here (with the others of its round) and not sunk past a branch.
__device__ __forceinline__ void in_sgpr(int v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void in_sgpr(double v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ void in_sgpr(long long v) { asm volatile("" ::"s"(v)); }

// Per-pair registration state, resident on the device for the whole ascent.
struct alignas(16) PairState {
    double T[12];        // current pose [R|t], maps the Z frame into the X frame
    double Tinv[12];     // inverse pose (used by the source-side backward pass)
    double ell;          // current lengthscale
    double i_prev;       // indicator at the previous iteration (NaN: none)
    double F, i_theta, curv, tau, gnorm, r_max, dF_dell;
    double grad[6];
    double n_pairs;      // |P| of the last evaluation (exact integer in a double)
    double total_pairs;  // sum of |P| over the registration
    double rc_build;     // cutoff radius the current views were built for
    // lengthscale objective at the last evaluation (when it was asked for):
    // J = sum_{W_j > 0} log W_j - 3 |Z+| log ell, dJ/dell, its maximiser, |Z+|
    double J, dJ_dell, ell_ml, zplus;
    long long it;        // steps taken
    int status;          // Status
    int done;            // nonzero: later launches skip this pair
    int cls_built;       // pair-density class of the current views (-1: not chosen by density)
    int pause;           // nonzero: views must be rebuilt; launches skip the pair until then
};

// Density class of an evaluation from its in-cutoff pairs per query point
// (-1: unknown): 3 from t[0], 2 from t[1], 1 from t[2], else 0.
__host__ __device__ inline int density_class(double ppq, const double t[3])
{
    return !(ppq >= 0.0) ? -1 : (ppq >= t[0] ? 3 : (ppq >= t[1] ? 2 : (ppq >= t[2] ? 1 : 0)));
}

// Per-pair constants of the ascent.
struct alignas(16) AlignConst {
    double ell_min, decay, ind_rel_tol, eps_rot, eps_trans, step_lambda;
    double sqrt_nm;      // sqrt(|X| |Z|)
    double inv_m;        // 1 / |Z|
    double kappa;        // cutoff radius / ell (infinite: no cutoff, views never rebuilt)
    double rebuild_ratio; // pause for new views once kappa ell < rebuild_ratio * rc_build
    long long max_iter;
    int fixed_iters;
    int metric;          // 0: kinetic-energy metric of the moving cloud, 1: identity
    int ell_mode;        // 0: annealing (Sec. IV), 1: adaptive (maximiser of the lengthscale objective)
    double ell_init;     // adaptive mode: upper clamp of ell
    int adaptive;        // nonzero: also pause when the density class drops below cls_built
    double cls_t[3];     // pairs per query where density classes 3, 2 and 1 begin
    const double *ell_sched;  // replay: lengthscale of every iteration (device; null: annealing)
    long long n_sched;        // replay: iterations to run
};

// Uniform grid of one cloud (reference role).
struct alignas(16) GridDesc {
    double ox, oy, oz;   // origin (cell (0,0,0) starts here)
    double h;            // cell edge (m)
    double inv_h;        // 1 / h; a coordinate p lies in cell floor((p - o) * inv_h)
    int nx, ny, nz;
    int cell_base;       // offset of this cloud's table in cell_start
    long long pt_base;   // sorted points of this cloud: [pt_base, pt_base + n)
    long long n;
};

// Clusters of one cloud (query role).
struct alignas(16) ClusterDesc {
    int clus_base, nclus;  // clusters [clus_base, clus_base + nclus)
    int pt_base, n;        // sorted points [pt_base, pt_base + n)
};

// Feature layout after combining the spec's blocks: all SE columns first
// (pre-scaled), then at most one LIN block.
struct FeatLayout {
    int sed, lind;     // SE columns, LIN columns of the kernel variant (padded)
    int d4;            // row stride (multiple of 4, >= sed + lind)
    int src_dim;       // D of the caller's rows
    // Several LIN blocks are folded into one by the tensor-product identity
    // of eq. (6), <u1 (x) u2, v1 (x) v2> = <u1, v1> <u2, v2>: destination LIN
    // column sed + c (c < prod lin_dim) holds prod_b u_b[digit_b(c)], the
    // digits of c in the mixed radix (lin_dim[0], ..., lin_dim[nlin - 1])
    // with block 0 most significant.  nlin = 0: at most one LIN block, mapped
    // column by column through col[].
    int nlin;
    int lin_src[8];    // first source column of each LIN block
    int lin_dim[8];    // its width
    int col[64];       // destination column -> source column (-1: zero padding; -2: tensor-product column)
    float scale[64];   // destination column scale (SE: sqrt(log2(e) / (2 ell_b^2)))
    double gscale[64]; // accumulated feature gradient -> dF/d(feature) (SE: 1/(scale ell_b^2))
    float sig2;        // sigma^2 * prod_b sigma_b^2 over SE blocks
};

// Arguments of the pair pass.  The unit of work is a piece: piece p of np
// takes every np-th 64-candidate chunk of one cluster's candidate list (the
// concatenation of its neighbourhood rows), so heavy clusters are split into
// pieces of similar work.  One wave per piece, pieces ordered heaviest first.
// One piece in dispatch order with what its wave needs first, gathered at
// planning time so the wave's prologue is one load: the piece (cluster, p,
// np, first output slot), its pair, its cluster's points and geometry.
struct alignas(32) PieceRec {
    int4 pc;
    int b, first, n, pad;
    double4 geo;
};

struct PairPassArgs {
    // query side (cluster view)
    const float4 *qpts;
    const float *qfeat;
    const int2 *clus;     // (first sorted index, count)
    const double4 *cgeo;  // (centre xyz in the query frame, radius)
    const int *cpair;     // pair of each cluster
    int nclus;
    const PieceRec *recs; // the pieces in processing order (heaviest first), with their cluster data
    int npieces;
    // reference side (grid view)
    const float4 *rpts;
    const float *rfeat;
    const int *cell_start;
    const GridDesc *grids;  // per pair
    // per-pair pose applied to query points (query frame -> reference frame),
    // and the pose in canonical orientation (Z frame -> X frame)
    const PairState *state;
    int pose_is_inverse;    // 0: query = Z (pose T); 1: query = X (pose T^-1)
    float sig2;
    double kappa;           // +inf: no cutoff
    // outputs, indexed by piece slot + position of the query in its cluster
    double *oW;
    double *oD;     // 3 per query
    float *oS;      // 6 per query (forward mode)
    int *oCnt;
    double *oG;     // d4 per query (backward mode): feature gradients
    double *oL;     // 1 per query (backward mode): sum w s'
};

}  // namespace cvo
