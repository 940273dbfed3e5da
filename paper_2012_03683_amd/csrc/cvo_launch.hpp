// cvo_launch.hpp -- host-side launchers of the device kernels (internal).
#pragma once
#include "cvo_internal.hpp"

namespace cvo {

struct CloudPtrs {
    const float *xyz;
    const float *feat;
    long long n;
};

typedef GridDesc GridBuild;

struct alignas(16) ClusterBuild {
    double ox, oy, oz;  // Morton origin
    double q;           // quantum (edge of a level-0 block)
    long long pt_base;
    long long n;
    double cap;           // largest cluster bounding-box edge (chunk rule)
    long long chunk_base; // first chunk of this cloud (chunk rule)
};

void launch_bbox(const CloudPtrs *clouds, int B, float *out, hipStream_t s);
void launch_grid_keys(const CloudPtrs *clouds, const GridBuild *gb, int B, long long nmax,
                      unsigned long long *keys, int *vals, int kbits, hipStream_t s);
void launch_morton_keys(const CloudPtrs *clouds, const ClusterBuild *cb, int B, long long nmax,
                        unsigned long long *keys, int *vals, int bits, hipStream_t s);
void launch_exclusive_scan(const int *in, int *out, int *bsum, long long n, int *total, hipStream_t s);
void launch_radix_sort(unsigned long long *keys, int *vals, unsigned long long *ktmp, int *vtmp, int *hist,
                       int *bsum, long long n, int bits, hipStream_t s, bool *result_in_tmp);
void launch_gather(const unsigned long long *keys, const int *vals, long long ntot, int cshift,
                   const CloudPtrs *clouds, const long long *pt_base, const FeatLayout &lay, float4 *pts,
                   float *feat, int *perm, hipStream_t s);
void launch_cell_table(const unsigned long long *keys, long long ntot, const GridBuild *gb, int B,
                       long long max_cells, int kbits, int *cell_start, hipStream_t s);
void launch_cluster_heads(const unsigned long long *keys, long long ntot, const int2 *caps, int cshift,
                          int *head, int2 *span, hipStream_t s);
// Chunk rule: each cloud's Morton-sorted points cut into chunks of at most
// cluster_max (caps[c].y) consecutive points, each chunk subdivided by
// halving until every part's bounding box edge is within cb[c].cap.
void launch_chunk_heads(const float4 *pts, const ClusterBuild *cb, const int2 *caps, int B, long long nchunks,
                        int *head, int2 *span, hipStream_t s);
void launch_cluster_emit(const int *head, const int *hidx, const int2 *span, const float4 *pts,
                         const unsigned long long *keys, int cshift, long long ntot, int2 *clus, double4 *cgeo,
                         int *cpair, int *tclus, hipStream_t s);

// pair pass: mode 0 = forward moments, 1 = backward (feature gradients)
// returns false when no kernel exists for the feature layout
bool launch_pair_pass(const PairPassArgs &a, const FeatLayout &lay, int mode, hipStream_t s);
void launch_plan_count(const PairPassArgs &a, int work, int *npieces, int *cmax, long long *ccount, hipStream_t s);
void launch_plan_emit(const PairPassArgs &a, const int *npieces, const int *pbase, const long long *ccount,
                      int4 *pieces, int *pn, unsigned long long *key, int *val, int2 *cpieces, hipStream_t s);
void launch_plan_slots(int4 *pieces, const int *tbase, int npieces, hipStream_t s);
void launch_plan_qmap(const int2 *clus, const int2 *cpieces, const int4 *pieces, int nclus, int4 *qmap,
                      hipStream_t s);
// recs[i] = piece porder[i] with its pair and cluster data (dispatch order)
void launch_plan_records(const int *porder, const int4 *pieces, const int *cpair, const int2 *clus,
                         const double4 *cgeo, int npieces, PieceRec *recs, hipStream_t s);


// Where a query's partial moments live: qmap[j] = (t, n, np, s0) for query j
// at position t of a cluster of n queries cut into np pieces; the cluster's
// pieces own consecutive blocks of n output slots, so the query's partial of
// piece k is at slot s0 + k n.  Partials are combined in piece order.
struct SlotMap {
    const int4 *qmap;
};

struct ReduceArgs {
    const float4 *qpts;
    const ClusterDesc *cdesc;  // per pair: query points [pt_base, pt_base + n)
    SlotMap map;
    const double *W;
    const double *D;
    const float *S;
    const int *cnt;
    PairState *state;
    const AlignConst *ac;
    double *partials;          // B * kRedVals * nblk (per pair value-major: value v of block k at v * nblk + k)
    double *trace;             // B * trace_rows * kTraceLen, may be null
    long long trace_rows;
    int nblk;
    int mode;                  // 0: evaluate only, 1: evaluate and take an ascent step
    int ellobj;                // nonzero: also reduce the lengthscale objective's sums
    int one_query;             // nonzero: nblk * kRedThreads >= every cloud's query count (one query per thread)
};
void launch_reduce(const ReduceArgs &a, int B, hipStream_t s);

// backward post-processing
struct BackwardArgs {
    SlotMap map;
    const int *qperm;         // sorted query index -> original index within its cloud
    const double *D;          // 3 per sorted query (scaled units)
    const double *G;          // d4 per sorted query
    const PairState *state;
    int pose_is_inverse;
    FeatLayout lay;
    double gF;
    float *dxyz;              // original-order output, n x 3 (may be null)
    float *dfeat;             // original-order output, n x src_dim (may be null)
    const float *src_feat;    // the query cloud's own feature rows (original order, n x src_dim), read
                              // for the chain rule through folded LIN blocks
    long long n;
};
void launch_backward_finish(const BackwardArgs &a, hipStream_t s);

// point selection (FAST scores, threshold, raster-order compaction)
struct SelectArgs {
    const uint8_t *gray;   // H x W
    const float *depth;    // H x W
    const float *feat;     // H x W x D (may be null if D == 0)
    int W, H, D;
    float dmin, dmax;      // valid depth range, compared in FP32
    double fx, fy, cx, cy;
    int cap;               // largest selection allowed
    short *key;            // H x W scratch: score if the pixel has depth, else -1
    short *score;          // H x W scores for the caller (may be null)
    int *hist;             // 256, zero on entry
    int *res;              // (threshold, count)
    int *bcount, *boff, *bsum;  // per 256-pixel block counts, their exclusive scan, scan scratch
    float *xyz;            // cap x 3
    float *fout;           // cap x D
};
void launch_select(const SelectArgs &a, hipStream_t s);
int select_blocks(long long npix);
void launch_sum_doubles(const double *in, long long n, double *out, hipStream_t s);

}  // namespace cvo
