// cvo_build.hip -- device-side preparation of point clouds for the pair pass.
//
// The paper's double sum (eq. (7)) is sparse (Sec. III-B): a point only
// interacts with points within the cutoff.  These kernels bin clouds so the
// pair pass scans neighbourhoods instead of all N*M pairs:
//   bbox_kernel       per-cloud bounding box and a non-finite-coordinate count
//   grid_keys         row-major cell index of every point (reference view)
//   morton_keys       Morton code of every point (query view)
//   radix_hist / radix_scatter   stable LSD radix sort of (key, index)
//   scan_*            exclusive prefix sums
//   gather_points     sorted float4 copies and padded, pre-scaled feature rows
//   cell_table        dense first-index-per-cell table (lower bounds)
//   cluster_heads / cluster_emit  octree clusters of at most cluster_max points
//   chunk_heads       or clusters as halved chunks of Morton-ordered points
// Every kernel is deterministic: counts use integer atomics only, and all
// orderings come from the stable sort.
#include "cvo_launch.hpp"

namespace cvo {

// ---------------------------------------------------------------- bbox
__global__ __launch_bounds__(1024) void bbox_kernel(const CloudPtrs *clouds, float *out)
{
    const int c = blockIdx.x;
    const float *xyz = clouds[c].xyz;
    const long long n = clouds[c].n;
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    int bad = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            float v = xyz[3 * i + k];
            if (!isfinite(v)) { bad = 1; continue; }
            mn[k] = fminf(mn[k], v);
            mx[k] = fmaxf(mx[k], v);
        }
    }
    __shared__ float smn[3][1024], smx[3][1024];
    __shared__ int sbad[1024];
    for (int k = 0; k < 3; ++k) { smn[k][threadIdx.x] = mn[k]; smx[k][threadIdx.x] = mx[k]; }
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            for (int k = 0; k < 3; ++k) {
                smn[k][threadIdx.x] = fminf(smn[k][threadIdx.x], smn[k][threadIdx.x + s]);
                smx[k][threadIdx.x] = fmaxf(smx[k][threadIdx.x], smx[k][threadIdx.x + s]);
            }
            sbad[threadIdx.x] += sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k) { out[8 * c + k] = smn[k][0]; out[8 * c + 3 + k] = smx[k][0]; }
        out[8 * c + 6] = (float)sbad[0];
        out[8 * c + 7] = 0.0f;
    }
}

// ---------------------------------------------------------------- keys
// Cell index along one axis: floor((p - o) * s) in FP64, clamped, with s the
// same 1/h (or 1/q) the range computations use.  Subtraction and
// multiplication by a positive constant are monotone under rounding, so a
// point inside [lo, hi] lands in a cell between those of lo and hi.
__device__ inline int cell_of(float p, double o, double s, int n)
{
    double f = floor(((double)p - o) * s);
    f = fmin(fmax(f, 0.0), (double)(n - 1));
    return (int)f;
}

__global__ void grid_keys(const CloudPtrs *clouds, const GridBuild *gb, unsigned long long *keys,
                          int *vals, int kbits)
{
    const int c = blockIdx.y;
    const GridBuild g = gb[c];
    const long long n = clouds[c].n;
    const float *xyz = clouds[c].xyz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        int ix = cell_of(xyz[3 * i + 0], g.ox, g.inv_h, g.nx);
        int iy = cell_of(xyz[3 * i + 1], g.oy, g.inv_h, g.ny);
        int iz = cell_of(xyz[3 * i + 2], g.oz, g.inv_h, g.nz);
        unsigned long long cell = (unsigned long long)ix +
                                  (unsigned long long)g.nx * ((unsigned long long)iy + (unsigned long long)g.ny * iz);
        keys[g.pt_base + i] = ((unsigned long long)c << kbits) | cell;
        vals[g.pt_base + i] = (int)(g.pt_base + i);
    }
}

__device__ inline unsigned long long spread3(unsigned long long v)
{
    // spread the low 21 bits of v so bit k lands at bit 3k
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

__global__ void morton_keys(const CloudPtrs *clouds, const ClusterBuild *cb, unsigned long long *keys,
                            int *vals, int bits)
{
    const int c = blockIdx.y;
    const ClusterBuild g = cb[c];
    const long long n = clouds[c].n;
    const float *xyz = clouds[c].xyz;
    const int lim = (1 << bits);
    const double iq = 1.0 / g.q;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        unsigned long long qx = (unsigned long long)cell_of(xyz[3 * i + 0], g.ox, iq, lim);
        unsigned long long qy = (unsigned long long)cell_of(xyz[3 * i + 1], g.oy, iq, lim);
        unsigned long long qz = (unsigned long long)cell_of(xyz[3 * i + 2], g.oz, iq, lim);
        unsigned long long m = spread3(qx) | (spread3(qy) << 1) | (spread3(qz) << 2);
        keys[g.pt_base + i] = ((unsigned long long)c << (3 * bits)) | m;
        vals[g.pt_base + i] = (int)(g.pt_base + i);
    }
}

// ---------------------------------------------------------------- scan
// Exclusive prefix sum of n ints in three launches: per-block scans of 2048
// elements, a single-block scan of the block sums, then the add-back.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ inline int block_exclusive_scan(int v, int *total)
{
    __shared__ int sh[kScanThreads];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int t = (threadIdx.x >= off) ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int incl = sh[threadIdx.x];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kScanThreads) void scan_tiles(const int *in, int *out, int *bsum, long long n)
{
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void scan_sums(int *bsum, int nb, int *total)
{
    // nb <= kScanTile * kScanTile is guaranteed by the launcher (chunks of 2048)
    int carry = 0;
    for (int base = 0; base < nb; base += kScanTile) {
        const int b0 = base + threadIdx.x * kScanItems;
        int v[kScanItems];
        int s = 0;
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = (b0 + k < nb) ? bsum[b0 + k] : 0;
            s += v[k];
        }
        int tot;
        int ex = block_exclusive_scan(s, &tot) + carry;
        for (int k = 0; k < kScanItems; ++k) {
            if (b0 + k < nb) bsum[b0 + k] = ex;
            ex += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_add(int *out, const int *bsum, long long n)
{
    const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
    const int add = bsum[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) out[base + k] += add;
}

void launch_exclusive_scan(const int *in, int *out, int *bsum, long long n, int *total, hipStream_t s)
{
    const int nb = (int)((n + kScanTile - 1) / kScanTile);
    if (nb == 0) {
        if (total) hipMemsetAsync(total, 0, sizeof(int), s);
        return;
    }
    hipLaunchKernelGGL(scan_tiles, dim3(nb), dim3(kScanThreads), 0, s, in, out, bsum, n);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, total);
    hipLaunchKernelGGL(scan_add, dim3(nb), dim3(kScanThreads), 0, s, out, bsum, n);
}

// ---------------------------------------------------------------- radix sort
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = kRadixTile / kRadixThreads;
static_assert(kRadixTile % kRadixThreads == 0, "radix tile");

__global__ __launch_bounds__(kRadixThreads) void radix_hist(const unsigned long long *keys, long long n,
                                                            int shift, int *hist, int ntiles)
{
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixItems; ++r) {
        long long e = base + r * kRadixThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: within a round of 256 consecutive elements, an element's
// rank among equal digits is (earlier lanes of its wave with the digit) +
// (counts of the digit in earlier waves); rounds and tiles follow in order.
__global__ __launch_bounds__(kRadixThreads) void radix_scatter(const unsigned long long *kin, const int *vin,
                                                               unsigned long long *kout, int *vout, long long n,
                                                               int shift, const int *hist, int ntiles)
{
    __shared__ int run[256];
    __shared__ int wcnt[kRadixThreads / kWave][256];
    __shared__ int woff[kRadixThreads / kWave][256];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    run[threadIdx.x] = hist[threadIdx.x * ntiles + blockIdx.x];
    const unsigned long long lt = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    const long long base = (long long)blockIdx.x * kRadixTile;
    for (int r = 0; r < kRadixItems; ++r) {
        const long long e = base + r * kRadixThreads + threadIdx.x;
        const bool valid = e < n;
        unsigned long long key = valid ? kin[e] : 0ULL;
        int val = valid ? vin[e] : 0;
        int d = valid ? (int)((key >> shift) & 255) : 256;
        unsigned long long peers = ~0ULL;
        for (int b = 0; b < 9; ++b) {
            unsigned long long bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        const int rank = __popcll(peers & lt);
        for (int k = threadIdx.x; k < (kRadixThreads / kWave) * 256; k += kRadixThreads)
            (&wcnt[0][0])[k] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wv][d] = __popcll(peers);
        __syncthreads();
        {
            const int dd = threadIdx.x;  // one thread per digit
            int acc = run[dd];
            for (int w = 0; w < kRadixThreads / kWave; ++w) {
                woff[w][dd] = acc;
                acc += wcnt[w][dd];
            }
            run[dd] = acc;
        }
        __syncthreads();
        if (valid) {
            const int pos = woff[wv][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

void launch_radix_sort(unsigned long long *keys, int *vals, unsigned long long *ktmp, int *vtmp, int *hist,
                       int *bsum, long long n, int bits, hipStream_t s, bool *result_in_tmp)
{
    const int ntiles = (int)((n + kRadixTile - 1) / kRadixTile);
    bool in_tmp = false;
    if (n > 1) {
        for (int shift = 0; shift < bits; shift += 8) {
            const unsigned long long *ki = in_tmp ? ktmp : keys;
            const int *vi = in_tmp ? vtmp : vals;
            unsigned long long *ko = in_tmp ? keys : ktmp;
            int *vo = in_tmp ? vals : vtmp;
            hipLaunchKernelGGL(radix_hist, dim3(ntiles), dim3(kRadixThreads), 0, s, ki, n, shift, hist, ntiles);
            launch_exclusive_scan(hist, hist, bsum, (long long)ntiles * 256, nullptr, s);
            hipLaunchKernelGGL(radix_scatter, dim3(ntiles), dim3(kRadixThreads), 0, s, ki, vi, ko, vo, n, shift,
                               hist, ntiles);
            in_tmp = !in_tmp;
        }
    }
    *result_in_tmp = in_tmp;
}

// ---------------------------------------------------------------- gather
// Sorted float4 copies of the raw coordinates, the permutation, and padded
// feature rows (destination column k = source column col[k] times scale[k]).
__global__ void gather_points(const unsigned long long *keys, const int *vals, long long ntot, int cshift,
                              const CloudPtrs *clouds, const long long *pt_base, FeatLayout lay,
                              float4 *pts, float *feat, int *perm)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < ntot;
         p += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(keys[p] >> cshift);
        const long long i = vals[p] - pt_base[c];
        const float *xyz = clouds[c].xyz;
        pts[p] = make_float4(xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2], 0.0f);
        perm[p] = (int)i;
        if (lay.d4 > 0) {
            const float *f = clouds[c].feat + i * lay.src_dim;
            for (int k = 0; k < lay.d4; ++k) {
                float v = 0.0f;
                if (lay.col[k] >= 0) {
                    v = f[lay.col[k]] * lay.scale[k];
                } else if (lay.col[k] == -2) {
                    // tensor-product column of the folded LIN blocks (eq. (6))
                    int cc = k - lay.sed;
                    v = 1.0f;
                    for (int b = lay.nlin - 1; b >= 0; --b) {
                        v *= f[lay.lin_src[b] + cc % lay.lin_dim[b]];
                        cc /= lay.lin_dim[b];
                    }
                }
                feat[p * lay.d4 + k] = v;
            }
        }
    }
}

// ---------------------------------------------------------------- cell table
__device__ inline long long lower_bound_u64(const unsigned long long *a, long long n, unsigned long long x)
{
    long long lo = 0, hi = n;
    while (lo < hi) {
        long long mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__global__ void cell_table(const unsigned long long *keys, long long ntot, const GridBuild *gb, int kbits,
                           int *cell_start)
{
    const int c = blockIdx.y;
    const GridBuild g = gb[c];
    const long long ncells = (long long)g.nx * g.ny * g.nz;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k <= ncells;
         k += (long long)gridDim.x * blockDim.x) {
        unsigned long long target = ((unsigned long long)c << kbits) | (unsigned long long)k;
        cell_start[g.cell_base + k] = (int)lower_bound_u64(keys, ntot, target);
    }
}

// ---------------------------------------------------------------- clusters
// A point's cluster is the largest aligned Morton block (level L <= lcap,
// edge 2^L quanta) holding at most tpw points, with (lcap, tpw) given per
// cloud.  Block counts grow with L, so every point of such a block makes the
// same choice.  A level-0 block with more than tpw points is cut into
// ceil(count/tpw) near-equal chunks.
__global__ void cluster_heads(const unsigned long long *keys, long long ntot, const int2 *caps, int cshift,
                              int *head, int2 *span)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < ntot;
         p += (long long)gridDim.x * blockDim.x) {
        const unsigned long long key = keys[p];
        const int2 cap = caps[key >> cshift];
        const int lcap = cap.x, tpw = cap.y;
        if (lcap < 0) continue;  // clustered by the chunk rule
        long long start = -1, end = -1;
        long long lo0 = 0, hi0 = 0;
        for (int L = lcap; L >= 0; --L) {
            const unsigned long long blk = key >> (3 * L);
            const long long lo = lower_bound_u64(keys, ntot, blk << (3 * L));
            const long long hi = lower_bound_u64(keys, ntot, (blk + 1) << (3 * L));
            if (hi - lo <= tpw) { start = lo; end = hi; break; }
            lo0 = lo; hi0 = hi;
        }
        if (start < 0) {
            const long long cnt = hi0 - lo0;
            const long long nch = (cnt + tpw - 1) / tpw;
            const long long sz = (cnt + nch - 1) / nch;
            const long long ch = (p - lo0) / sz;
            start = lo0 + ch * sz;
            end = start + sz < hi0 ? start + sz : hi0;
        }
        head[p] = (p == start) ? 1 : 0;
        span[p] = make_int2((int)start, (int)(end - start));
    }
}

// Chunk clusters, one wavefront per chunk of cluster_max consecutive
// Morton-ordered points (lane l holds point l).  Level k splits the chunk
// into aligned parts of cluster_max >> k points; a part is final when its
// bounding box edge fits the cap or it holds one point.  Parts are thus
// runs of cluster_max / 2^k points (the last chunk of a cloud clipped),
// which fill the pair pass's power-of-two lane groups, and each stays
// compact in space.  head/span as cluster_heads writes them.
__global__ __launch_bounds__(kWave) void chunk_heads(const float4 *pts, const ClusterBuild *cb, const int2 *caps,
                                                      int B, long long nchunks, int *head, int2 *span)
{
    const long long w = blockIdx.x;
    if (w >= nchunks) return;
    // the cloud of this chunk (chunk_base ascending)
    int c = 0;
    while (c + 1 < B && cb[c + 1].chunk_base <= w) ++c;
    const ClusterBuild g = cb[c];
    const int tpw = caps[c].y;
    const long long c0 = g.pt_base + (w - g.chunk_base) * tpw;
    const int len = (int)min((long long)tpw, g.pt_base + g.n - c0);
    const int l = threadIdx.x;
    const bool in = l < len;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    if (in) q = pts[c0 + l];
    bool done = !in;
    for (int sz = tpw; sz >= 1; sz >>= 1) {
        // bounding box of each aligned part of sz lanes (lanes beyond len neutral)
        double lo[3] = {in ? (double)q.x : INFINITY, in ? (double)q.y : INFINITY, in ? (double)q.z : INFINITY};
        double hi[3] = {in ? (double)q.x : -INFINITY, in ? (double)q.y : -INFINITY, in ? (double)q.z : -INFINITY};
        for (int off = 1; off < sz; off <<= 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], __shfl_xor(lo[a], off));
                hi[a] = fmax(hi[a], __shfl_xor(hi[a], off));
            }
        }
        const double edge = fmax(hi[0] - lo[0], fmax(hi[1] - lo[1], hi[2] - lo[2]));
        const int first = l & ~(sz - 1);
        const int plen = min(sz, len - first);
        if (!done && (edge <= g.cap || plen <= 1)) {
            head[c0 + l] = (l == first) ? 1 : 0;
            span[c0 + l] = make_int2((int)(c0 + first), plen);
            done = true;
        }
        if (__all(done)) break;
    }
}

__global__ void cluster_emit(const int *head, const int *hidx, const int2 *span, const float4 *pts,
                             const unsigned long long *keys, int cshift, long long ntot, int2 *clus,
                             double4 *cgeo, int *cpair, int *tclus)
{
    for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < ntot;
         p += (long long)gridDim.x * blockDim.x) {
        if (!head[p]) continue;
        const int idx = hidx[p];
        const int2 sp = span[p];
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int k = 0; k < sp.y; ++k) {
            float4 q = pts[sp.x + k];
            double v[3] = {(double)q.x, (double)q.y, (double)q.z};
            for (int a = 0; a < 3; ++a) { lo[a] = fmin(lo[a], v[a]); hi[a] = fmax(hi[a], v[a]); }
        }
        double cc[3], r2 = 0.0, mag = 0.0;
        for (int a = 0; a < 3; ++a) { cc[a] = 0.5 * (lo[a] + hi[a]); mag = fmax(mag, fabs(cc[a])); }
        for (int k = 0; k < sp.y; ++k) {
            float4 q = pts[sp.x + k];
            double dx = (double)q.x - cc[0], dy = (double)q.y - cc[1], dz = (double)q.z - cc[2];
            r2 = fmax(r2, dx * dx + dy * dy + dz * dz);
        }
        // inflate so FP64 rounding of the transformed centre and points can
        // never place a member outside the sphere
        const double r = sqrt(r2) * (1.0 + 1e-12) + 1e-12 * (mag + 1.0);
        clus[idx] = sp;
        cgeo[idx] = make_double4(cc[0], cc[1], cc[2], r);
        cpair[idx] = (int)(keys[p] >> cshift);
        for (int k = 0; k < sp.y; ++k) tclus[sp.x + k] = idx;
    }
}

// ---------------------------------------------------------------- launchers
void launch_bbox(const CloudPtrs *clouds, int B, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(bbox_kernel, dim3(B), dim3(1024), 0, s, clouds, out);
}

static int blocks_for(long long n, int threads, int cap = 65535)
{
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

void launch_grid_keys(const CloudPtrs *clouds, const GridBuild *gb, int B, long long nmax,
                      unsigned long long *keys, int *vals, int kbits, hipStream_t s)
{
    hipLaunchKernelGGL(grid_keys, dim3(blocks_for(nmax, 256, 4096), B), dim3(256), 0, s, clouds, gb, keys, vals,
                       kbits);
}

void launch_morton_keys(const CloudPtrs *clouds, const ClusterBuild *cb, int B, long long nmax,
                        unsigned long long *keys, int *vals, int bits, hipStream_t s)
{
    hipLaunchKernelGGL(morton_keys, dim3(blocks_for(nmax, 256, 4096), B), dim3(256), 0, s, clouds, cb, keys,
                       vals, bits);
}

void launch_gather(const unsigned long long *keys, const int *vals, long long ntot, int cshift,
                   const CloudPtrs *clouds, const long long *pt_base, const FeatLayout &lay, float4 *pts,
                   float *feat, int *perm, hipStream_t s)
{
    hipLaunchKernelGGL(gather_points, dim3(blocks_for(ntot, 256)), dim3(256), 0, s, keys, vals, ntot, cshift,
                       clouds, pt_base, lay, pts, feat, perm);
}

void launch_cell_table(const unsigned long long *keys, long long ntot, const GridBuild *gb, int B,
                       long long max_cells, int kbits, int *cell_start, hipStream_t s)
{
    hipLaunchKernelGGL(cell_table, dim3(blocks_for(max_cells + 1, 256, 8192), B), dim3(256), 0, s, keys, ntot,
                       gb, kbits, cell_start);
}

void launch_chunk_heads(const float4 *pts, const ClusterBuild *cb, const int2 *caps, int B, long long nchunks,
                        int *head, int2 *span, hipStream_t s)
{
    if (nchunks <= 0) return;
    hipLaunchKernelGGL(chunk_heads, dim3((unsigned)nchunks), dim3(kWave), 0, s, pts, cb, caps, B, nchunks, head, span);
}

void launch_cluster_heads(const unsigned long long *keys, long long ntot, const int2 *caps, int cshift,
                          int *head, int2 *span, hipStream_t s)
{
    hipLaunchKernelGGL(cluster_heads, dim3(blocks_for(ntot, 256)), dim3(256), 0, s, keys, ntot, caps, cshift, head,
                       span);
}

void launch_cluster_emit(const int *head, const int *hidx, const int2 *span, const float4 *pts,
                         const unsigned long long *keys, int cshift, long long ntot, int2 *clus, double4 *cgeo,
                         int *cpair, int *tclus, hipStream_t s)
{
    hipLaunchKernelGGL(cluster_emit, dim3(blocks_for(ntot, 256)), dim3(256), 0, s, head, hidx, span, pts, keys,
                       cshift, ntot, clus, cgeo, cpair, tclus);
}

}  // namespace cvo
