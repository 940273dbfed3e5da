// cvo_select.hip -- point selection before registration (the paper's
// performance considerations, Sec. IV): pixels passing the FAST 9-of-16
// segment test, no non-maximum suppression, with the intensity threshold
// chosen so that the number of selected pixels with depth stays within a cap;
// the selection is compacted in raster order and back-projected.
//
//   score(p) = the largest integer t at which p is a corner: an arc A of 9
//              contiguous pixels of the radius-3 circle is all brighter than
//              I_p + t for t <= min_A I - I_p - 1 and all darker than I_p - t
//              for t <= I_p - max_A I - 1, so score(p) is the maximum of
//              these bounds over the 16 arcs (-1: a corner at no threshold,
//              or within 3 pixels of the border).
//   count(t) = #{p with depth : score(p) >= t} is non-increasing in t, so one
//              256-bin histogram of the scores gives every count; the
//              threshold is the smallest t with count(t) <= cap.
//
// Kernels: score + histogram (64 x 4 pixel tiles staged in LDS with a 3-pixel
// halo), threshold (one workgroup), per-block selected counts, an exclusive
// scan of those, and the emit pass (wave ballots give each selected pixel its
// rank).  All integer work, so the selection is exact.
#include "cvo_launch.hpp"

namespace cvo {

namespace {
constexpr int kTX = 64, kTY = 4;  // score tile: one wave per row of the tile
constexpr int kHalo = 3;
constexpr int kSelThreads = 256;
}  // namespace

__global__ __launch_bounds__(kTX *kTY) void fast_score_kernel(const uint8_t *gray, const float *depth, int W, int H,
                                                               float dmin, float dmax, short *key, short *score_out,
                                                               int *hist)
{
    // int cells: byte cells would put four neighbours in one LDS bank
    __shared__ int tile[kTY + 2 * kHalo][kTX + 2 * kHalo];
    __shared__ int lh[256];
    const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * kTX + tx;
    const int u0 = blockIdx.x * kTX, v0 = blockIdx.y * kTY;
    lh[tid] = 0;
    for (int i = tid; i < (kTY + 2 * kHalo) * (kTX + 2 * kHalo); i += kTX * kTY) {
        const int r = i / (kTX + 2 * kHalo), c = i % (kTX + 2 * kHalo);
        const int u = u0 + c - kHalo, v = v0 + r - kHalo;
        tile[r][c] = (u >= 0 && u < W && v >= 0 && v < H) ? (int)gray[(long long)v * W + u] : 0;
    }
    __syncthreads();
    const int u = u0 + tx, v = v0 + ty;
    if (u < W && v < H) {
        int s = -1;
        if (u >= kHalo && v >= kHalo && u < W - kHalo && v < H - kHalo) {
            // the radius-3 circle, (du, dv) in circular order
            constexpr int du[16] = {0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3, -3, -3, -2, -1};
            constexpr int dv[16] = {-3, -3, -2, -1, 0, 1, 2, 3, 3, 3, 2, 1, 0, -1, -2, -3};
            const int c = tile[ty + kHalo][tx + kHalo];
            int r[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) r[k] = tile[ty + kHalo + dv[k]][tx + kHalo + du[k]];
            // min and max of every circular window of 9: windows of 2, 4, 8, then 9
            int a2[16], b2[16], a4[16], b4[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                a2[k] = min(r[k], r[(k + 1) & 15]);
                b2[k] = max(r[k], r[(k + 1) & 15]);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                a4[k] = min(a2[k], a2[(k + 2) & 15]);
                b4[k] = max(b2[k], b2[(k + 2) & 15]);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int mn = min(min(a4[k], a4[(k + 4) & 15]), r[(k + 8) & 15]);
                const int mx = max(max(b4[k], b4[(k + 4) & 15]), r[(k + 8) & 15]);
                s = max(s, max(mn - c - 1, c - mx - 1));
            }
        }
        const long long p = (long long)v * W + u;
        const float d = depth[p];
        const bool valid = (d >= dmin) && (d <= dmax);  // false for NaN and +-inf (finite bounds)
        if (score_out) score_out[p] = (short)s;
        key[p] = valid ? (short)s : (short)-1;
        if (valid && s >= 0) atomicAdd(&lh[s], 1);
    }
    __syncthreads();
    if (lh[tid]) atomicAdd(&hist[tid], lh[tid]);
}

// res = (threshold, count): count(t) = sum of hist[s >= t] by a suffix scan;
// the threshold is the smallest t with count(t) <= cap (hist[255] is always
// 0, as scores never exceed 254, so t = 255 always qualifies).
__global__ __launch_bounds__(256) void select_threshold_kernel(const int *hist, int cap, int *res)
{
    __shared__ int cnt[256];
    __shared__ int best;
    const int t = threadIdx.x;
    cnt[t] = hist[t];
    if (t == 0) best = 255;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int add = (t + off < 256) ? cnt[t + off] : 0;
        __syncthreads();
        cnt[t] += add;
        __syncthreads();
    }
    if (cnt[t] <= cap) atomicMin(&best, t);
    __syncthreads();
    if (t == 0) {
        res[0] = best;
        res[1] = cnt[best];
    }
}

__global__ __launch_bounds__(kSelThreads) void select_count_kernel(const short *key, long long npix, const int *res,
                                                                   int *bcount)
{
    const long long p = (long long)blockIdx.x * kSelThreads + threadIdx.x;
    const int t = res[0];
    const int n = __syncthreads_count(p < npix && key[p] >= t);
    if (threadIdx.x == 0) bcount[blockIdx.x] = n;
}

// Row r of the output takes the r-th selected pixel in raster order:
// z = depth, x = (u - cx) z / fx, y = (v - cy) z / fy, each operation a
// rounded IEEE double (no contraction), then rounded to FP32; the feature row
// is copied unchanged.
__global__ __launch_bounds__(kSelThreads) void select_emit_kernel(const short *key, const float *depth,
                                                                  const float *feat, long long npix, int W, int D,
                                                                  double fx, double fy, double cx, double cy,
                                                                  const int *res, const int *boff, float *xyz,
                                                                  float *fout)
{
#pragma clang fp contract(off)
    __shared__ int wsum[kSelThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long p = (long long)blockIdx.x * kSelThreads + threadIdx.x;
    const int t = res[0];
    const bool sel = p < npix && key[p] >= t;
    const unsigned long long m = __ballot(sel);
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    if (!sel) return;
    long long r = boff[blockIdx.x] + __popcll(m & ((1ULL << lane) - 1ULL));
    for (int w = 0; w < wv; ++w) r += wsum[w];
    const int u = (int)(p % W), v = (int)(p / W);
    const float zf = depth[p];
    const double z = (double)zf;
    xyz[3 * r + 0] = (float)((((double)u - cx) * z) / fx);
    xyz[3 * r + 1] = (float)((((double)v - cy) * z) / fy);
    xyz[3 * r + 2] = zf;
    for (int k = 0; k < D; ++k) fout[r * D + k] = feat[p * D + k];
}

void launch_select(const SelectArgs &a, hipStream_t s)
{
    const long long npix = (long long)a.W * a.H;
    hipLaunchKernelGGL(fast_score_kernel, dim3((a.W + kTX - 1) / kTX, (a.H + kTY - 1) / kTY), dim3(kTX, kTY), 0, s,
                       a.gray, a.depth, a.W, a.H, a.dmin, a.dmax, a.key, a.score, a.hist);
    hipLaunchKernelGGL(select_threshold_kernel, dim3(1), dim3(256), 0, s, a.hist, a.cap, a.res);
    const int nb = (int)((npix + kSelThreads - 1) / kSelThreads);
    hipLaunchKernelGGL(select_count_kernel, dim3(nb), dim3(kSelThreads), 0, s, a.key, npix, a.res, a.bcount);
    launch_exclusive_scan(a.bcount, a.boff, a.bsum, nb, nullptr, s);
    hipLaunchKernelGGL(select_emit_kernel, dim3(nb), dim3(kSelThreads), 0, s, a.key, a.depth, a.feat, npix, a.W, a.D,
                       a.fx, a.fy, a.cx, a.cy, a.res, a.boff, a.xyz, a.fout);
}

int select_blocks(long long npix) { return (int)((npix + kSelThreads - 1) / kSelThreads); }

}  // namespace cvo
