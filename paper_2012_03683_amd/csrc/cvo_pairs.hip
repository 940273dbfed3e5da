// cvo_pairs.hip -- the pair pass: the truncated double sum of eq. (7) and its
// per-query moments, for one or many point-cloud pairs in one launch.
//
// Work decomposition (one 64-wide wavefront per piece: every np-th chunk of
// 64 candidates of one query cluster, np set per cluster at planning time):
//   * The cluster's n <= 64 query points are transformed into the reference
//     frame once (FP64), then re-expressed relative to the transformed
//     cluster centre c' and scaled by sqrt(a), a = log2(e) / (2 ell^2), in
//     FP32.  Relative coordinates are small, so FP32 keeps ~1e-7 of the
//     cutoff radius even at 40 m from the origin.
//   * Lanes are split into SUB = 64 / n' sub-streams (n' = n rounded up to a
//     power of two); lane (q, t) pairs query t with every SUB-th candidate, so
//     all 64 lanes stay busy for clusters of any size.
//   * Candidates are the reference points in the grid cells overlapping the
//     box around the ball of radius r_c + rho (rho: cluster radius).  The
//     box's x-runs of cells are contiguous in the sorted reference array; up
//     to 64 runs are measured at once (one per lane), prefix-summed, and
//     their points loaded 64 at a time (each position finds its run by a
//     running max over the runs' first positions; both scans use DPP, not
//     the LDS, which the other waves' walks keep busy).  Points outside the
//     ball are culled; survivors (coordinates and feature rows) are compacted
//     with a ballot into a per-wave LDS queue.
//   * When the queue holds at least kQueueFlush entries every lane walks its
//     share: FP32 squared distance, cutoff test, one exp2 for the geometric
//     kernel and every SE feature block together, the LIN dot product; W =
//     sum w and D = sum w d are summed in FP32 over the flush and then added
//     in FP64, S = sum w d d^T is summed in FP32.
//   * Pairs whose FP32 squared distance lies within a proven error band of
//     the cutoff are decided again with the FP64 expression that defines the
//     pair set, so |P| is exact.
//   * The sub-streams are combined with lane shuffles (fixed order, so the
//     result is bitwise reproducible) and one lane per query writes its
//     moments.
#include "cvo_launch.hpp"

#include <algorithm>

namespace cvo {

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Inclusive scans over the 64 lanes of a wave with DPP row shifts and row
// broadcasts (no LDS traffic): within each row of 16 lanes a Hillis-Steele
// scan over shifts 1, 2, 4, 8 (lanes shifted in from outside the row add
// the identity 0), then row 0's last lane is added to row 1 and row 2's to
// row 3, then lane 31 to rows 2 and 3.  The max scan needs values >= 0.
__device__ __forceinline__ int wave_scan_add(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ int wave_scan_max(int v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
    return v;
}

// Wave-uniform floating values kept in scalar registers.
__device__ __forceinline__ float uniform_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ double uniform_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Membership of (x, z) in the pair set, decided exactly as the set is defined:
// z'_r = ((R_r0 z0 + R_r1 z1) + R_r2 z2) + t_r, d = x - z',
// s = (dx dx + dy dy) + dz dz, member iff s <= rc2; every operation is a
// separately rounded IEEE double (contraction into FMA is switched off).
__device__ __noinline__ bool canonical_member(const double *T, float x0, float x1, float x2, float z0,
                                              float z1, float z2, double rc2)
{
#pragma clang fp contract(off)
    const double a0 = (double)z0, a1 = (double)z1, a2 = (double)z2;
    double zt[3];
    for (int r = 0; r < 3; ++r) {
        const double p = T[4 * r + 0] * a0;
        const double q = T[4 * r + 1] * a1;
        const double u = T[4 * r + 2] * a2;
        zt[r] = ((p + q) + u) + T[4 * r + 3];
    }
    const double dx = (double)x0 - zt[0];
    const double dy = (double)x1 - zt[1];
    const double dz = (double)x2 - zt[2];
    const double s = (dx * dx + dy * dy) + dz * dz;
    return s <= rc2;
}

// Cells [i0, i1] along one axis covering [c - R, c + R]; false if none.
// Uses the same floor((p - o) * inv_h) as the binning.
__device__ __forceinline__ bool axis_range(double c, double R, double o, double inv_h, int n, int &i0, int &i1)
{
    const double f0 = floor(((c - R) - o) * inv_h);
    const double f1 = floor(((c + R) - o) * inv_h);
    if (!(f1 >= 0.0) || !(f0 <= (double)(n - 1))) return false;
    i0 = (int)fmax(f0, 0.0);
    i1 = (int)fmin(f1, (double)(n - 1));
    return true;
}

// Geometry shared by the planner and the pass: the cluster centre in the
// reference frame, the cull radius, and the cell ranges of its neighbourhood.
struct Neighbourhood {
    double cx, cy, cz, Rm;
    int ix0, ix1, iy0, iy1, iz0, iz1;
    bool any;
};

__device__ __forceinline__ Neighbourhood neighbourhood(const double *Pm, const double4 g, double rc, bool cut,
                                                       const GridDesc &gd)
{
    Neighbourhood nb;
    nb.cx = Pm[0] * g.x + Pm[1] * g.y + Pm[2] * g.z + Pm[3];
    nb.cy = Pm[4] * g.x + Pm[5] * g.y + Pm[6] * g.z + Pm[7];
    nb.cz = Pm[8] * g.x + Pm[9] * g.y + Pm[10] * g.z + Pm[11];
    nb.Rm = cut ? (rc + g.w) * (1.0 + 1e-5) : INFINITY;
    nb.ix0 = 0; nb.ix1 = gd.nx - 1; nb.iy0 = 0; nb.iy1 = gd.ny - 1; nb.iz0 = 0; nb.iz1 = gd.nz - 1;
    nb.any = gd.n > 0;
    if (cut && nb.any)
        nb.any = axis_range(nb.cx, nb.Rm, gd.ox, gd.inv_h, gd.nx, nb.ix0, nb.ix1) &&
                 axis_range(nb.cy, nb.Rm, gd.oy, gd.inv_h, gd.ny, nb.iy0, nb.iy1) &&
                 axis_range(nb.cz, nb.Rm, gd.oz, gd.inv_h, gd.nz, nb.iz0, nb.iz1);
    return nb;
}


template <int SED, int LIND, int MODE> struct PassTraits {
    static constexpr int D = SED + LIND;
    static constexpr int D4 = (D + 3) & ~3;
    // waves per SIMD the register budget is sized for (no spills)
    static constexpr int kMinWaves = (MODE == 0 && D4 <= 24) ? 4 : 2;
};

template <int SED, int LIND, int MODE>
__global__ __launch_bounds__(kWave * kWavesPerBlock, (PassTraits<SED, LIND, MODE>::kMinWaves))
void pair_pass_kernel(const PairPassArgs a)
{
    constexpr int D = SED + LIND;
    constexpr int D4 = (D + 3) & ~3;
    constexpr int F4 = D4 / 4;
    constexpr int F4s = F4 > 0 ? F4 : 1;
    constexpr int VF = D4 > 0 ? D4 : 1;
    // candidate queue, one entry of E4 float4s per candidate: (scaled
    // coordinates relative to the cluster centre, source index bits), then
    // the feature row
    constexpr int E4 = 1 + F4;
    __shared__ float4 s_q[kWavesPerBlock][kQueueCap * E4];
    __shared__ int s_rs[kWavesPerBlock][kWave];
    __shared__ int s_rx[kWavesPerBlock][kWave];
    __shared__ int s_row[kWavesPerBlock][kWave];

    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const unsigned long long lt_mask = (lane == 0) ? 0ULL : (~0ULL >> (64 - lane));
    const float sig2 = a.sig2;
    const bool cut = isfinite(a.kappa);

    // one piece per wave; pieces are ordered heaviest first, so the largest
    // pieces are dispatched first and the light ones fill in behind them
    {
        // The prologue's loads are requested in two dependent rounds: the
        // piece record (its index clamped, so the load stays in bounds before
        // the range check), then together the pair's flags, pose, lengthscale
        // and grid.  The query row follows the exit test of finished pairs, in
        // the round of the first cell-table reads.
        const int tk = wave_uniform(blockIdx.x * kWavesPerBlock + wv);
        const int npieces = a.npieces;
        const PieceRec rec = a.recs[min(tk, npieces - 1)];
        const int4 pc = rec.pc;
        const int b = wave_uniform(rec.b);
        const PairState *st = a.state + b;
        const double *P = a.pose_is_inverse ? st->Tinv : st->T;
        double Pm[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) Pm[k] = P[k];
        const double ell = st->ell;
        const int2 cl = make_int2(rec.first, rec.n);
        const double4 g = rec.geo;
        const GridDesc gd = a.grids[b];
        __builtin_amdgcn_sched_barrier(0);  // (the exit test below must not be scheduled between these loads)
        const int skip = st->done | st->pause;

#pragma unroll
        for (int k = 0; k < 12; ++k) in_sgpr(Pm[k]);
        in_sgpr(ell);
        in_sgpr(pc.y), in_sgpr(pc.z), in_sgpr(pc.w);
        in_sgpr(cl.x), in_sgpr(cl.y);
        in_sgpr(g.x), in_sgpr(g.y), in_sgpr(g.z), in_sgpr(g.w);
        in_sgpr(gd.ox), in_sgpr(gd.oy), in_sgpr(gd.oz), in_sgpr(gd.inv_h);
        in_sgpr(gd.nx), in_sgpr(gd.ny), in_sgpr(gd.nz), in_sgpr(gd.cell_base), in_sgpr(gd.n);
        in_sgpr(a.kappa);
        in_sgpr((long long)a.qpts), in_sgpr((long long)a.qfeat);
        if (tk >= npieces || skip) return;

        // query point owned by this lane; SUB sub-streams share the candidates
        const int n = cl.y;
        const int np2 = (n <= 1) ? 1 : (1 << (32 - __clz(n - 1)));
        const int lg = __ffs(np2) - 1;
        const int t = lane & (np2 - 1);
        const int qs = lane >> lg;
        const int SUB = kWave >> lg;
        const bool active = t < n;
        const int pq = cl.x + (active ? t : 0);
        const float4 zq = a.qpts[pq];  // (reloaded on the rare exact-recheck path)
        float vf[VF];
#pragma unroll
        for (int f = 0; f < VF / 4; ++f) vf[4 * f] = vf[4 * f + 1] = vf[4 * f + 2] = vf[4 * f + 3] = 0.0f;
#pragma unroll
        for (int f = 0; f < F4; ++f) {
            const float4 v4 = reinterpret_cast<const float4 *>(a.qfeat)[(long long)pq * F4 + f];
            vf[4 * f + 0] = v4.x;
            vf[4 * f + 1] = v4.y;
            vf[4 * f + 2] = v4.z;
            vf[4 * f + 3] = v4.w;
        }

        const double ascale = 1.4426950408889634 / (2.0 * ell * ell);  // log2(e) / (2 ell^2)
        const double sc = uniform_d(sqrt(ascale));
        const double rc = a.kappa * ell;
        const double rc2 = rc * rc;
        const Neighbourhood nb = neighbourhood(Pm, g, rc, cut, gd);
        const double cx = uniform_d(nb.cx), cy = uniform_d(nb.cy), cz = uniform_d(nb.cz);

        // thresholds in scaled units: s' <= lo is certainly in P, s' > hi is
        // certainly out; between them the FP64 definition decides.  The band
        // is 8x the worst-case FP32 error 2^-24 (4 (1 + rho/rc) + 3) a rc^2
        // plus the rounding of the thresholds themselves.
        float hi = INFINITY, lo = INFINITY, cull2 = INFINITY;
        if (cut) {
            const double u = 5.9604644775390625e-8;
            const double G = u * (8.0 * (4.0 * (1.0 + g.w / rc) + 3.0) + 4.0);
            const double r2s = rc2 * ascale;
            hi = uniform_f((float)(r2s * (1.0 + G)));
            lo = uniform_f((float)(r2s * (1.0 - G)));
            cull2 = uniform_f((float)(nb.Rm * nb.Rm * ascale));
        }

        const double zpx = Pm[0] * zq.x + Pm[1] * zq.y + Pm[2] * zq.z + Pm[3];
        const double zpy = Pm[4] * zq.x + Pm[5] * zq.y + Pm[6] * zq.z + Pm[7];
        const double zpz = Pm[8] * zq.x + Pm[9] * zq.y + Pm[10] * zq.z + Pm[11];
        const float zrx = (float)((zpx - cx) * sc);
        const float zry = (float)((zpy - cy) * sc);
        const float zrz = (float)((zpz - cz) * sc);

        double W = 0.0, Dx = 0.0, Dy = 0.0, Dz = 0.0;
        float S00 = 0.f, S01 = 0.f, S02 = 0.f, S11 = 0.f, S12 = 0.f, S22 = 0.f;
        int cnt = 0;
        double Gf[MODE == 1 ? VF : 1];
        double Ls = 0.0;
#pragma unroll
        for (int k = 0; k < (MODE == 1 ? VF : 1); ++k) Gf[k] = 0.0;

        // W and D are summed in FP32 over one queue flush (at most kQueueCap
        // terms per lane) and added to the FP64 accumulators after it.
        float w32 = 0.f, dx32 = 0.f, dy32 = 0.f, dz32 = 0.f;
        // one candidate entry (at `ent`; its offset d from the query and
        // squared distance s already taken) against this lane's query;
        // `valid` false only in the tail of a flush, for lanes past its end
        auto pair_term = [&](float dx, float dy, float dz, float s, const float4 *ent, bool valid) {
            if (valid && active && s <= hi) {
                bool pass = true;
                if (s > lo) {
                    const float4 rp = a.rpts[__float_as_int(ent[0].w)];
                    const float4 zq2 = a.qpts[pq];
                    pass = a.pose_is_inverse
                               ? canonical_member(st->T, zq2.x, zq2.y, zq2.z, rp.x, rp.y, rp.z, rc2)
                               : canonical_member(st->T, rp.x, rp.y, rp.z, zq2.x, zq2.y, zq2.z, rc2);
                }
                if (pass) {
                    float E = s;
                    float lin = 0.0f, lin1 = 0.0f;  // even / odd LIN columns: two shorter FMA chains
#pragma unroll
                    for (int f = 0; f < F4; ++f) {
                        const float4 u4 = ent[1 + f];
                        const float uu[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int d = 4 * f + q;
                            if (d < SED) {
                                const float df = uu[q] - vf[d];
                                E = fmaf(df, df, E);
                            } else if (d < D) {
                                if ((d - SED) & 1) lin1 = fmaf(uu[q], vf[d], lin1);
                                else lin = fmaf(uu[q], vf[d], lin);
                            }
                        }
                    }
                    lin += lin1;
                    // sigma^2 prod sigma_b^2 is applied once per query at the end
                    const float wnl = __builtin_amdgcn_exp2f(-E);
                    const float w = (LIND > 0) ? wnl * lin : wnl;
                    w32 += w;
                    const float wx = w * dx, wy = w * dy, wz = w * dz;
                    dx32 += wx;
                    dy32 += wy;
                    dz32 += wz;
                    cnt += 1;
                    if (MODE == 0) {
                        S00 = fmaf(wx, dx, S00);
                        S01 = fmaf(wx, dy, S01);
                        S02 = fmaf(wx, dz, S02);
                        S11 = fmaf(wy, dy, S11);
                        S12 = fmaf(wy, dz, S12);
                        S22 = fmaf(wz, dz, S22);
                    } else {
                        Ls += (double)(w * s);
#pragma unroll
                        for (int f = 0; f < F4; ++f) {
                            const float4 u4 = ent[1 + f];
                            const float uu[4] = {u4.x, u4.y, u4.z, u4.w};
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                const int d = 4 * f + q;
                                if (MODE == 1 && d < SED) Gf[d] += (double)(w * (uu[q] - vf[d]));
                                else if (MODE == 1 && d < D) Gf[d] += (double)(wnl * uu[q]);
                            }
                        }
                    }
                }
            }
        };
        // Lane (q, t) walks entries q, q + SUB, ...: first the rows of SUB
        // entries that every sub-stream has (a wave-uniform loop, the next
        // entry's coordinates read while this one is used), then the last,
        // partial row.
        auto process = [&](int qn_) {
            w32 = 0.f, dx32 = 0.f, dy32 = 0.f, dz32 = 0.f;
            const int qn = wave_uniform(qn_);
            const int nfull = wave_uniform(qn >> (6 - lg));  // qn / SUB
            const float4 *ent = &s_q[wv][qs * E4];
            const int step = SUB * E4;
            float4 e = ent[0];
            for (int it = 0; it < nfull; ++it) {
                const float dx = e.x - zrx, dy = e.y - zry, dz = e.z - zrz;
                const float s = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                const float4 *cur = ent;
                ent += (it + 1 < nfull) ? step : 0;  // (the last row re-reads itself)
                e = *ent;
                pair_term(dx, dy, dz, s, cur, true);
            }
            const int done = wave_uniform(nfull << (6 - lg));
            if (done < qn) {
                const int kt = qs + done;
                const bool in = kt < qn;
                const float4 *tl = &s_q[wv][(in ? kt : 0) * E4];
                const float4 c = *tl;
                const float dx = c.x - zrx, dy = c.y - zry, dz = c.z - zrz;
                const float s = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                pair_term(dx, dy, dz, s, tl, in);
            }
            W += (double)w32;
            Dx += (double)dx32;
            Dy += (double)dy32;
            Dz += (double)dz32;
        };

        // this piece takes chunks pidx, pidx + np, pidx + 2 np, ... of the
        // cluster's candidates (the neighbourhood rows concatenated; chunk k =
        // candidates [64 k, 64 k + 64)), so the np pieces of a cluster sample
        // its whole neighbourhood alike and together cover it at any pose
        const int pidx = pc.y, pstride = pc.z;
        int qn = 0;
        if (nb.any) {
            const int nyr = nb.iy1 - nb.iy0 + 1;
            const int nrows = nyr * (nb.iz1 - nb.iz0 + 1);
            const int run = nb.ix1 - nb.ix0 + 1;
            int base = 0;  // candidates in earlier row batches
            for (int rb = 0; rb < nrows; rb += kWave) {
                const int r = rb + lane;
                int rs = 0, len = 0;
                if (r < nrows) {
                    const int iy = nb.iy0 + r % nyr, iz = nb.iz0 + r / nyr;
                    const long long k0 =
                        (long long)gd.cell_base + nb.ix0 + (long long)gd.nx * (iy + (long long)gd.ny * iz);
                    rs = a.cell_start[k0];
                    len = a.cell_start[k0 + run] - rs;
                }
                const int incl = wave_scan_add(len);
                const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
                // first chunk of this piece reaching into [base, base + total)
                int k = base / kWave;
                k += ((pidx - k) % pstride + pstride) % pstride;
                if (k * kWave < base + total) {
                    s_rs[wv][lane] = rs;
                    s_rx[wv][lane] = incl - len;
                    s_row[wv][lane] = 0;  // marks left by earlier chunks of this batch never exceed a later chunk's rows
                    wave_sync();
                    for (; k * kWave < base + total; k += pstride) {
                        // the part of chunk k inside this batch of rows
                        const int m = k * kWave - base + lane;
                        bool keep = false;
                        int src = 0;
                        float x0 = 0.f, x1 = 0.f, x2 = 0.f;
                        // the row (cell run) of each position of the chunk: every
                        // non-empty row reaching into the chunk marks its first
                        // position in it with its index, and a running max over
                        // the positions (on all lanes, before the branch below)
                        // fills in the rest
                        {
                            const int c0 = k * kWave - base;
                            const int rx = incl - len;
                            if (len > 0 && rx < c0 + kWave && rx + len > c0) s_row[wv][max(rx - c0, 0)] = lane;
                        }
                        wave_sync();
                        const int row_ = wave_scan_max(s_row[wv][lane]);
                        if (m >= 0 && m < total) {
                            src = s_rs[wv][row_] + (m - s_rx[wv][row_]);
                            const float4 xp = a.rpts[src];
                            x0 = (float)(((double)xp.x - cx) * sc);
                            x1 = (float)(((double)xp.y - cy) * sc);
                            x2 = (float)(((double)xp.z - cz) * sc);
                            keep = fmaf(x2, x2, fmaf(x1, x1, x0 * x0)) <= cull2;
                        }
                        const unsigned long long mask = __ballot(keep);
                        if (keep) {
                            const int slot = qn + __popcll(mask & lt_mask);
                            s_q[wv][slot * E4] = make_float4(x0, x1, x2, __int_as_float(src));
                            const float4 *fr = reinterpret_cast<const float4 *>(a.rfeat) + (long long)src * F4;
#pragma unroll
                            for (int f = 0; f < F4; ++f) s_q[wv][slot * E4 + 1 + f] = fr[f];
                        }
                        qn += __popcll(mask);
                        wave_sync();
                        if (qn >= kQueueFlush) {
                            process(qn);
                            qn = 0;
                            wave_sync();
                        }
                    }
                    wave_sync();
                }
                base += total;
            }
        }
        process(qn);
        wave_sync();

        // combine the sub-streams of each query (fixed shuffle order)
        for (int off = np2; off < kWave; off <<= 1) {
            W += __shfl_xor(W, off);
            Dx += __shfl_xor(Dx, off);
            Dy += __shfl_xor(Dy, off);
            Dz += __shfl_xor(Dz, off);
            cnt += __shfl_xor(cnt, off);
            if (MODE == 0) {
                S00 += __shfl_xor(S00, off);
                S01 += __shfl_xor(S01, off);
                S02 += __shfl_xor(S02, off);
                S11 += __shfl_xor(S11, off);
                S12 += __shfl_xor(S12, off);
                S22 += __shfl_xor(S22, off);
            } else {
                Ls += __shfl_xor(Ls, off);
#pragma unroll
                for (int k = 0; k < (MODE == 1 ? VF : 1); ++k) Gf[k] += __shfl_xor(Gf[k], off);
            }
        }
        if (qs == 0 && active) {
            const long long o = (long long)pc.w + t;
            const double sg = (double)sig2;  // every output is linear in the kernel weights
            a.oW[o] = sg * W;
            a.oD[3 * o + 0] = sg * Dx;
            a.oD[3 * o + 1] = sg * Dy;
            a.oD[3 * o + 2] = sg * Dz;
            a.oCnt[o] = cnt;
            if (MODE == 0) {
                float *S = a.oS + 6 * o;
                S[0] = sig2 * S00; S[1] = sig2 * S01; S[2] = sig2 * S02;
                S[3] = sig2 * S11; S[4] = sig2 * S12; S[5] = sig2 * S22;
            } else {
                a.oL[o] = sg * Ls;
#pragma unroll
                for (int k = 0; k < (MODE == 1 ? D4 : 0); ++k) a.oG[o * D4 + k] = sg * Gf[k];
            }
        }
    }
}

// ---------------------------------------------------------------- planning
// Per cluster, at the current pose: the number of candidates of its
// neighbourhood and how many pieces to cut it into (work per piece about
// `work` query-candidate products, at least 512 candidates per piece).
__global__ void plan_count(const PairPassArgs a, int work, int *npieces, int *cmax, long long *ccount)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.nclus; c += gridDim.x * blockDim.x) {
        const int b = a.cpair[c];
        const PairState *st = a.state + b;
        const double *P = a.pose_is_inverse ? st->Tinv : st->T;
        double Pm[12];
        for (int k = 0; k < 12; ++k) Pm[k] = P[k];
        const bool cut = isfinite(a.kappa);
        const double rc = a.kappa * st->ell;
        const GridDesc gd = a.grids[b];
        const Neighbourhood nb = neighbourhood(Pm, a.cgeo[c], rc, cut, gd);
        long long C = 0;
        if (nb.any) {
            const int run = nb.ix1 - nb.ix0 + 1;
            for (int iz = nb.iz0; iz <= nb.iz1; ++iz)
                for (int iy = nb.iy0; iy <= nb.iy1; ++iy) {
                    const long long k0 =
                        (long long)gd.cell_base + nb.ix0 + (long long)gd.nx * (iy + (long long)gd.ny * iz);
                    C += a.cell_start[k0 + run] - a.cell_start[k0];
                }
        }
        const int n = a.clus[c].y;
        const int cm = max(512, work / max(n, 1));
        const long long np = C > 0 ? (C + cm - 1) / cm : 1;
        npieces[c] = (int)min(np, 4096LL);
        cmax[c] = cm;
        ccount[c] = C;
    }
}

// A piece's cost on 16 bits, non-decreasing in the cost: exact below 49152
// (every piece of the default plan: n <= 64 queries x at most 576), then
// 1024 steps per doubling.
constexpr unsigned long long kCostLinear = 49152;
__device__ __forceinline__ unsigned int piece_cost_code(unsigned long long cost)
{
    if (cost < kCostLinear) return (unsigned int)cost;
    const double q = (log2((double)cost) - log2((double)kCostLinear)) * 1024.0;
    return (unsigned int)min((double)kCostLinear + floor(q), 65535.0);
}

// Emit the pieces of each cluster (cluster-major) as (cluster, p, np), their
// query counts (for the output-slot scan) and a sort key: the heaviest piece
// gets the smallest key; the stable sort keeps a cluster's pieces together.
__global__ void plan_emit(const PairPassArgs a, const int *npieces, const int *pbase, const long long *ccount,
                          int4 *pieces, int *pn, unsigned long long *key, int *val, int2 *cpieces)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.nclus; c += gridDim.x * blockDim.x) {
        const int np = npieces[c], pb = pbase[c];
        const int n = a.clus[c].y;
        const long long C = ccount[c];
        cpieces[c] = make_int2(pb, np);
        const long long cand = (C + np - 1) / np;  // candidates per piece
        for (int p = 0; p < np; ++p) {
            pieces[pb + p] = make_int4(c, p, np, 0);
            pn[pb + p] = n;
            const unsigned long long cost = (unsigned long long)n * (unsigned long long)(cand + 64);
            key[pb + p] = 0xffffULL - (unsigned long long)piece_cost_code(cost);  // 16-bit key
            val[pb + p] = pb + p;
        }
    }
}

__global__ void plan_slots(int4 *pieces, const int *tbase, int npieces)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npieces; i += gridDim.x * blockDim.x)
        pieces[i].w = tbase[i];
}

__global__ void plan_qmap(const int2 *clus, const int2 *cpieces, const int4 *pieces, int nclus, int4 *qmap)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nclus; c += gridDim.x * blockDim.x) {
        const int2 cl = clus[c];
        const int2 cp = cpieces[c];
        const int slot0 = pieces[cp.x].w;
        for (int t = 0; t < cl.y; ++t) qmap[cl.x + t] = make_int4(t, cl.y, cp.y, slot0 + t);
    }
}

void launch_plan_qmap(const int2 *clus, const int2 *cpieces, const int4 *pieces, int nclus, int4 *qmap,
                      hipStream_t s)
{
    const int nb = std::max(1, std::min(4096, (nclus + 255) / 256));
    hipLaunchKernelGGL(plan_qmap, dim3(nb), dim3(256), 0, s, clus, cpieces, pieces, nclus, qmap);
}

__global__ void plan_records(const int *porder, const int4 *pieces, const int *cpair, const int2 *clus,
                             const double4 *cgeo, int npieces, PieceRec *recs)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npieces; i += gridDim.x * blockDim.x) {
        const int4 pc = pieces[porder[i]];
        const int2 cl = clus[pc.x];
        PieceRec r;
        r.pc = pc;
        r.b = cpair[pc.x];
        r.first = cl.x;
        r.n = cl.y;
        r.pad = 0;
        r.geo = cgeo[pc.x];
        recs[i] = r;
    }
}

void launch_plan_records(const int *porder, const int4 *pieces, const int *cpair, const int2 *clus,
                         const double4 *cgeo, int npieces, PieceRec *recs, hipStream_t s)
{
    if (npieces <= 0) return;
    const int nb = std::max(1, std::min(4096, (npieces + 255) / 256));
    hipLaunchKernelGGL(plan_records, dim3(nb), dim3(256), 0, s, porder, pieces, cpair, clus, cgeo, npieces, recs);
}

void launch_plan_count(const PairPassArgs &a, int work, int *npieces, int *cmax, long long *ccount, hipStream_t s)
{
    const int nb = std::max(1, std::min(4096, (a.nclus + 255) / 256));
    hipLaunchKernelGGL(plan_count, dim3(nb), dim3(256), 0, s, a, work, npieces, cmax, ccount);
}

void launch_plan_emit(const PairPassArgs &a, const int *npieces, const int *pbase, const long long *ccount,
                      int4 *pieces, int *pn, unsigned long long *key, int *val, int2 *cpieces, hipStream_t s)
{
    const int nb = std::max(1, std::min(4096, (a.nclus + 255) / 256));
    hipLaunchKernelGGL(plan_emit, dim3(nb), dim3(256), 0, s, a, npieces, pbase, ccount, pieces, pn, key, val,
                       cpieces);
}

void launch_plan_slots(int4 *pieces, const int *tbase, int npieces, hipStream_t s)
{
    const int nb = std::max(1, std::min(4096, (npieces + 255) / 256));
    hipLaunchKernelGGL(plan_slots, dim3(nb), dim3(256), 0, s, pieces, tbase, npieces);
}

// ---------------------------------------------------------------- dispatch
// Compiled feature layouts (SE columns, LIN columns); other layouts are
// padded with zero columns up to the nearest compiled one.
#define CVO_LAYOUTS(X)                                                                                     \
    X(0, 0) X(0, 4) X(0, 19) X(0, 32) X(0, 64) X(5, 0) X(5, 4) X(5, 19) X(5, 32) X(8, 0) X(8, 4) X(8, 19)    \
        X(8, 32) X(16, 0) X(16, 19) X(16, 32) X(32, 0) X(32, 19) X(32, 32)

bool pair_layout_supported(int sed, int lind)
{
#define CVO_CHECK(S, L) if (sed == S && lind == L) return true;
    CVO_LAYOUTS(CVO_CHECK)
#undef CVO_CHECK
    return false;
}

template <int S, int L, int MODE>
static void launch_one(const PairPassArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((pair_pass_kernel<S, L, MODE>), dim3((a.npieces + kWavesPerBlock - 1) / kWavesPerBlock),
                       dim3(kWave * kWavesPerBlock), 0, s, a);
}

bool launch_pair_pass(const PairPassArgs &a, const FeatLayout &lay, int mode, hipStream_t s)
{
    if (a.npieces <= 0) return true;
#define CVO_LAUNCH(S, L)                                          \
    if (lay.sed == S && lay.lind == L) {                          \
        if (mode == 0) launch_one<S, L, 0>(a, s);                 \
        else launch_one<S, L, 1>(a, s);                           \
        return true;                                              \
    }
    CVO_LAYOUTS(CVO_LAUNCH)
#undef CVO_LAUNCH
    return false;
}

}  // namespace cvo

