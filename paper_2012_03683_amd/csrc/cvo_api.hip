// cvo_api.hip -- host side of the library: the handle, its scratch arena,
// preparation of the two cloud views, and the C ABI of include/cvo.h.
//
// Every call runs entirely on the GPU in the kernels of cvo_build.hip,
// cvo_pairs.hip and cvo_reduce.hip; the host only validates arguments,
// sizes buffers, launches, and copies small results back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "cvo.h"
#include "cvo_launch.hpp"

namespace cvo {
bool pair_layout_supported(int sed, int lind);
}

using namespace cvo;

namespace {

struct CvoError : std::runtime_error {
    cvo_status code;
    CvoError(cvo_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                                                    \
    do {                                                                                                \
        hipError_t e_ = (expr);                                                                         \
        if (e_ != hipSuccess)                                                                           \
            throw CvoError(e_ == hipErrorOutOfMemory ? CVO_ERR_OUT_OF_MEMORY : CVO_ERR_DEVICE,          \
                           std::string(#expr) + ": " + hipGetErrorString(e_));                          \
    } while (0)

inline void require(bool ok, const std::string &msg)
{
    if (!ok) throw CvoError(CVO_ERR_INVALID_ARGUMENT, msg);
}

constexpr double kLog2e = 1.4426950408889634;

}  // namespace

// ------------------------------------------------------------------ fixed scratch
// Device scratch of the allocation-free entry point (cvo_evaluate_noalloc):
// one copy of this array per device, held from the library's load until the
// process ends.  Host code never uses the name itself (on the host it is
// only a stand-in, not a device address): cvo_create looks up each device's
// address once with hipGetSymbolAddress and every kernel gets that address.
static __device__ __align__(256) unsigned char scratch[(size_t)CVO_NOALLOC_SCRATCH_MIB << 20];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;  // device ordinal -> that device's copy of `scratch`

// With `device` current: the device address of its copy of the array,
// looked up on the first call for the device.
hipError_t scratch_address(int device, void **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it != g_scratch_addr.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
    *out = ptr;
    return hipSuccess;
}
}  // namespace

// ------------------------------------------------------------------ handle
struct cvo_context {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    struct Buf {
        void *p = nullptr;
        size_t cap = 0;
    };
    std::map<std::string, Buf> bufs;
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    cvo_tuning tuning{16, 1.0, 0.5, 0.6, 16, 512, CVO_CLUSTER_OCTREE, 1};
    bool profiling = false;
    cvo_timing timing{0, 0.0, 0, 0, 0, 0, 0, 0};
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pending;
    std::map<std::string, cvo_tuning> tune_cache;
    // autotuned view shape per (feature rows of at most 8 floats?, density
    // class); consulted before the built-in table by adaptive registrations
    struct Shape {
        int32_t cluster_max;
        double cell_factor, cluster_factor;
        int32_t rule;
    };
    std::map<std::pair<int, int>, Shape> class_shape;
    // captured batched graph, and the library-owned stream it is captured on
    // (the legacy default stream cannot be captured)
    hipGraphExec_t graph = nullptr;
    std::string graph_key;
    hipStream_t own_stream = nullptr;

    // Allocation-free mode: buffers are carved from a fixed device array
    // (base, cap) by a bump pointer that restarts with every call; a name
    // asked for again within the call gets its earlier region back when it
    // fits, as the arena below hands back the same buffer.
    struct Fixed {
        bool on = false;
        char *base = nullptr;
        size_t cap = 0, top = 0;
        std::map<std::string, std::pair<size_t, size_t>> regions;  // name -> (offset, bytes)
    } fixed;
    std::string fixed_error;  // why the fixed scratch is unavailable, if it is

    void *get(const std::string &name, size_t bytes)
    {
        if (bytes == 0) bytes = 16;
        if (fixed.on) return get_fixed(name, bytes);
        Buf &b = bufs[name];
        if (b.cap < bytes) {
            if (b.p) HIP_OK(hipFree(b.p));
            b.p = nullptr;
            size_t cap = std::max(bytes, b.cap + b.cap / 2);
            cap = (cap + 255) & ~size_t(255);
            hipError_t e = hipMalloc(&b.p, cap);
            if (e != hipSuccess) {
                b.p = nullptr;
                b.cap = 0;
                throw CvoError(CVO_ERR_OUT_OF_MEMORY, "device allocation of " + std::to_string(cap) +
                                                          " bytes for " + name + " failed");
            }
            b.cap = cap;
        }
        return b.p;
    }
    void *get_fixed(const std::string &name, size_t bytes)
    {
        auto it = fixed.regions.find(name);
        if (it != fixed.regions.end() && it->second.second >= bytes) return fixed.base + it->second.first;
        const size_t need = (bytes + 255) & ~size_t(255);
        if (need > fixed.cap - fixed.top)
            throw CvoError(CVO_ERR_OUT_OF_MEMORY,
                           "the allocation-free scratch (" + std::to_string(fixed.cap >> 20) +
                               " MiB per device) is too small for this input: " + name + " needs " +
                               std::to_string(need) + " bytes with " + std::to_string(fixed.cap - fixed.top) +
                               " left");
        const size_t off = fixed.top;
        fixed.top += need;
        fixed.regions[name] = {off, need};
        return fixed.base + off;
    }
    template <class T> T *get_t(const std::string &name, size_t count)
    {
        return static_cast<T *>(get(name, count * sizeof(T)));
    }
    void *host(size_t bytes)
    {
        if (pinned_cap < bytes) {
            if (pinned) HIP_OK(hipHostFree(pinned));
            pinned = nullptr;
            size_t cap = std::max(bytes, size_t(1) << 16);
            HIP_OK(hipHostMalloc(&pinned, cap, hipHostMallocDefault));
            pinned_cap = cap;
        }
        return pinned;
    }
    // Host -> device copies are staged in a pinned ring and not waited for.
    // A ring slot is written again only after the stream that reads it has
    // been synchronised (the ring restarts then), so a pending copy never
    // sees its source change.
    void *ring = nullptr;
    size_t ring_cap = 0, ring_off = 0;
    hipStream_t ring_stream = nullptr;
    void ring_drain()
    {
        if (ring_off) {
            timing.host_waits += 1;
            HIP_OK(hipStreamSynchronize(ring_stream));
            ring_off = 0;
        }
    }
    void upload(void *dst, const void *src, size_t bytes)
    {
        if (!bytes) return;
        if (fixed.on) {
            // no pinned staging: copy from the caller's memory and wait
            HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
            HIP_OK(hipStreamSynchronize(stream));
            return;
        }
        const size_t need = (bytes + 255) & ~size_t(255);
        if (ring_off && (ring_stream != stream || ring_off + need > ring_cap)) ring_drain();
        if (need > ring_cap) {
            if (ring) HIP_OK(hipHostFree(ring));
            ring = nullptr;
            ring_cap = 0;
            const size_t cap = std::max(need, size_t(1) << 20);
            HIP_OK(hipHostMalloc(&ring, cap, hipHostMallocDefault));
            ring_cap = cap;
        }
        char *h = static_cast<char *>(ring) + ring_off;
        std::memcpy(h, src, bytes);
        HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream));
        ring_off += need;
        ring_stream = stream;
    }
    // device -> host, waiting for the stream (which also frees the ring)
    void download(void *dst, const void *src, size_t bytes)
    {
        if (!bytes) return;
        timing.host_waits += 1;
        if (fixed.on) {
            HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
            HIP_OK(hipStreamSynchronize(stream));
            return;
        }
        void *h = host(bytes);
        HIP_OK(hipMemcpyAsync(h, src, bytes, hipMemcpyDeviceToHost, stream));
        HIP_OK(hipStreamSynchronize(stream));
        if (stream == ring_stream) ring_off = 0;
        std::memcpy(dst, h, bytes);
    }
    void check_launch(const char *what)
    {
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) throw CvoError(CVO_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
    hipEvent_t event()
    {
        if (!ev_free.empty()) {
            hipEvent_t e = ev_free.back();
            ev_free.pop_back();
            return e;
        }
        // timing only: no system-scope fence (cache write-back and invalidate)
        // when the event is recorded, so the events neither slow nor pad the
        // kernels they bracket; their times are read after a stream wait
        hipEvent_t e;
        HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
        return e;
    }
    // adds the times of the first `count` pending launches (all by default;
    // their events must have completed)
    void harvest_events(size_t count = SIZE_MAX)
    {
        count = std::min(count, ev_pending.size());
        for (size_t k = 0; k < count; ++k) {
            auto &pr = ev_pending[k];
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, pr.first, pr.second));
            timing.pair_ms += ms;
            timing.pair_launches += 1;
            ev_free.push_back(pr.first);
            ev_free.push_back(pr.second);
        }
        ev_pending.erase(ev_pending.begin(), ev_pending.begin() + (long)count);
    }
    hipStream_t capture_stream()
    {
        if (!own_stream) HIP_OK(hipStreamCreateWithFlags(&own_stream, hipStreamNonBlocking));
        return own_stream;
    }
    void release()
    {
        if (graph) hipGraphExecDestroy(graph);
        graph = nullptr;
        if (own_stream) hipStreamDestroy(own_stream);
        own_stream = nullptr;
        for (auto &kv : bufs)
            if (kv.second.p) hipFree(kv.second.p);
        bufs.clear();
        if (pinned) hipHostFree(pinned);
        pinned = nullptr;
        if (ring) hipHostFree(ring);
        ring = nullptr;
        ring_off = ring_cap = 0;
        for (auto &pr : ev_pending) {
            hipEventDestroy(pr.first);
            hipEventDestroy(pr.second);
        }
        for (auto e : ev_free) hipEventDestroy(e);
        ev_free.clear();
        ev_pending.clear();
    }
};

namespace {

// ------------------------------------------------------------------ validation
void check_pose(const double *T)
{
    require(T != nullptr, "pose pointer is NULL");
    for (int k = 0; k < 12; ++k) require(std::isfinite(T[k]), "pose has a non-finite entry");
    double dev = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += T[4 * k + r] * T[4 * k + c];
            dev = std::max(dev, std::fabs(s - (r == c ? 1.0 : 0.0)));
        }
    const double det = T[0] * (T[5] * T[10] - T[6] * T[9]) - T[1] * (T[4] * T[10] - T[6] * T[8]) +
                       T[2] * (T[4] * T[9] - T[5] * T[8]);
    require(dev <= 1e-9 && det > 0.0, "pose rotation is not orthonormal with det +1 (tolerance 1e-9)");
}

int spec_dim(const cvo_feature_spec *sp)
{
    int D = 0;
    for (int b = 0; b < sp->nblocks; ++b) D += sp->dim[b];
    return D;
}

void check_spec(const cvo_feature_spec *sp)
{
    require(sp != nullptr, "feature spec is NULL");
    require(sp->nblocks >= 0 && sp->nblocks <= CVO_MAX_BLOCKS, "nblocks out of range [0, 8]");
    int nlin = 0;
    for (int b = 0; b < sp->nblocks; ++b) {
        require(sp->dim[b] > 0, "feature block dimension must be positive");
        require(sp->kind[b] == CVO_SE || sp->kind[b] == CVO_LIN, "unknown feature block kind");
        if (sp->kind[b] == CVO_SE)
            require(std::isfinite(sp->ell[b]) && sp->ell[b] > 0.0 && std::isfinite(sp->sigma[b]) &&
                        sp->sigma[b] > 0.0,
                    "SE feature block needs finite ell > 0 and sigma > 0");
        else
            ++nlin;
    }
    if (spec_dim(sp) > CVO_MAX_FEATURE_DIM) throw CvoError(CVO_ERR_UNSUPPORTED, "feature dimension above 64");
    if (nlin > 1) {
        // several LIN blocks run as their tensor product (eq. (6))
        long long prod = 1;
        int sed = 0;
        for (int b = 0; b < sp->nblocks; ++b) {
            if (sp->kind[b] == CVO_LIN) prod *= sp->dim[b];
            else sed += sp->dim[b];
        }
        if (prod > 64 || sed + prod > CVO_MAX_FEATURE_DIM)
            throw CvoError(CVO_ERR_UNSUPPORTED, "the tensor product of the LIN blocks has " + std::to_string(prod) +
                                                    " columns; at most 64 (with the SE columns) are supported");
    }
}

void check_cloud(const cvo_cloud *c, int D, const char *name)
{
    require(c != nullptr, std::string(name) + " cloud is NULL");
    require(c->n >= 0 && c->n < (1LL << 30), std::string(name) + ": point count out of range");
    if (c->n > 0) {
        require(c->xyz != nullptr, std::string(name) + ": xyz is NULL");
        if (D > 0) require(c->feat != nullptr, std::string(name) + ": feat is NULL but the spec has features");
    }
}

void check_kp(const cvo_kernel_params *kp)
{
    require(kp != nullptr, "kernel params are NULL");
    require(std::isfinite(kp->ell) && kp->ell > 0.0, "ell must be finite and > 0");
    require(std::isfinite(kp->sigma) && kp->sigma > 0.0, "sigma must be finite and > 0");
    require(!std::isnan(kp->kappa) && kp->kappa > 0.0, "kappa must be > 0 (+inf allowed)");
}

// ------------------------------------------------------------------ feature layout
FeatLayout make_layout(const cvo_feature_spec *sp, double sigma)
{
    FeatLayout L;
    std::memset(&L, 0, sizeof(L));
    int sed = 0, lind = 0, nlinb = 0, lprod = 1;
    for (int b = 0; b < sp->nblocks; ++b) {
        (sp->kind[b] == CVO_SE ? sed : lind) += sp->dim[b];
        if (sp->kind[b] == CVO_LIN) {
            ++nlinb;
            lprod *= sp->dim[b];
        }
    }
    if (nlinb > 1) lind = lprod;  // the tensor product of the LIN blocks (eq. (6))
    static const int S_opts[] = {0, 5, 8, 16, 32};
    static const int L_opts[] = {0, 4, 19, 32, 64};
    int bestS = -1, bestL = -1;
    for (int S : S_opts)
        for (int Lo : L_opts) {
            if (S < sed || Lo < lind || !pair_layout_supported(S, Lo)) continue;
            if (bestS < 0 || S + Lo < bestS + bestL) { bestS = S; bestL = Lo; }
        }
    if (bestS < 0) throw CvoError(CVO_ERR_UNSUPPORTED, "no compiled kernel for this feature layout");
    L.sed = bestS;
    L.lind = bestL;
    L.d4 = (bestS + bestL + 3) & ~3;
    L.src_dim = spec_dim(sp);
    for (int k = 0; k < 64; ++k) { L.col[k] = -1; L.scale[k] = 0.f; L.gscale[k] = 0.0; }
    double sig2 = sigma * sigma;
    int dst = 0, src = 0;
    for (int b = 0; b < sp->nblocks; ++b) {
        if (sp->kind[b] == CVO_SE) {
            const double f = std::sqrt(kLog2e / (2.0 * sp->ell[b] * sp->ell[b]));
            for (int k = 0; k < sp->dim[b]; ++k) {
                L.col[dst] = src + k;
                L.scale[dst] = (float)f;
                L.gscale[dst] = 1.0 / ((double)(float)f * sp->ell[b] * sp->ell[b]);
                ++dst;
            }
            sig2 *= sp->sigma[b] * sp->sigma[b];
        }
        src += sp->dim[b];
    }
    dst = bestS;
    src = 0;
    if (nlinb > 1) {
        L.nlin = nlinb;
        int i = 0;
        for (int b = 0; b < sp->nblocks; ++b) {
            if (sp->kind[b] == CVO_LIN) {
                L.lin_src[i] = src;
                L.lin_dim[i] = sp->dim[b];
                ++i;
            }
            src += sp->dim[b];
        }
        for (int c = 0; c < lprod; ++c) {
            L.col[dst] = -2;
            L.scale[dst] = 1.f;
            L.gscale[dst] = 1.0;
            ++dst;
        }
    } else {
        for (int b = 0; b < sp->nblocks; ++b) {
            if (sp->kind[b] == CVO_LIN)
                for (int k = 0; k < sp->dim[b]; ++k) {
                    L.col[dst] = src + k;
                    L.scale[dst] = 1.f;
                    L.gscale[dst] = 1.0;
                    ++dst;
                }
            src += sp->dim[b];
        }
    }
    L.sig2 = (float)sig2;
    return L;
}

// ------------------------------------------------------------------ views
struct GridView {
    int B = 0;
    std::vector<GridDesc> desc;
    GridDesc *d_desc = nullptr;
    float4 *pts = nullptr;
    float *feat = nullptr;
    int *perm = nullptr;
    int *cell_start = nullptr;
    long long ntot = 0;
    std::vector<double> rc;
};

struct ClusterView {
    int B = 0;
    std::vector<ClusterDesc> desc;
    ClusterDesc *d_desc = nullptr;
    float4 *pts = nullptr;
    float *feat = nullptr;
    int *perm = nullptr;
    int2 *clus = nullptr;
    double4 *cgeo = nullptr;
    int *cpair = nullptr;
    int *tclus = nullptr;  // cluster of every sorted point
    int nclus = 0;
    long long ntot = 0;
    std::vector<double> rc;
};

int bits_for(unsigned long long v)
{
    int b = 0;
    while ((1ULL << b) <= v && b < 63) ++b;
    return b;
}

// bounding boxes and the non-finite check
// Bounding boxes of one call's clouds, kept for the views rebuilt later in
// the same call (the clouds cannot change while a call runs).
struct BoxCache {
    std::vector<float> box;
    CloudPtrs *dc = nullptr;
};

std::vector<float> cloud_boxes(cvo_context *ctx, const std::string &pre, const std::vector<CloudPtrs> &cl,
                               CloudPtrs **d_clouds, BoxCache *cache = nullptr)
{
    if (cache && cache->dc) {
        *d_clouds = cache->dc;
        return cache->box;
    }
    const int B = (int)cl.size();
    CloudPtrs *dc = ctx->get_t<CloudPtrs>(pre + ".clouds", B);
    ctx->upload(dc, cl.data(), sizeof(CloudPtrs) * B);
    float *d_box = ctx->get_t<float>(pre + ".box", 8 * B);
    launch_bbox(dc, B, d_box, ctx->stream);
    ctx->check_launch("bbox");
    std::vector<float> box(8 * B);
    ctx->download(box.data(), d_box, sizeof(float) * 8 * B);
    for (int c = 0; c < B; ++c)
        require(box[8 * c + 6] == 0.0f, "a cloud has non-finite coordinates");
    *d_clouds = dc;
    if (cache) {
        cache->box = box;
        cache->dc = dc;
    }
    return box;
}

// Shape of the views of one pair: query points per cluster, grid cell edge
// and cluster edge cap, both relative to the cutoff radius.
struct ViewShape {
    int cluster_max;
    double cell_factor;
    double cluster_factor;
    int rule;  // CVO_CLUSTER_OCTREE or CVO_CLUSTER_CHUNKS
    bool operator==(const ViewShape &o) const
    {
        return cluster_max == o.cluster_max && cell_factor == o.cell_factor && cluster_factor == o.cluster_factor &&
               rule == o.rule;
    }
};

ViewShape fixed_shape(const cvo_context *ctx)
{
    return ViewShape{ctx->tuning.cluster_max, ctx->tuning.cell_factor, ctx->tuning.cluster_factor,
                     ctx->tuning.cluster_rule};
}

// Density classes and their view shapes, measured per feature layout (a
// same-box sweep of both cluster rules x 16/32/64 points x cell edge 0.5/1.0
// x cluster edge 0.5/1.0/1.5 r_c on the stereo and RGB-D pairs).  Chunk
// clusters win in every band but the sparsest, where the rules tie: their
// parts fill the power-of-two lane groups.  Dense bands cut the neighbourhood
// finer (cell edge r_c / 2) and keep clusters small in space; sparse bands
// let clusters grow past the cutoff radius so a wave's fixed cost is shared
// by more queries.  Rows of at most 8 floats (cheap pairs) keep 32-point
// clusters down to 100 pairs per query; wider rows switch to 16 below 500.
bool light_layout(const FeatLayout &lay) { return lay.d4 <= 8; }

void class_thresholds(const FeatLayout &lay, double t[3])
{
    t[0] = INFINITY;  // (no class 3: the densest shape is also class 2's)
    t[1] = light_layout(lay) ? 100.0 : 500.0;
    t[2] = light_layout(lay) ? 0.0 : 200.0;
}

ViewShape density_shape(cvo_context *ctx, int cls, const FeatLayout &lay)
{
    if (!ctx->tuning.adaptive) return fixed_shape(ctx);
    const bool light = light_layout(lay);
    auto it = ctx->class_shape.find({light ? 1 : 0, cls});
    if (it != ctx->class_shape.end()) {
        ctx->timing.tuned_view_shapes += 1;
        const auto &t = it->second;
        return ViewShape{t.cluster_max, t.cell_factor, t.cluster_factor, t.rule};
    }
    const int r = CVO_CLUSTER_CHUNKS;
    switch (cls) {
    case 3: return ViewShape{32, 0.5, 0.5, r};
    case 2: return light ? ViewShape{32, 0.5, 1.0, r} : ViewShape{32, 0.5, 0.5, r};
    case 1: return light ? ViewShape{16, 1.0, 1.5, r} : ViewShape{16, 0.5, 1.0, r};
    case 0: return light ? ViewShape{16, 1.0, 1.5, r} : ViewShape{16, 1.0, 1.0, r};
    default: return fixed_shape(ctx);
    }
}

GridView build_grid(cvo_context *ctx, const std::string &pre, const std::vector<CloudPtrs> &cl,
                    const std::vector<double> &rc, const FeatLayout &lay, const std::vector<ViewShape> &shape,
                    BoxCache *bc = nullptr)
{
    GridView v;
    const int B = (int)cl.size();
    v.B = B;
    v.rc = rc;
    CloudPtrs *dc = nullptr;
    std::vector<float> box = cloud_boxes(ctx, pre, cl, &dc, bc);
    const long long cell_cap = 1LL << 23;
    v.desc.resize(B);
    long long cell_base = 0, pt_base = 0, max_cells = 0, nmax = 0;
    std::vector<long long> bases(B);
    for (int c = 0; c < B; ++c) {
        GridDesc &g = v.desc[c];
        std::memset(&g, 0, sizeof(g));
        const long long n = cl[c].n;
        if (n == 0) {
            g.ox = g.oy = g.oz = 0.0;
            g.h = 1.0;
            g.inv_h = 1.0;
            g.nx = g.ny = g.nz = 1;
        } else {
            const double lo[3] = {box[8 * c], box[8 * c + 1], box[8 * c + 2]};
            const double hi[3] = {box[8 * c + 3], box[8 * c + 4], box[8 * c + 5]};
            double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-6});
            double h = std::isfinite(rc[c]) ? shape[c].cell_factor * rc[c] : ext * 1.01;
            h = std::max(h, ext * 1e-6);
            int nn[3];
            double inv = 1.0 / h;
            for (;;) {
                inv = 1.0 / h;
                long long tot = 1;
                for (int k = 0; k < 3; ++k) {
                    // same expression as the device binning: floor((p - o) * inv_h)
                    nn[k] = (int)std::floor((hi[k] - lo[k]) * inv) + 1;
                    tot *= nn[k];
                }
                if (tot <= cell_cap && nn[0] < (1 << 30) / std::max(1, nn[1])) break;
                h *= 1.25;
            }
            g.ox = lo[0];
            g.oy = lo[1];
            g.oz = lo[2];
            g.h = h;
            g.inv_h = inv;
            g.nx = nn[0];
            g.ny = nn[1];
            g.nz = nn[2];
        }
        g.cell_base = (int)cell_base;
        g.pt_base = pt_base;
        g.n = n;
        bases[c] = pt_base;
        const long long nc = (long long)g.nx * g.ny * g.nz;
        max_cells = std::max(max_cells, nc);
        cell_base += nc + 1;
        pt_base += n;
        nmax = std::max(nmax, n);
    }
    require(cell_base < (1LL << 31), "cell tables too large");
    v.ntot = pt_base;
    const int kbits = bits_for((unsigned long long)max_cells);  // max_cells itself must fit
    const int cbits = bits_for((unsigned long long)(B > 1 ? B - 1 : 0));
    require(kbits + cbits <= 62, "grid keys exceed 62 bits");
    v.d_desc = ctx->get_t<GridDesc>(pre + ".desc", B);
    ctx->upload(v.d_desc, v.desc.data(), sizeof(GridDesc) * B);
    long long *d_base = ctx->get_t<long long>(pre + ".base", B);
    ctx->upload(d_base, bases.data(), sizeof(long long) * B);

    const long long ntot = std::max(v.ntot, 1LL);
    unsigned long long *keys = ctx->get_t<unsigned long long>(pre + ".keys", ntot);
    unsigned long long *ktmp = ctx->get_t<unsigned long long>(pre + ".ktmp", ntot);
    int *vals = ctx->get_t<int>(pre + ".vals", ntot);
    int *vtmp = ctx->get_t<int>(pre + ".vtmp", ntot);
    const long long ntiles = (ntot + kRadixTile - 1) / kRadixTile;
    int *hist = ctx->get_t<int>(pre + ".hist", ntiles * 256);
    int *bsum = ctx->get_t<int>(pre + ".bsum", (ntiles * 256 + 2047) / 2048 + 1);
    v.pts = ctx->get_t<float4>(pre + ".pts", ntot);
    v.feat = ctx->get_t<float>(pre + ".feat", ntot * std::max(lay.d4, 1));
    v.perm = ctx->get_t<int>(pre + ".perm", ntot);
    v.cell_start = ctx->get_t<int>(pre + ".cells", cell_base);
    if (v.ntot > 0) {
        launch_grid_keys(dc, v.d_desc, B, nmax, keys, vals, kbits, ctx->stream);
        bool in_tmp = false;
        launch_radix_sort(keys, vals, ktmp, vtmp, hist, bsum, v.ntot, kbits + cbits, ctx->stream, &in_tmp);
        if (in_tmp) { std::swap(keys, ktmp); std::swap(vals, vtmp); }
        launch_gather(keys, vals, v.ntot, kbits, dc, d_base, lay, v.pts, v.feat, v.perm, ctx->stream);
    }
    launch_cell_table(keys, v.ntot, v.d_desc, B, max_cells, kbits, v.cell_start, ctx->stream);
    ctx->check_launch("grid build");
    return v;
}

ClusterView build_clusters(cvo_context *ctx, const std::string &pre, const std::vector<CloudPtrs> &cl,
                           const std::vector<double> &rc, const FeatLayout &lay, const std::vector<ViewShape> &shape,
                           BoxCache *bc = nullptr)
{
    ClusterView v;
    const int B = (int)cl.size();
    v.B = B;
    v.rc = rc;
    CloudPtrs *dc = nullptr;
    std::vector<float> box = cloud_boxes(ctx, pre, cl, &dc, bc);
    const int cbits = bits_for((unsigned long long)(B > 1 ? B - 1 : 0));
    const int maxbits = std::min(19, (62 - cbits) / 3);
    std::vector<ClusterBuild> cb(B);
    std::vector<int2> lcap(B);  // (largest octree level, max points per cluster)
    std::vector<long long> bases(B);
    v.desc.resize(B);
    long long pt_base = 0, nmax = 0, nchunks = 0;
    bool any_chunks = false, any_octree = false;
    int bits = 1;  // Morton bits per axis: as many as the widest cloud needs
    for (int c = 0; c < B; ++c) {
        const long long n = cl[c].n;
        ClusterBuild &g = cb[c];
        std::memset(&g, 0, sizeof(g));
        double lo[3] = {0, 0, 0}, ext = 1.0;
        if (n > 0) {
            for (int k = 0; k < 3; ++k) lo[k] = box[8 * c + k];
            ext = std::max({box[8 * c + 3] - lo[0], box[8 * c + 4] - lo[1], box[8 * c + 5] - lo[2], 1e-6});
        }
        const double cap = std::isfinite(rc[c]) ? shape[c].cluster_factor * rc[c] : ext * 2.0;
        // octree blocks need 16 quanta per cap; chunks only use the Morton
        // order, which a finer quantum makes more local
        const bool chunks = shape[c].rule == CVO_CLUSTER_CHUNKS;
        int L = chunks ? 6 : 4;
        double q = cap / (double)(1 << L);
        // quanta needed to cover the box must fit in maxbits per axis
        if (ext / q + 1.0 > (double)(1 << maxbits)) {
            q = ext / ((double)(1 << maxbits) - 2.0);
            L = std::max(0, (int)std::floor(std::log2(std::max(cap / q, 1.0))));
        }
        L = std::min(L, maxbits);
        // quanta along the widest axis (+1 for rounding at the far face)
        bits = std::max({bits, L, bits_for((unsigned long long)std::floor(ext / q) + 1)});
        g.ox = lo[0];
        g.oy = lo[1];
        g.oz = lo[2];
        g.q = q;
        g.pt_base = pt_base;
        g.n = n;
        g.cap = cap;
        g.chunk_base = nchunks;
        nchunks += (n + shape[c].cluster_max - 1) / shape[c].cluster_max;
        any_chunks = any_chunks || chunks;
        // (octree level -1 marks a cloud clustered by the chunk rule)
        lcap[c] = make_int2(chunks ? -1 : L, shape[c].cluster_max);
        any_octree = any_octree || !chunks;
        bases[c] = pt_base;
        ClusterDesc &d = v.desc[c];
        d.clus_base = 0;
        d.nclus = 0;
        d.pt_base = (int)pt_base;
        d.n = (int)n;
        pt_base += n;
        nmax = std::max(nmax, n);
    }
    v.ntot = pt_base;
    bits = std::min(bits, maxbits);
    ClusterBuild *d_cb = ctx->get_t<ClusterBuild>(pre + ".cb", B);
    ctx->upload(d_cb, cb.data(), sizeof(ClusterBuild) * B);
    long long *d_base = ctx->get_t<long long>(pre + ".base", B);
    ctx->upload(d_base, bases.data(), sizeof(long long) * B);
    int2 *d_lcap = ctx->get_t<int2>(pre + ".lcap", B);
    ctx->upload(d_lcap, lcap.data(), sizeof(int2) * B);
    v.d_desc = ctx->get_t<ClusterDesc>(pre + ".desc", B);

    const long long ntot = std::max(v.ntot, 1LL);
    unsigned long long *keys = ctx->get_t<unsigned long long>(pre + ".keys", ntot);
    unsigned long long *ktmp = ctx->get_t<unsigned long long>(pre + ".ktmp", ntot);
    int *vals = ctx->get_t<int>(pre + ".vals", ntot);
    int *vtmp = ctx->get_t<int>(pre + ".vtmp", ntot);
    const long long ntiles = (ntot + kRadixTile - 1) / kRadixTile;
    int *hist = ctx->get_t<int>(pre + ".hist", std::max(ntiles * 256, ntot));
    int *bsum = ctx->get_t<int>(pre + ".bsum", (std::max(ntiles * 256, ntot) + 2047) / 2048 + 1);
    v.pts = ctx->get_t<float4>(pre + ".pts", ntot);
    v.feat = ctx->get_t<float>(pre + ".feat", ntot * std::max(lay.d4, 1));
    v.perm = ctx->get_t<int>(pre + ".perm", ntot);
    v.clus = ctx->get_t<int2>(pre + ".clus", ntot);
    v.cgeo = ctx->get_t<double4>(pre + ".cgeo", ntot);
    v.cpair = ctx->get_t<int>(pre + ".cpair", ntot);
    v.tclus = ctx->get_t<int>(pre + ".tclus", ntot);
    int *head = ctx->get_t<int>(pre + ".head", ntot);
    int *hidx = ctx->get_t<int>(pre + ".hidx", ntot);
    int2 *span = ctx->get_t<int2>(pre + ".span", ntot);
    int *d_total = ctx->get_t<int>(pre + ".total", 1);
    v.nclus = 0;
    if (v.ntot > 0) {
        launch_morton_keys(dc, d_cb, B, nmax, keys, vals, bits, ctx->stream);
        bool in_tmp = false;
        launch_radix_sort(keys, vals, ktmp, vtmp, hist, bsum, v.ntot, 3 * bits + cbits, ctx->stream, &in_tmp);
        if (in_tmp) { std::swap(keys, ktmp); std::swap(vals, vtmp); }
        launch_gather(keys, vals, v.ntot, 3 * bits, dc, d_base, lay, v.pts, v.feat, v.perm, ctx->stream);
        // each cloud by its own rule: the octree kernel skips chunk-rule
        // clouds, and chunks exist only for chunk-rule clouds
        if (any_octree) launch_cluster_heads(keys, v.ntot, d_lcap, 3 * bits, head, span, ctx->stream);
        if (any_chunks) launch_chunk_heads(v.pts, d_cb, d_lcap, B, nchunks, head, span, ctx->stream);
        launch_exclusive_scan(head, hidx, bsum, v.ntot, d_total, ctx->stream);
        launch_cluster_emit(head, hidx, span, v.pts, keys, 3 * bits, v.ntot, v.clus, v.cgeo, v.cpair, v.tclus,
                            ctx->stream);
        ctx->check_launch("cluster build");
        int total = 0;
        ctx->download(&total, d_total, sizeof(int));
        v.nclus = total;
    }
    ctx->upload(v.d_desc, v.desc.data(), sizeof(ClusterDesc) * B);
    return v;
}

// ------------------------------------------------------------------ work plan
// Pieces: every cluster's candidate list (at the pose in the device state) is
// shared by pieces of about `piece_work` query x candidate products, each
// taking every np-th chunk of 64 candidates, and the pieces are processed
// heaviest first.
struct Plan {
    int4 *qmap = nullptr;   // per query: (t, cluster size, pieces, first slot)
    int4 *pieces = nullptr;
    int *porder = nullptr;
    PieceRec *recs = nullptr;
    int2 *cpieces = nullptr;
    int npieces = 0;
    long long nslots = 0;
};

// With exact_slots false, nslots is only an upper bound (64 queries per
// piece), which sizes the forward moments without a host read.
Plan make_plan(cvo_context *ctx, const std::string &pre, const ClusterView &q, const GridView &r,
               const PairState *d_state, int inverse, double kappa, bool exact_slots = true)
{
    Plan pl;
    if (q.nclus == 0) return pl;
    PairPassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.clus = q.clus;
    a.cgeo = q.cgeo;
    a.cpair = q.cpair;
    a.nclus = q.nclus;
    a.cell_start = r.cell_start;
    a.grids = r.d_desc;
    a.state = d_state;
    a.pose_is_inverse = inverse;
    a.kappa = kappa;
    const int nc = q.nclus;
    int *npc = ctx->get_t<int>(pre + ".npc", nc);
    int *cmax = ctx->get_t<int>(pre + ".cmax", nc);
    long long *ccount = ctx->get_t<long long>(pre + ".ccount", nc);
    int *pbase = ctx->get_t<int>(pre + ".pbase", nc);
    int *bsum = ctx->get_t<int>(pre + ".pbsum", (nc + 2047) / 2048 + 1);
    int *d_total = ctx->get_t<int>(pre + ".ptotal", 2);
    launch_plan_count(a, ctx->tuning.piece_work, npc, cmax, ccount, ctx->stream);
    launch_exclusive_scan(npc, pbase, bsum, nc, d_total, ctx->stream);
    ctx->check_launch("plan count");
    int P = 0;
    ctx->download(&P, d_total, sizeof(int));
    pl.npieces = P;
    pl.pieces = ctx->get_t<int4>(pre + ".pieces", P);
    int *pn = ctx->get_t<int>(pre + ".pn", P);
    int *tbase = ctx->get_t<int>(pre + ".tbase", P);
    unsigned long long *key = ctx->get_t<unsigned long long>(pre + ".pkey", P);
    unsigned long long *ktmp = ctx->get_t<unsigned long long>(pre + ".pktmp", P);
    int *val = ctx->get_t<int>(pre + ".pval", P);
    int *vtmp = ctx->get_t<int>(pre + ".pvtmp", P);
    const long long ntiles = (P + kRadixTile - 1) / kRadixTile;
    int *hist = ctx->get_t<int>(pre + ".phist", ntiles * 256);
    int *bsum2 = ctx->get_t<int>(pre + ".pbsum2", (std::max<long long>(ntiles * 256, P) + 2047) / 2048 + 1);
    pl.cpieces = ctx->get_t<int2>(pre + ".cpieces", nc);
    launch_plan_emit(a, npc, pbase, ccount, pl.pieces, pn, key, val, pl.cpieces, ctx->stream);
    launch_exclusive_scan(pn, tbase, bsum2, P, d_total + 1, ctx->stream);
    launch_plan_slots(pl.pieces, tbase, P, ctx->stream);
    pl.qmap = ctx->get_t<int4>(pre + ".qmap", std::max<long long>(q.ntot, 1));
    launch_plan_qmap(q.clus, pl.cpieces, pl.pieces, nc, pl.qmap, ctx->stream);
    bool in_tmp = false;
    launch_radix_sort(key, val, ktmp, vtmp, hist, bsum2, P, 16, ctx->stream, &in_tmp);
    pl.porder = in_tmp ? vtmp : val;
    pl.recs = ctx->get_t<PieceRec>(pre + ".recs", std::max(P, 1));
    launch_plan_records(pl.porder, pl.pieces, q.cpair, q.clus, q.cgeo, P, pl.recs, ctx->stream);
    ctx->check_launch("plan emit");
    if (exact_slots) {
        int nslots = 0;
        ctx->download(&nslots, d_total + 1, sizeof(int));
        pl.nslots = nslots;
    } else {
        pl.nslots = (long long)P * kWave;
    }
    return pl;
}

// ------------------------------------------------------------------ pair pass + reduce
struct Moments {
    double *W, *D, *G, *L;
    float *S;
    int *cnt;
};

Moments moments(cvo_context *ctx, const std::string &pre, long long n, int d4, bool backward)
{
    Moments m{};
    n = std::max(n, 1LL);
    m.W = ctx->get_t<double>(pre + ".W", n);
    m.D = ctx->get_t<double>(pre + ".D", 3 * n);
    m.cnt = ctx->get_t<int>(pre + ".cnt", n);
    if (backward) {
        m.G = ctx->get_t<double>(pre + ".G", n * std::max(d4, 1));
        m.L = ctx->get_t<double>(pre + ".L", n);
        m.S = nullptr;
    } else {
        m.S = ctx->get_t<float>(pre + ".S", 6 * n);
        m.G = m.L = nullptr;
    }
    return m;
}

PairPassArgs pass_args(const ClusterView &q, const GridView &r, const PairState *st, int inverse, float sig2,
                       double kappa, const Moments &m, const Plan &pl)
{
    PairPassArgs a;
    std::memset(&a, 0, sizeof(a));
    a.qpts = q.pts;
    a.qfeat = q.feat;
    a.clus = q.clus;
    a.cgeo = q.cgeo;
    a.cpair = q.cpair;
    a.nclus = q.nclus;
    a.rpts = r.pts;
    a.rfeat = r.feat;
    a.cell_start = r.cell_start;
    a.grids = r.d_desc;
    a.state = st;
    a.pose_is_inverse = inverse;
    a.sig2 = sig2;
    a.kappa = kappa;
    a.oW = m.W;
    a.oD = m.D;
    a.oS = m.S;
    a.oCnt = m.cnt;
    a.oG = m.G;
    a.oL = m.L;
    a.recs = pl.recs;
    a.npieces = pl.npieces;
    return a;
}

SlotMap slot_map(const Plan &pl)
{
    SlotMap m;
    m.qmap = pl.qmap;
    return m;
}

void run_pair_pass(cvo_context *ctx, const PairPassArgs &a, const FeatLayout &lay, int mode)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ctx->profiling) {
        e0 = ctx->event();
        e1 = ctx->event();
        HIP_OK(hipEventRecord(e0, ctx->stream));
    }
    if (!launch_pair_pass(a, lay, mode, ctx->stream))
        throw CvoError(CVO_ERR_UNSUPPORTED, "no compiled pair kernel for the feature layout");
    ctx->check_launch("pair pass");
    if (ctx->profiling) {
        HIP_OK(hipEventRecord(e1, ctx->stream));
        ctx->ev_pending.push_back({e0, e1});
    }
    ctx->timing.evaluations += 1;
}

// Blocks per pair of the reduction: one thread per query point, up to 512
// blocks.
int reduce_blocks(const std::vector<ClusterDesc> &cd)
{
    long long mx = 1;
    for (auto &d : cd) mx = std::max(mx, (long long)d.n);
    long long nb = (mx + kRedThreads - 1) / kRedThreads;
    return (int)std::min(std::max(nb, 1LL), 512LL);
}

PairState init_state(const double *T, double ell)
{
    PairState s;
    std::memset(&s, 0, sizeof(s));
    std::memcpy(s.T, T, sizeof(double) * 12);
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) s.Tinv[4 * r + k] = T[4 * k + r];
        s.Tinv[4 * r + 3] = -(T[r] * T[3] + T[4 + r] * T[7] + T[8 + r] * T[11]);
    }
    s.ell = ell;
    s.i_prev = NAN;
    s.status = ST_RUNNING;
    s.done = 0;
    s.cls_built = -1;
    s.pause = 0;
    return s;
}

// Everything a forward evaluation or an ascent needs for B pairs.
struct Problem {
    FeatLayout lay;
    GridView grid;       // X clouds, reference role
    ClusterView clus;    // Z clouds, query role
    Plan plan;
    Moments mom;
    std::vector<ViewShape> shape;  // per pair, of the current views
    PairState *d_state = nullptr;
    AlignConst *d_ac = nullptr;
    double *partials = nullptr;
    int nblk = 1;
    double kappa = 3.0;
    float sig2 = 1.f;
    int ellobj = 0;         // reduce the lengthscale objective's sums too
    BoxCache box_x, box_z;  // bounding boxes from the first view build
};

// Grid of X, clusters of Z, and the work plan at the pose held in the device
// state (which must be current).
void build_views(cvo_context *ctx, Problem &p, const std::vector<CloudPtrs> &X, const std::vector<CloudPtrs> &Z,
                 const std::vector<double> &ell, const std::vector<ViewShape> &shape)
{
    p.shape = shape;
    ctx->timing.view_builds += 1;
    std::vector<double> rc(ell.size());
    for (size_t k = 0; k < ell.size(); ++k) rc[k] = p.kappa * ell[k];
    p.grid = build_grid(ctx, "fx", X, rc, p.lay, shape, &p.box_x);
    p.clus = build_clusters(ctx, "fz", Z, rc, p.lay, shape, &p.box_z);
    // the fixed scratch of the allocation-free entry point is sized by the
    // exact slot count (one host read) rather than its loose upper bound
    p.plan = make_plan(ctx, "fp", p.clus, p.grid, p.d_state, 0, p.kappa, ctx->fixed.on);
    p.mom = moments(ctx, "fm", p.plan.nslots, p.lay.d4, false);
    p.nblk = reduce_blocks(p.clus.desc);
    p.partials = ctx->get_t<double>("partials", shape.size() * (size_t)p.nblk * kRedVals);
}

void setup_problem(cvo_context *ctx, Problem &p, const std::vector<CloudPtrs> &X, const std::vector<CloudPtrs> &Z,
                   const std::vector<PairState> &st, const std::vector<AlignConst> &ac)
{
    const int B = (int)X.size();
    std::vector<double> ell(B);
    for (int b = 0; b < B; ++b) ell[b] = st[b].ell;
    p.d_state = ctx->get_t<PairState>("state", B);
    ctx->upload(p.d_state, st.data(), sizeof(PairState) * B);
    build_views(ctx, p, X, Z, ell, std::vector<ViewShape>(B, fixed_shape(ctx)));
    p.d_ac = ctx->get_t<AlignConst>("aconst", B);
    ctx->upload(p.d_ac, ac.data(), sizeof(AlignConst) * B);
}

// Kernel arguments of one ascent iteration (pair pass, then reduction).
void iteration_args(const Problem &p, int mode, double *trace, long long trace_rows, PairPassArgs &a,
                    ReduceArgs &r)
{
    a = pass_args(p.clus, p.grid, p.d_state, 0, p.sig2, p.kappa, p.mom, p.plan);
    std::memset(&r, 0, sizeof(r));
    r.qpts = p.clus.pts;
    r.cdesc = p.clus.d_desc;
    r.map = slot_map(p.plan);
    r.W = p.mom.W;
    r.D = p.mom.D;
    r.S = p.mom.S;
    r.cnt = p.mom.cnt;
    r.state = p.d_state;
    r.ac = p.d_ac;
    r.partials = p.partials;
    r.trace = trace;
    r.trace_rows = trace_rows;
    r.nblk = p.nblk;
    r.mode = mode;
    r.ellobj = p.ellobj;
    long long mx = 0;
    for (const auto &d : p.clus.desc) mx = std::max(mx, (long long)d.n);
    r.one_query = (long long)p.nblk * kRedThreads >= mx;
}

void enqueue_iteration(cvo_context *ctx, Problem &p, int mode, double *trace, long long trace_rows, bool timed)
{
    PairPassArgs a;
    ReduceArgs r;
    iteration_args(p, mode, trace, trace_rows, a, r);
    if (timed) run_pair_pass(ctx, a, p.lay, 0);
    else {
        if (!launch_pair_pass(a, p.lay, 0, ctx->stream))
            throw CvoError(CVO_ERR_UNSUPPORTED, "no compiled pair kernel for the feature layout");
        ctx->timing.evaluations += 1;
    }
    launch_reduce(r, p.grid.B, ctx->stream);
    ctx->check_launch("reduce");
}

// Everything a captured run of U iterations bakes into its launches: the
// kernel arguments (buffers, counts, plan), the feature layout, the batch
// size and U.  A graph is replayed only while this key is unchanged.
std::string iteration_key(const Problem &p, double *trace, long long trace_rows, int B, int U)
{
    PairPassArgs a;
    ReduceArgs r;
    iteration_args(p, 1, trace, trace_rows, a, r);
    std::string k;
    k.append(reinterpret_cast<const char *>(&a), sizeof(a));
    k.append(reinterpret_cast<const char *>(&r), sizeof(r));
    k.append(reinterpret_cast<const char *>(&p.lay), sizeof(p.lay));
    k.append(reinterpret_cast<const char *>(&B), sizeof(B));
    k.append(reinterpret_cast<const char *>(&U), sizeof(U));
    return k;
}

CloudPtrs to_ptrs(const cvo_cloud *c)
{
    CloudPtrs p;
    p.xyz = c->xyz;
    p.feat = c->feat;
    p.n = c->n;
    return p;
}

AlignConst const_for(const cvo_align_params *ap, long long N, long long M)
{
    AlignConst a;
    std::memset(&a, 0, sizeof(a));
    if (ap) {
        a.ell_min = ap->ell_min;
        a.decay = ap->decay;
        a.ind_rel_tol = ap->ind_rel_tol;
        a.eps_rot = ap->eps_rot;
        a.eps_trans = ap->eps_trans;
        a.step_lambda = ap->step_lambda;
        a.max_iter = ap->max_iter;
        a.fixed_iters = ap->fixed_iters;
        a.metric = ap->metric;
        a.ell_mode = ap->ell_mode;
        a.ell_init = ap->ell_init;
        a.kappa = ap->kappa;
    } else {
        a.max_iter = 1;
        a.step_lambda = 1.0;
        a.kappa = INFINITY;
    }
    a.rebuild_ratio = 1.0;
    a.adaptive = 0;
    a.cls_t[0] = a.cls_t[1] = a.cls_t[2] = INFINITY;
    a.sqrt_nm = std::sqrt((double)N * (double)M);
    a.inv_m = M > 0 ? 1.0 / (double)M : 0.0;
    return a;
}

void check_align_params(const cvo_align_params *ap)
{
    require(ap != nullptr, "align params are NULL");
    require(std::isfinite(ap->ell_init) && ap->ell_init > 0.0, "ell_init must be finite and > 0");
    require(std::isfinite(ap->ell_min) && ap->ell_min > 0.0, "ell_min must be finite and > 0");
    require(ap->decay > 0.0 && ap->decay < 1.0, "decay must lie in (0, 1)");
    require(ap->ind_rel_tol >= 0.0, "ind_rel_tol must be >= 0");
    require(ap->eps_rot >= 0.0 && ap->eps_trans >= 0.0, "eps must be >= 0");
    require(std::isfinite(ap->step_lambda) && ap->step_lambda > 0.0, "step_lambda must be > 0");
    require(std::isfinite(ap->sigma) && ap->sigma > 0.0, "sigma must be > 0");
    require(!std::isnan(ap->kappa) && ap->kappa > 0.0, "kappa must be > 0");
    require(ap->max_iter >= 1, "max_iter must be >= 1");
    require(ap->metric == CVO_METRIC_KINETIC || ap->metric == CVO_METRIC_IDENTITY, "unknown metric");
    require(ap->ell_mode == CVO_ELL_ANNEAL || ap->ell_mode == CVO_ELL_ADAPTIVE, "unknown ell_mode");
    require(ap->reserved == 0, "reserved must be 0");
}

// single forward evaluation
void evaluate_one(cvo_context *ctx, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                  const cvo_kernel_params *kp, const double *T, PairState *out, bool ellobj = false)
{
    check_spec(spec);
    const int D = spec_dim(spec);
    check_cloud(X, D, "X");
    check_cloud(Z, D, "Z");
    check_kp(kp);
    check_pose(T);
    PairState s0 = init_state(T, kp->ell);
    if (X->n == 0 || Z->n == 0) {
        *out = s0;
        return;
    }
    Problem p;
    p.kappa = kp->kappa;
    p.lay = make_layout(spec, kp->sigma);
    p.sig2 = p.lay.sig2;
    p.ellobj = ellobj ? 1 : 0;
    AlignConst ac = const_for(nullptr, X->n, Z->n);
    setup_problem(ctx, p, {to_ptrs(X)}, {to_ptrs(Z)}, {s0}, {ac});
    enqueue_iteration(ctx, p, 0, nullptr, 0, ctx->profiling);
    ctx->download(out, p.d_state, sizeof(PairState));
    if (ctx->profiling) {
        ctx->harvest_events();
        ctx->timing.pair_count += (long long)out->n_pairs;
    }
}

cvo_status fail(cvo_context *ctx, const CvoError &e)
{
    if (ctx) ctx->err = e.what();
    return e.code;
}

template <class F> cvo_status guarded(cvo_context *ctx, F &&f)
{
    if (!ctx) return CVO_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    try {
        HIP_OK(hipSetDevice(ctx->device));
        (void)hipGetLastError();  // drop any error left by an earlier failure
        ctx->ring_drain();        // copies an earlier, failed call may have left in flight
        f();
        return CVO_OK;
    } catch (const CvoError &e) {
        return fail(ctx, e);
    } catch (const std::exception &e) {
        ctx->err = e.what();
        return CVO_ERR_DEVICE;
    }
}

// ------------------------------------------------------------------ ascent driver
void align_many(cvo_context *ctx, const std::vector<CloudPtrs> &X, const std::vector<CloudPtrs> &Z,
                const cvo_feature_spec *spec, const std::vector<cvo_align_params> &prm,
                const std::vector<const double *> &T0, std::vector<PairState> &final_state, double *trace_host,
                bool use_graph, const double *d_sched = nullptr, long long n_sched = 0)
{
    const int B = (int)X.size();
    Problem p;
    p.kappa = prm[0].kappa;
    p.lay = make_layout(spec, prm[0].sigma);
    p.sig2 = p.lay.sig2;
    const bool cut = std::isfinite(p.kappa);
    const bool adapt = cut && ctx->tuning.adaptive;
    for (int b = 0; b < B; ++b)
        if (prm[b].ell_mode == CVO_ELL_ADAPTIVE && !prm[b].fixed_iters && !d_sched) p.ellobj = 1;
    std::vector<PairState> st(B);
    std::vector<AlignConst> ac(B);
    long long trace_rows = 0;
    for (int b = 0; b < B; ++b) {
        st[b] = init_state(T0[b], prm[b].ell_init);
        st[b].rc_build = p.kappa * prm[b].ell_init;
        ac[b] = const_for(&prm[b], X[b].n, Z[b].n);
        ac[b].ell_sched = d_sched;
        ac[b].n_sched = n_sched;
        ac[b].rebuild_ratio = ctx->tuning.rebuild_ratio;
        ac[b].adaptive = adapt ? 1 : 0;
        class_thresholds(p.lay, ac[b].cls_t);
        if (X[b].n == 0 || Z[b].n == 0) {
            st[b].status = ST_NO_OVERLAP;
            st[b].done = 1;
        }
        trace_rows = std::max(trace_rows, (long long)prm[b].max_iter);
    }
    double *d_trace = trace_host ? ctx->get_t<double>("trace", (size_t)B * trace_rows * kTraceLen) : nullptr;
    setup_problem(ctx, p, X, Z, st, ac);
    const int U = std::max(1, std::min(64, (int)ctx->tuning.unroll));
    // Views are rebuilt only where the device paused a pair (its cutoff
    // shrank, or its pair density fell a class) -- a function of the iterates
    // alone.  With adaptive shapes, the first iteration runs by itself and its
    // measured density picks the first shape.
    std::vector<double> ell_build(B);
    for (int b = 0; b < B; ++b) ell_build[b] = prm[b].ell_init;
    bool probe = adapt;
    std::vector<PairState> now(B);
    // Every launched iteration either ends a running pair or advances its
    // step count, so a batch after which a pair that was running has done
    // neither means the device state is not what the host expects: an error,
    // not another batch (the loop below otherwise ends only when every pair
    // is done).
    std::vector<PairState> ref = st;
    size_t timed_done = 0;  // pending timed launches of batches already waited for
    for (;;) {
        if (probe) {
            enqueue_iteration(ctx, p, 1, d_trace, trace_rows, ctx->profiling);
        } else if (use_graph) {
            const std::string key = iteration_key(p, d_trace, trace_rows, B, U);
            if (!ctx->graph || ctx->graph_key != key) {
                if (ctx->graph) HIP_OK(hipGraphExecDestroy(ctx->graph));
                ctx->graph = nullptr;
                hipGraph_t g = nullptr;
                HIP_OK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
                try {
                    for (int u = 0; u < U; ++u) enqueue_iteration(ctx, p, 1, d_trace, trace_rows, false);
                } catch (...) {
                    hipStreamEndCapture(ctx->stream, &g);
                    if (g) hipGraphDestroy(g);
                    (void)hipGetLastError();
                    throw;
                }
                HIP_OK(hipStreamEndCapture(ctx->stream, &g));
                HIP_OK(hipGraphInstantiate(&ctx->graph, g, nullptr, nullptr, 0));
                HIP_OK(hipGraphDestroy(g));
                ctx->graph_key = key;
                ctx->timing.graph_captures += 1;
                ctx->timing.evaluations -= U;  // counted per replay below, not at capture
            }
            HIP_OK(hipGraphLaunch(ctx->graph, ctx->stream));
            ctx->timing.graph_launches += 1;
            ctx->timing.evaluations += U;
        } else {
            for (int u = 0; u < U; ++u) enqueue_iteration(ctx, p, 1, d_trace, trace_rows, ctx->profiling);
        }
        // the previous batch's launch times are read while this batch runs
        if (ctx->profiling) ctx->harvest_events(timed_done);
        ctx->download(now.data(), p.d_state, sizeof(PairState) * B);
        timed_done = ctx->ev_pending.size();
        for (int b = 0; b < B; ++b)
            if (!ref[b].done && !ref[b].pause && !now[b].done && now[b].it <= ref[b].it)
                throw CvoError(CVO_ERR_DEVICE, "pair " + std::to_string(b) +
                                                   ": a launched batch of iterations left it running at step " +
                                                   std::to_string(now[b].it));
        bool all_done = true, rebuild = false, changed = false;
        std::vector<ViewShape> shape = p.shape;
        for (int b = 0; b < B; ++b) {
            if (now[b].done) continue;
            all_done = false;
            if (!probe && !now[b].pause) continue;
            const int cls = adapt ? density_class(now[b].n_pairs / (double)std::max(Z[b].n, 1LL), ac[b].cls_t) : -1;
            const ViewShape want = adapt ? density_shape(ctx, cls, p.lay) : fixed_shape(ctx);
            if (now[b].pause || !(want == p.shape[b])) {
                rebuild = true;
                ell_build[b] = now[b].ell;
                shape[b] = want;
                now[b].rc_build = p.kappa * now[b].ell;
            }
            now[b].cls_built = cls;
            now[b].pause = 0;
            changed = true;
        }
        probe = false;
        if (all_done) {
            if (ctx->profiling) ctx->harvest_events();
            break;
        }
        if (rebuild) build_views(ctx, p, X, Z, ell_build, shape);
        if (changed) ctx->upload(p.d_state, now.data(), sizeof(PairState) * B);
        ref = now;
    }
    final_state = now;
    if (ctx->profiling)
        for (int b = 0; b < B; ++b) ctx->timing.pair_count += (long long)now[b].total_pairs;
    if (trace_host && d_trace)
        ctx->download(trace_host, d_trace, sizeof(double) * (size_t)B * trace_rows * kTraceLen);
}

void fill_report(const PairState &s, cvo_align_report *r)
{
    std::memset(r, 0, sizeof(*r));
    r->iterations = s.it;
    r->final_ell = s.ell;
    r->F = s.F;
    r->i_theta = s.i_theta;
    r->n_pairs = (int64_t)s.n_pairs;
    r->status = s.status == ST_RUNNING ? CVO_MAX_ITER : s.status;
    r->total_pairs = (int64_t)s.total_pairs;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

cvo_status cvo_create(cvo_handle *out, int device, void *stream)
{
    if (!out) return CVO_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CVO_ERR_INVALID_ARGUMENT;
    cvo_context *ctx = new (std::nothrow) cvo_context();
    if (!ctx) return CVO_ERR_OUT_OF_MEMORY;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete ctx;
        return CVO_ERR_DEVICE;
    }
    // this device's copy of the allocation-free scratch; a failed lookup
    // only disables cvo_evaluate_noalloc (it reports the error)
    void *fixed = nullptr;
    const hipError_t e = scratch_address(device, &fixed);
    if (e == hipSuccess) {
        ctx->fixed.base = static_cast<char *>(fixed);
        ctx->fixed.cap = (size_t)CVO_NOALLOC_SCRATCH_MIB << 20;
    } else {
        ctx->fixed_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        (void)hipGetLastError();
    }
    *out = ctx;
    return CVO_OK;
}

void cvo_destroy(cvo_handle h)
{
    if (!h) return;
    hipSetDevice(h->device);
    if (h->stream) hipStreamSynchronize(h->stream);
    if (h->ring_off) hipStreamSynchronize(h->ring_stream);
    h->release();
    delete h;
}

cvo_status cvo_set_stream(cvo_handle h, void *stream)
{
    if (!h) return CVO_ERR_INVALID_ARGUMENT;
    h->stream = static_cast<hipStream_t>(stream);
    return CVO_OK;
}

const char *cvo_last_error(cvo_handle h) { return h ? h->err.c_str() : "NULL handle"; }

cvo_status cvo_inner_product(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                             const cvo_kernel_params *kp, const double T[12], double *F, int64_t *n_pairs)
{
    return guarded(h, [&] {
        require(F != nullptr, "F output is NULL");
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s);
        *F = s.F;
        if (n_pairs) *n_pairs = (int64_t)s.n_pairs;
    });
}

cvo_status cvo_gradient(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                        const cvo_kernel_params *kp, const double T[12], double *F, double grad[6],
                        int64_t *n_pairs)
{
    return guarded(h, [&] {
        require(grad != nullptr, "grad output is NULL");
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s);
        if (F) *F = s.F;
        for (int k = 0; k < 6; ++k) grad[k] = s.grad[k];
        if (n_pairs) *n_pairs = (int64_t)s.n_pairs;
    });
}

cvo_status cvo_evaluate(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                        const cvo_kernel_params *kp, const double T[12], cvo_eval *out)
{
    return guarded(h, [&] {
        require(out != nullptr, "output is NULL");
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s);
        out->F = s.F;
        for (int k = 0; k < 6; ++k) out->grad[k] = s.grad[k];
        out->curv = s.curv;
        out->dF_dell = s.dF_dell;
        out->r_max = s.r_max;
        out->i_theta = s.i_theta;
        out->n_pairs = (int64_t)s.n_pairs;
    });
}

cvo_status cvo_ell_objective(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                             const cvo_kernel_params *kp, const double T[12], double out[4])
{
    return guarded(h, [&] {
        require(out != nullptr, "output is NULL");
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s, true);
        const bool empty = X->n == 0 || Z->n == 0;
        out[0] = empty ? 0.0 : s.J;
        out[1] = empty ? 0.0 : s.dJ_dell;
        out[2] = empty ? 0.0 : s.ell_ml;
        out[3] = empty ? 0.0 : s.zplus;
    });
}

cvo_status cvo_evaluate_noalloc(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                                const cvo_kernel_params *kp, const double T[12], cvo_eval *out)
{
    return guarded(h, [&] {
        require(out != nullptr, "output is NULL");
        require(X != nullptr && Z != nullptr, "cloud is NULL");
        require(X->n <= CVO_NOALLOC_MAX_POINTS && Z->n <= CVO_NOALLOC_MAX_POINTS,
                "cvo_evaluate_noalloc takes at most " + std::to_string(CVO_NOALLOC_MAX_POINTS) +
                    " points per cloud (got " + std::to_string(X->n) + " and " + std::to_string(Z->n) + ")");
        if (!h->fixed.base) throw CvoError(CVO_ERR_DEVICE, "no allocation-free scratch: " + h->fixed_error);
        // every buffer of this call comes from the fixed array; no events
        struct Scope {
            cvo_context *c;
            bool prof;
            explicit Scope(cvo_context *c_) : c(c_), prof(c_->profiling)
            {
                c->fixed.on = true;
                c->fixed.top = 0;
                c->fixed.regions.clear();
                c->profiling = false;
            }
            ~Scope()
            {
                c->fixed.on = false;
                c->profiling = prof;
            }
        } scope(h);
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s);
        out->F = s.F;
        for (int k = 0; k < 6; ++k) out->grad[k] = s.grad[k];
        out->curv = s.curv;
        out->dF_dell = s.dF_dell;
        out->r_max = s.r_max;
        out->i_theta = s.i_theta;
        out->n_pairs = (int64_t)s.n_pairs;
    });
}

cvo_status cvo_metric(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                      const cvo_kernel_params *kp, const double T[12], double *i_theta)
{
    return guarded(h, [&] {
        require(i_theta != nullptr, "output is NULL");
        PairState s;
        evaluate_one(h, X, Z, spec, kp, T, &s);
        *i_theta = (X->n > 0 && Z->n > 0) ? s.i_theta : 0.0;
    });
}

cvo_status cvo_cosine(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                      const cvo_kernel_params *kp, const double T[12], double *cos_theta, double sums[3])
{
    return guarded(h, [&] {
        require(cos_theta != nullptr, "output is NULL");
        static const double I[12] = {1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
        PairState sxz, sxx, szz;
        evaluate_one(h, X, Z, spec, kp, T, &sxz);
        evaluate_one(h, X, X, spec, kp, I, &sxx);
        evaluate_one(h, Z, Z, spec, kp, I, &szz);
        const double fxz = (X->n > 0 && Z->n > 0) ? sxz.F : 0.0;
        const double fxx = X->n > 0 ? sxx.F : 0.0, fzz = Z->n > 0 ? szz.F : 0.0;
        // sqrt of the product: when the three sums coincide (the moved f_Z is
        // f_X) the quotient is exactly 1, as sqrt(fl(F * F)) == F
        *cos_theta = (fxx > 0.0 && fzz > 0.0) ? fxz / std::sqrt(fxx * fzz) : 0.0;
        if (sums) {
            sums[0] = fxz;
            sums[1] = fxx;
            sums[2] = fzz;
        }
    });
}

cvo_status cvo_align(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                     const cvo_align_params *ap, const double T_init[12], double T_out[12],
                     cvo_align_report *report, double *trace)
{
    return guarded(h, [&] {
        check_spec(spec);
        const int D = spec_dim(spec);
        check_cloud(X, D, "X");
        check_cloud(Z, D, "Z");
        check_align_params(ap);
        check_pose(T_init);
        require(T_out != nullptr && report != nullptr, "T_out / report is NULL");
        if (X->n == 0 || Z->n == 0) {
            std::memcpy(T_out, T_init, sizeof(double) * 12);
            PairState s = init_state(T_init, ap->ell_init);
            s.status = ST_NO_OVERLAP;
            fill_report(s, report);
            return;
        }
        std::vector<PairState> fin;
        align_many(h, {to_ptrs(X)}, {to_ptrs(Z)}, spec, {*ap}, {T_init}, fin, trace, false);
        std::memcpy(T_out, fin[0].T, sizeof(double) * 12);
        fill_report(fin[0], report);
    });
}

cvo_status cvo_align_replay(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                            const cvo_align_params *ap, const double T_init[12], const double *ell_sched,
                            int64_t n, double T_out[12], cvo_align_report *report, double *trace)
{
    return guarded(h, [&] {
        check_spec(spec);
        const int D = spec_dim(spec);
        check_cloud(X, D, "X");
        check_cloud(Z, D, "Z");
        check_align_params(ap);
        check_pose(T_init);
        require(T_out != nullptr && report != nullptr, "T_out / report is NULL");
        require(ell_sched != nullptr && n >= 1, "the schedule needs at least one lengthscale");
        for (int64_t i = 0; i < n; ++i)
            require(std::isfinite(ell_sched[i]) && ell_sched[i] > 0.0, "schedule lengthscales must be finite and > 0");
        cvo_align_params rp = *ap;
        rp.ell_init = ell_sched[0];
        rp.max_iter = n;
        rp.fixed_iters = 0;
        if (X->n == 0 || Z->n == 0) {
            std::memcpy(T_out, T_init, sizeof(double) * 12);
            PairState s = init_state(T_init, rp.ell_init);
            s.status = ST_NO_OVERLAP;
            fill_report(s, report);
            return;
        }
        double *d_sched = h->get_t<double>("replay.ell", (size_t)n);
        h->upload(d_sched, ell_sched, sizeof(double) * (size_t)n);
        std::vector<PairState> fin;
        align_many(h, {to_ptrs(X)}, {to_ptrs(Z)}, spec, {rp}, {T_init}, fin, trace, false, d_sched, n);
        std::memcpy(T_out, fin[0].T, sizeof(double) * 12);
        fill_report(fin[0], report);
    });
}

cvo_status cvo_align_batched(cvo_handle h, int32_t B, const cvo_cloud *X, const cvo_cloud *Z,
                             const cvo_feature_spec *spec, const cvo_align_params *params, int32_t nparams,
                             const double *T_init, double *T_out, cvo_align_report *reports)
{
    return guarded(h, [&] {
        require(B >= 1, "B must be >= 1");
        require(X && Z && params && T_init && T_out && reports, "NULL argument");
        require(nparams == 1 || nparams == B, "nparams must be 1 or B");
        check_spec(spec);
        const int D = spec_dim(spec);
        std::vector<CloudPtrs> xs(B), zs(B);
        std::vector<cvo_align_params> prm(B);
        std::vector<const double *> T0(B);
        for (int b = 0; b < B; ++b) {
            check_cloud(&X[b], D, "X");
            check_cloud(&Z[b], D, "Z");
            prm[b] = params[nparams == 1 ? 0 : b];
            check_align_params(&prm[b]);
            require(prm[b].kappa == prm[0].kappa && prm[b].sigma == prm[0].sigma,
                    "kappa and sigma must be shared by all pairs of a batch");
            T0[b] = T_init + 12 * b;
            check_pose(T0[b]);
            xs[b] = to_ptrs(&X[b]);
            zs[b] = to_ptrs(&Z[b]);
        }
        // the whole batched call runs on the library's own stream, ordered
        // after everything already enqueued on the caller's stream
        std::vector<PairState> fin;
        hipStream_t user = h->stream;
        HIP_OK(hipStreamSynchronize(user));
        h->stream = h->capture_stream();
        try {
            align_many(h, xs, zs, spec, prm, T0, fin, nullptr, true);
        } catch (...) {
            h->stream = user;
            throw;
        }
        HIP_OK(hipStreamSynchronize(h->stream));
        h->stream = user;
        for (int b = 0; b < B; ++b) {
            std::memcpy(T_out + 12 * b, fin[b].T, sizeof(double) * 12);
            fill_report(fin[b], &reports[b]);
        }
    });
}

cvo_status cvo_odometry(cvo_handle h, int32_t F, const cvo_cloud *frames, const cvo_feature_spec *spec,
                        const cvo_align_params *first, const cvo_align_params *rest, double *T_rel,
                        cvo_align_report *reports)
{
    return guarded(h, [&] {
        require(F >= 2, "a sequence needs at least two frames");
        require(frames && first && rest && T_rel && reports, "NULL argument");
        check_spec(spec);
        const int D = spec_dim(spec);
        for (int k = 0; k < F; ++k)
            check_cloud(&frames[k], D, "frame");
        check_align_params(first);
        check_align_params(rest);
        // pair k: frame k fixed, frame k + 1 moving; warm start from pair k - 1
        double T[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
        for (int k = 0; k + 1 < F; ++k) {
            const cvo_align_params &ap = k == 0 ? *first : *rest;
            const cvo_cloud *X = &frames[k], *Z = &frames[k + 1];
            PairState s;
            if (X->n == 0 || Z->n == 0) {
                s = init_state(T, ap.ell_init);
                s.status = ST_NO_OVERLAP;
            } else {
                std::vector<PairState> fin;
                align_many(h, {to_ptrs(X)}, {to_ptrs(Z)}, spec, {ap}, {T}, fin, nullptr, false);
                s = fin[0];
            }
            std::memcpy(T, s.T, sizeof(double) * 12);
            std::memcpy(T_rel + 12 * k, T, sizeof(double) * 12);
            fill_report(s, &reports[k]);
        }
    });
}

cvo_status cvo_select_points(cvo_handle h, const uint8_t *gray, const float *depth, const float *feat,
                             int32_t width, int32_t height, int32_t D, const cvo_camera *cam, int32_t max_points,
                             float *xyz, float *feat_out, int64_t capacity, int16_t *score, int64_t *n_out,
                             int32_t *threshold_out)
{
    return guarded(h, [&] {
        require(cam && n_out && threshold_out, "NULL argument");
        require(width >= 0 && height >= 0, "width and height must be >= 0");
        const long long npix = (long long)width * height;
        require(npix < (1LL << 31), "width x height must be < 2^31");
        require(D >= 0 && D <= 256, "D must be in [0, 256]");
        require(std::isfinite(cam->fx) && std::isfinite(cam->fy) && cam->fx > 0.0 && cam->fy > 0.0,
                "fx and fy must be finite and > 0");
        require(std::isfinite(cam->cx) && std::isfinite(cam->cy), "cx and cy must be finite");
        require(std::isfinite(cam->depth_min) && std::isfinite(cam->depth_max) && cam->depth_min > 0.0 &&
                    cam->depth_min <= cam->depth_max,
                "need 0 < depth_min <= depth_max, both finite");
        require(max_points >= 0 && capacity >= max_points, "need 0 <= max_points <= capacity");
        require(npix == 0 || (gray && depth), "gray / depth is NULL");
        require(npix == 0 || D == 0 || feat, "feat is NULL");
        require(max_points == 0 || xyz, "xyz is NULL");
        require(max_points == 0 || D == 0 || feat_out, "feat_out is NULL");
        *n_out = 0;
        *threshold_out = 0;
        if (npix == 0) return;
        const int nb = select_blocks(npix);
        SelectArgs a{};
        a.gray = gray;
        a.depth = depth;
        a.feat = feat;
        a.W = width;
        a.H = height;
        a.D = D;
        a.dmin = (float)cam->depth_min;
        a.dmax = (float)cam->depth_max;
        a.fx = cam->fx;
        a.fy = cam->fy;
        a.cx = cam->cx;
        a.cy = cam->cy;
        a.cap = max_points;
        a.key = h->get_t<short>("sel.key", npix);
        a.score = score;
        a.hist = h->get_t<int>("sel.hist", 256);
        a.res = h->get_t<int>("sel.res", 2);
        a.bcount = h->get_t<int>("sel.bcount", nb);
        a.boff = h->get_t<int>("sel.boff", nb);
        a.bsum = h->get_t<int>("sel.bsum", nb / 2048 + 2);
        a.xyz = xyz;
        a.fout = feat_out;
        HIP_OK(hipMemsetAsync(a.hist, 0, 256 * sizeof(int), h->stream));
        launch_select(a, h->stream);
        h->check_launch("point selection");
        int res[2];
        h->download(res, a.res, sizeof(res));
        *threshold_out = res[0];
        *n_out = res[1];
    });
}

cvo_status cvo_inner_product_backward(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z,
                                      const cvo_feature_spec *spec, const cvo_kernel_params *kp, const double T[12],
                                      double gF, float *dX, float *dZ, float *dU, float *dV, double *dEll)
{
    return guarded(h, [&] {
        check_spec(spec);
        const int D = spec_dim(spec);
        check_cloud(X, D, "X");
        check_cloud(Z, D, "Z");
        check_kp(kp);
        check_pose(T);
        require(std::isfinite(gF), "gF must be finite");
        if (D == 0) { dU = nullptr; dV = nullptr; }
        const long long N = X->n, M = Z->n;
        if (N == 0 || M == 0) {
            if (dX && N) HIP_OK(hipMemsetAsync(dX, 0, sizeof(float) * 3 * N, h->stream));
            if (dU && N) HIP_OK(hipMemsetAsync(dU, 0, sizeof(float) * D * N, h->stream));
            if (dZ && M) HIP_OK(hipMemsetAsync(dZ, 0, sizeof(float) * 3 * M, h->stream));
            if (dV && M) HIP_OK(hipMemsetAsync(dV, 0, sizeof(float) * D * M, h->stream));
            HIP_OK(hipStreamSynchronize(h->stream));
            if (dEll) *dEll = 0.0;
            return;
        }
        const FeatLayout lay = make_layout(spec, kp->sigma);
        const double rc = kp->kappa * kp->ell;
        PairState s0 = init_state(T, kp->ell);
        PairState *d_state = h->get_t<PairState>("bstate", 1);
        h->upload(d_state, &s0, sizeof(PairState));
        // target side: queries Z (pose T) against the X grid
        if (dZ || dV || dEll) {
            GridView gx = build_grid(h, "fx", {to_ptrs(X)}, {rc}, lay, {fixed_shape(h)});
            ClusterView cz = build_clusters(h, "fz", {to_ptrs(Z)}, {rc}, lay, {fixed_shape(h)});
            Plan pl = make_plan(h, "bp", cz, gx, d_state, 0, kp->kappa);
            Moments m = moments(h, "bm", pl.nslots, lay.d4, true);
            PairPassArgs a = pass_args(cz, gx, d_state, 0, lay.sig2, kp->kappa, m, pl);
            run_pair_pass(h, a, lay, 1);
            BackwardArgs ba;
            std::memset(&ba, 0, sizeof(ba));
            ba.map = slot_map(pl);
            ba.qperm = cz.perm;
            ba.D = m.D;
            ba.G = m.G;
            ba.state = d_state;
            ba.pose_is_inverse = 0;
            ba.lay = lay;
            ba.gF = gF;
            ba.dxyz = dZ;
            ba.dfeat = dV;
            ba.src_feat = Z->feat;
            ba.n = M;
            launch_backward_finish(ba, h->stream);
            if (dEll) {
                double *d_sum = h->get_t<double>("bsum", 1);
                launch_sum_doubles(m.L, pl.nslots, d_sum, h->stream);
                double sl = 0.0;
                h->download(&sl, d_sum, sizeof(double));
                const double ascale = kLog2e / (2.0 * kp->ell * kp->ell);
                *dEll = gF * sl / (ascale * kp->ell * kp->ell * kp->ell);
            }
            h->check_launch("backward (target side)");
        }
        // source side: queries X (pose T^-1) against the Z grid
        if (dX || dU) {
            GridView gz = build_grid(h, "rz", {to_ptrs(Z)}, {rc}, lay, {fixed_shape(h)});
            ClusterView cx = build_clusters(h, "rx", {to_ptrs(X)}, {rc}, lay, {fixed_shape(h)});
            Plan pl = make_plan(h, "bq", cx, gz, d_state, 1, kp->kappa);
            Moments m = moments(h, "bm2", pl.nslots, lay.d4, true);
            PairPassArgs a = pass_args(cx, gz, d_state, 1, lay.sig2, kp->kappa, m, pl);
            run_pair_pass(h, a, lay, 1);
            BackwardArgs ba;
            std::memset(&ba, 0, sizeof(ba));
            ba.map = slot_map(pl);
            ba.qperm = cx.perm;
            ba.D = m.D;
            ba.G = m.G;
            ba.state = d_state;
            ba.pose_is_inverse = 1;
            ba.lay = lay;
            ba.gF = gF;
            ba.dxyz = dX;
            ba.dfeat = dU;
            ba.src_feat = X->feat;
            ba.n = N;
            launch_backward_finish(ba, h->stream);
            h->check_launch("backward (source side)");
        }
        HIP_OK(hipStreamSynchronize(h->stream));
        if (h->profiling) h->harvest_events();
    });
}

cvo_status cvo_get_tuning(cvo_handle h, cvo_tuning *out)
{
    if (!h || !out) return CVO_ERR_INVALID_ARGUMENT;
    *out = h->tuning;
    return CVO_OK;
}

cvo_status cvo_set_tuning(cvo_handle h, const cvo_tuning *in)
{
    return guarded(h, [&] {
        require(in != nullptr, "tuning is NULL");
        require(in->cluster_max == 8 || in->cluster_max == 16 || in->cluster_max == 32 || in->cluster_max == 64,
                "cluster_max must be 8, 16, 32 or 64");
        require(in->cell_factor >= 0.25 && in->cell_factor <= 4.0, "cell_factor out of [0.25, 4]");
        require(in->cluster_factor >= 0.05 && in->cluster_factor <= 2.0, "cluster_factor out of [0.05, 2]");
        require(in->rebuild_ratio > 0.0 && in->rebuild_ratio <= 1.0, "rebuild_ratio out of (0, 1]");
        require(in->unroll >= 1 && in->unroll <= 64, "unroll out of [1, 64]");
        require(in->piece_work >= 256 && in->piece_work <= (1 << 24), "piece_work out of [256, 2^24]");
        require(in->adaptive == 0 || in->adaptive == 1, "adaptive must be 0 or 1");
        require(in->cluster_rule == CVO_CLUSTER_OCTREE || in->cluster_rule == CVO_CLUSTER_CHUNKS,
                "cluster_rule must be CVO_CLUSTER_OCTREE or CVO_CLUSTER_CHUNKS");
        h->tuning = *in;
    });
}

cvo_status cvo_set_profiling(cvo_handle h, int32_t enable)
{
    if (!h) return CVO_ERR_INVALID_ARGUMENT;
    h->profiling = enable != 0;
    h->timing = cvo_timing{0, 0.0, 0, 0, 0, 0, 0, 0, 0};
    return CVO_OK;
}

cvo_status cvo_get_timing(cvo_handle h, cvo_timing *out)
{
    if (!h || !out) return CVO_ERR_INVALID_ARGUMENT;
    *out = h->timing;
    return CVO_OK;
}

cvo_status cvo_autotune(cvo_handle h, const cvo_cloud *X, const cvo_cloud *Z, const cvo_feature_spec *spec,
                        const cvo_kernel_params *kp, const double T[12], cvo_tuning *chosen)
{
    return guarded(h, [&] {
        check_spec(spec);
        const int D = spec_dim(spec);
        check_cloud(X, D, "X");
        check_cloud(Z, D, "Z");
        check_kp(kp);
        check_pose(T);
        require(X->n > 0 && Z->n > 0, "autotune needs two non-empty clouds");
        const FeatLayout lay = make_layout(spec, kp->sigma);
        auto bucket = [](long long n) { return bits_for((unsigned long long)std::max(n, 1LL)); };
        const std::string key = std::to_string(bucket(X->n)) + "/" + std::to_string(bucket(Z->n)) + "/" +
                                std::to_string(D) + "/" + std::to_string((int)std::floor(std::log2(kp->ell) * 2));
        auto it = h->tune_cache.find(key);
        if (it != h->tune_cache.end()) {
            const cvo_tuning t = it->second;
            h->tuning.cluster_max = t.cluster_max;
            h->tuning.cell_factor = t.cell_factor;
            h->tuning.cluster_factor = t.cluster_factor;
            h->tuning.cluster_rule = t.cluster_rule;
            if (chosen) *chosen = h->tuning;
            return;
        }
        const cvo_tuning base = h->tuning;
        const bool prof = h->profiling;
        const cvo_timing saved = h->timing;
        h->profiling = false;
        cvo_tuning best = base;
        float best_ms = INFINITY;
        double npairs = -1.0;
        try {
            // chunk clusters only (the octree rule ties with them at best), with
            // the finer cells and tighter clusters that the densest bands favour
            for (int rule : {CVO_CLUSTER_CHUNKS})
                for (int cm : {16, 32, 64})
                    for (double cell : {0.35, 0.5, 1.0})
                        for (double cf : {0.3, 0.5, 1.0, 1.5}) {
                            cvo_tuning t = base;
                            t.cluster_rule = rule;
                            t.cluster_max = cm;
                            t.cell_factor = cell;
                            t.cluster_factor = cf;
                            h->tuning = t;
                            Problem p;
                            p.kappa = kp->kappa;
                            p.lay = lay;
                            p.sig2 = p.lay.sig2;
                            PairState s0 = init_state(T, kp->ell);
                            AlignConst ac = const_for(nullptr, X->n, Z->n);
                            setup_problem(h, p, {to_ptrs(X)}, {to_ptrs(Z)}, {s0}, {ac});
                            PairPassArgs a = pass_args(p.clus, p.grid, p.d_state, 0, p.sig2, p.kappa, p.mom, p.plan);
                            if (npairs < 0.0) {
                                // the evaluation's pair count sets its density class
                                enqueue_iteration(h, p, 0, nullptr, 0, false);
                                PairState st;
                                h->download(&st, p.d_state, sizeof(PairState));
                                npairs = st.n_pairs;
                            }
                            hipEvent_t e0 = h->event(), e1 = h->event();
                            std::vector<float> ms;
                            for (int rep = 0; rep < 4; ++rep) {
                                HIP_OK(hipEventRecord(e0, h->stream));
                                if (!launch_pair_pass(a, p.lay, 0, h->stream))
                                    throw CvoError(CVO_ERR_UNSUPPORTED, "no compiled pair kernel for the feature layout");
                                HIP_OK(hipEventRecord(e1, h->stream));
                                HIP_OK(hipEventSynchronize(e1));
                                float v = 0.f;
                                HIP_OK(hipEventElapsedTime(&v, e0, e1));
                                if (rep > 0) ms.push_back(v);
                            }
                            h->ev_free.push_back(e0);
                            h->ev_free.push_back(e1);
                            std::sort(ms.begin(), ms.end());
                            const float med = ms[ms.size() / 2];
                            if (med < best_ms) {
                                best_ms = med;
                                best = t;
                            }
                        }
        } catch (...) {
            h->tuning = base;
            h->profiling = prof;
            h->timing = saved;
            throw;
        }
        h->profiling = prof;
        h->timing = saved;
        // the winner becomes the one-shot shape and its density class's shape
        cvo_tuning out = base;
        out.cluster_rule = best.cluster_rule;
        out.cluster_max = best.cluster_max;
        out.cell_factor = best.cell_factor;
        out.cluster_factor = best.cluster_factor;
        h->tuning = out;
        h->tune_cache[key] = out;
        double t3[3];
        class_thresholds(lay, t3);
        const int cls = density_class(npairs / (double)Z->n, t3);
        h->class_shape[{light_layout(lay) ? 1 : 0, cls}] =
            cvo_context::Shape{out.cluster_max, out.cell_factor, out.cluster_factor, out.cluster_rule};
        if (chosen) *chosen = out;
    });
}

cvo_status cvo_clear_tuning(cvo_handle h)
{
    if (!h) return CVO_ERR_INVALID_ARGUMENT;
    h->class_shape.clear();
    h->tune_cache.clear();
    return CVO_OK;
}

cvo_status cvo_save_tuning(cvo_handle h, const char *path)
{
    return guarded(h, [&] {
        require(path != nullptr, "path is NULL");
        FILE *f = std::fopen(path, "w");
        require(f != nullptr, std::string("cannot open ") + path + " for writing");
        std::fprintf(f, "cvo-tuning 1\n");
        for (const auto &kv : h->class_shape)
            std::fprintf(f, "class %d %d %d %.17g %.17g %d\n", kv.first.first, kv.first.second, kv.second.cluster_max,
                         kv.second.cell_factor, kv.second.cluster_factor, kv.second.rule);
        for (const auto &kv : h->tune_cache)
            std::fprintf(f, "oneshot %s %d %.17g %.17g %d\n", kv.first.c_str(), kv.second.cluster_max,
                         kv.second.cell_factor, kv.second.cluster_factor, kv.second.cluster_rule);
        const bool ok = std::fclose(f) == 0;
        require(ok, std::string("writing ") + path + " failed");
    });
}

cvo_status cvo_load_tuning(cvo_handle h, const char *path)
{
    return guarded(h, [&] {
        require(path != nullptr, "path is NULL");
        FILE *f = std::fopen(path, "r");
        require(f != nullptr, std::string("cannot open ") + path);
        auto valid = [](int cm, double cell, double cf, int rule) {
            return (cm == 8 || cm == 16 || cm == 32 || cm == 64) && cell >= 0.25 && cell <= 4.0 && cf >= 0.05 &&
                   cf <= 2.0 && (rule == CVO_CLUSTER_OCTREE || rule == CVO_CLUSTER_CHUNKS);
        };
        std::map<std::pair<int, int>, cvo_context::Shape> cls_tab;
        std::map<std::string, cvo_tuning> one;
        char line[512];
        bool header = false, bad = false;
        while (std::fgets(line, sizeof(line), f)) {
            int a = 0, b = 0, cm = 0, rule = 0, ver = 0;
            double cell = 0.0, cf = 0.0;
            char key[256];
            if (!header) {
                header = std::sscanf(line, "cvo-tuning %d", &ver) == 1 && ver == 1;
                if (!header) { bad = true; break; }
            } else if (std::sscanf(line, "class %d %d %d %lf %lf %d", &a, &b, &cm, &cell, &cf, &rule) == 6) {
                if (!valid(cm, cell, cf, rule) || (a != 0 && a != 1) || b < 0 || b > 3) { bad = true; break; }
                cls_tab[{a, b}] = cvo_context::Shape{cm, cell, cf, rule};
            } else if (std::sscanf(line, "oneshot %255s %d %lf %lf %d", key, &cm, &cell, &cf, &rule) == 5) {
                if (!valid(cm, cell, cf, rule)) { bad = true; break; }
                cvo_tuning t = h->tuning;
                t.cluster_max = cm;
                t.cell_factor = cell;
                t.cluster_factor = cf;
                t.cluster_rule = rule;
                one[key] = t;
            } else if (line[0] != '\n') {
                bad = true;
                break;
            }
        }
        std::fclose(f);
        require(header && !bad, std::string(path) + " is not a cvo tuning file");
        for (auto &kv : cls_tab) h->class_shape[kv.first] = kv.second;
        for (auto &kv : one) h->tune_cache[kv.first] = kv.second;
    });
}

}  // extern "C"
