// Host driver and C ABI of libsqh (see include/sqh.h for the contract).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/sqh.h"
#include "sqh_kernels.hip"

using namespace sqh;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxGrid = kMaxChunks;  // workgroups of the persistent kernel (upper bound)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int64_t N, nsets, scap, rcap, W;
    size_t x[2], y[2], id[2];
    size_t gstart, sets, recs, rec_cid, segs[2], seg_cid[2], vstart[2];
    size_t bitmap, vidx, vlist, wprefix, slots, ctab, bar, err, stats, sv, info;
    int64_t vcap;
    size_t bytes;
};

bool make_layout(int64_t N, int64_t nsets, Layout& L)
{
    if (N < 0 || nsets < 1 || N > (int64_t)INT32_MAX - 2 || nsets > (int64_t)INT32_MAX / 8) return false;
    L.N = N;
    L.nsets = nsets;
    // Active segments: pass k+1 has at most min(2 S_k, V_k - S_k) <= 2N/3
    // (each child needs a point; each parent loses its farthest point); the
    // first table has at most 4 per set.
    const int64_t s_first = std::min<int64_t>(4 * nsets, N + 4);
    L.scap = std::max<int64_t>(s_first, (2 * N + 2) / 3) + 8;
    L.rcap = std::max<int64_t>(4 * nsets, 2 * L.scap) + 8;
    L.W = (N + 63) / 64 + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    for (int b = 0; b < 2; ++b) {
        L.x[b] = take(sizeof(float) * (size_t)std::max<int64_t>(N, 1));
        L.y[b] = take(sizeof(float) * (size_t)std::max<int64_t>(N, 1));
        L.id[b] = take(sizeof(int) * (size_t)std::max<int64_t>(N, 1));
    }
    L.gstart = take(sizeof(int) * (size_t)(nsets + 1));
    L.sets = take(sizeof(SetInfo) * (size_t)nsets);
    L.recs = take(sizeof(Seg) * (size_t)L.rcap);
    L.rec_cid = take(sizeof(int) * (size_t)L.rcap);
    for (int b = 0; b < 2; ++b) {
        L.segs[b] = take(sizeof(Seg) * (size_t)L.scap);
        L.seg_cid[b] = take(sizeof(int) * (size_t)L.scap);
        L.vstart[b] = take(sizeof(int) * (size_t)(L.scap + 1));
    }
    L.bitmap = take(sizeof(uint64_t) * (size_t)L.W);
    L.vidx = take(sizeof(int) * (size_t)std::max<int64_t>(N, 1));
    L.vcap = std::min<int64_t>(N + 8, kSmallHull);
    L.vlist = take(sizeof(int2) * (size_t)L.vcap);
    L.wprefix = take(sizeof(int) * (size_t)L.W);
    L.slots = take(sizeof(ChunkSlot<4>) * (size_t)kMaxGrid);
    L.ctab = take(sizeof(Pair) * (size_t)kMaxGrid);
    L.bar = take(sizeof(GridBar));
    L.err = take(sizeof(int));
    L.stats = take(sizeof(uint32_t) * 4 * kStatSlots);
    L.sv = take(sizeof(int) * 4);
    L.info = take(sizeof(HullInfo));
    L.bytes = o;
    return true;
}

}  // namespace

struct sqh_ctx {
    int device = 0;
    int cus = 0;
    int fp64 = 0;
    int grid = 0;  // co-resident workgroups of k_hull
    int trace = 0; // SQH_TRACE=1: per-workgroup timestamps in the info block
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    HullInfo* hinfo = nullptr;  // pinned host copy of the info block
    uint32_t* hstats = nullptr;  // pinned host copy of the counters
    int* herr = nullptr;
    sqh_stats stats{};
};

namespace {

#define HIP_OK(expr)                                       \
    do {                                                   \
        if ((expr) != hipSuccess) return SQH_EDEVICE;      \
    } while (0)

int run(sqh_ctx* ctx, const float* d_xy, int64_t N, int64_t nsets, const int64_t* d_set_off, int32_t* d_out,
        int64_t* d_out_off, int64_t out_cap, int64_t* h_total, void* d_ws, size_t ws_bytes, hipStream_t st)
{
    Layout L;
    if (!make_layout(N, nsets, L)) return SQH_EINVAL;
    if (!d_ws || ws_bytes < L.bytes) return SQH_ENOMEM;
    if (out_cap < 0) return SQH_EINVAL;
    if (N > 0 && !d_xy) return SQH_EINVAL;
    if (out_cap > 0 && !d_out) return SQH_EINVAL;
    HIP_OK(hipSetDevice(ctx->device));

    char* ws = static_cast<char*>(d_ws);
    auto at = [&](size_t off) { return static_cast<void*>(ws + off); };
    HullArgs a;
    a.xy = reinterpret_cast<const float2*>(d_xy);
    a.N = (int)N;
    a.G = (int)nsets;
    a.set_off = d_set_off;
    a.out = d_out;
    a.cap = out_cap;
    a.out_off = d_out_off;
    for (int b = 0; b < 2; ++b) {
        a.X[b] = static_cast<float*>(at(L.x[b]));
        a.Y[b] = static_cast<float*>(at(L.y[b]));
        a.I[b] = static_cast<int*>(at(L.id[b]));
        a.segs[b] = static_cast<Seg*>(at(L.segs[b]));
        a.seg_cid[b] = static_cast<int*>(at(L.seg_cid[b]));
        a.vstart[b] = static_cast<int*>(at(L.vstart[b]));
    }
    a.gstart = static_cast<int*>(at(L.gstart));
    a.sets = static_cast<SetInfo*>(at(L.sets));
    a.recs = static_cast<Seg*>(at(L.recs));
    a.rec_cid = static_cast<int*>(at(L.rec_cid));
    a.sv = static_cast<int*>(at(L.sv));
    a.bitmap = static_cast<uint64_t*>(at(L.bitmap));
    a.vidx = static_cast<int*>(at(L.vidx));
    a.vlist = static_cast<int2*>(at(L.vlist));
    a.vcap = (int)L.vcap;
    a.wprefix = static_cast<int*>(at(L.wprefix));
    a.W = (int)((N + 63) / 64);
    a.slots = at(L.slots);
    a.ctab = static_cast<Pair*>(at(L.ctab));
    a.bar = static_cast<GridBar*>(at(L.bar));
    a.err = static_cast<int*>(at(L.err));
    a.stats = static_cast<uint32_t*>(at(L.stats));
    a.info = static_cast<HullInfo*>(at(L.info));
    a.fp64 = ctx->fp64;
    a.timing = ctx->trace ? 2 : 1;

    HIP_OK(hipEventRecord(ctx->ev0, st));
    {
        const int64_t work = std::max<int64_t>(std::max<int64_t>(a.W, 4 * nsets), nsets + 1);
        const int grid = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (work + 255) / 256));
        k_reset<<<grid, 256, 0, st>>>(a);
        HIP_OK(hipGetLastError());
    }
    void* argv[] = {static_cast<void*>(&a)};
    HIP_OK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_hull), dim3(ctx->grid), dim3(kBlock), argv,
                                      0, st));
    HIP_OK(hipEventRecord(ctx->ev1, st));
    HIP_OK(hipMemcpyAsync(ctx->hinfo, a.info, ctx->trace ? sizeof(HullInfo) : offsetof(HullInfo, trace),
                          hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ctx->hstats, a.stats, sizeof(uint32_t) * 4 * kStatSlots, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ctx->herr, a.err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));

    const HullInfo& hi = *ctx->hinfo;
    const int e = *ctx->herr;
    sqh_stats& S = ctx->stats;
    S = sqh_stats{};
    S.points = N;
    S.passes = hi.passes;
    S.first_survivors = hi.first_v;
    for (int p = 0; p < hi.passes && p < kMaxInfoPasses; ++p) {
        S.survivors_total += hi.pass_v[p];
        S.max_segments = std::max<int64_t>(S.max_segments, hi.pass_s[p]);
        if (p < SQH_MAX_TIMED_PASSES) {
            S.pass_points[p] = hi.pass_v[p];
            S.pass_segments[p] = hi.pass_s[p];
        }
    }
    for (int i = 0; i < kStatSlots; ++i) {
        S.orient_evals += ctx->hstats[4 * i + 0];
        S.orient_exact += ctx->hstats[4 * i + 1];
        S.cmp_exact += ctx->hstats[4 * i + 2];
    }
    // device timestamps (100 MHz constant clock) at phase ends, block 0
    if (hi.nstamps > 1) {
        const double tick_ms = 1e-5;
        auto dt = [&](int i) { return (double)(hi.stamp[i] - hi.stamp[i - 1]) * tick_ms; };
        for (int i = 1; i < hi.nstamps && i < kMaxStamps; ++i) {
            const int tag = hi.stamp_tag[i];
            if (tag == 1) S.ms_seed += dt(i);
            else if (tag == 2) S.ms_split += dt(i);
            else if (tag == 3) S.ms_first += dt(i);
            else if (tag == 4) S.ms_emit += dt(i);
            else if (tag >= 100) {
                S.ms_pass += dt(i);
                if (tag - 100 < SQH_MAX_TIMED_PASSES) S.pass_ms[tag - 100] = dt(i);
            }
        }
    }
    const int64_t h = hi.h_total;
    S.hull_size = h;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) == hipSuccess) S.ms_total = ms;
    if (h_total) *h_total = h;
    if (e & (kErrNonFinite | kErrBounds)) return SQH_EINVAL;
    if (e) return SQH_EDEVICE;
    return h > out_cap ? SQH_ECAPACITY : SQH_OK;
}

}  // namespace

extern "C" {

int sqh_create(sqh_ctx** out, int device)
{
    if (!out) return SQH_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return SQH_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return SQH_EDEVICE;
    sqh_ctx* c = new (std::nothrow) sqh_ctx();
    if (!c) return SQH_ENOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return SQH_EDEVICE; }
    c->cus = prop.multiProcessorCount;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_hull), kBlock, 0) !=
            hipSuccess ||
        per_cu < 1) {
        delete c;
        return SQH_EDEVICE;
    }
    c->grid = std::min(kMaxGrid, per_cu * c->cus);
    {
        const char* t = getenv("SQH_TRACE");
        c->trace = t && t[0] == '1';
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->hinfo), sizeof(HullInfo), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->hstats), sizeof(uint32_t) * 4 * kStatSlots,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->herr), sizeof(int), hipHostMallocDefault) != hipSuccess) {
        sqh_destroy(c);
        return SQH_EDEVICE;
    }
    *out = c;
    return SQH_OK;
}

void sqh_destroy(sqh_ctx* c)
{
    if (!c) return;
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->hinfo) (void)hipHostFree(c->hinfo);
    if (c->hstats) (void)hipHostFree(c->hstats);
    if (c->herr) (void)hipHostFree(c->herr);
    delete c;
}

int sqh_set_precision(sqh_ctx* c, int mode)
{
    if (!c || (mode != SQH_FP32_FILTER && mode != SQH_FP64_ONLY)) return SQH_EINVAL;
    c->fp64 = mode == SQH_FP64_ONLY;
    return SQH_OK;
}

size_t sqh_workspace_bytes(int64_t n_total, int64_t n_sets)
{
    Layout L;
    if (!make_layout(n_total, n_sets, L)) return 0;
    return L.bytes;
}

int sqh_hull(sqh_ctx* c, const float* d_xy, int64_t n, int32_t* d_out, int64_t out_cap, int64_t* h_count,
             void* d_ws, size_t ws_bytes, void* stream)
{
    if (!c || !h_count || n < 0) return SQH_EINVAL;
    *h_count = 0;
    return run(c, d_xy, n, 1, nullptr, d_out, nullptr, out_cap, h_count, d_ws, ws_bytes,
               static_cast<hipStream_t>(stream));
}

int sqh_hull_batched(sqh_ctx* c, const float* d_xy, const int64_t* d_set_off, int64_t n_sets, int64_t n_total,
                     int32_t* d_out, int64_t* d_out_off, int64_t out_cap, int64_t* h_total, void* d_ws,
                     size_t ws_bytes, void* stream)
{
    if (!c || !d_set_off || !d_out_off || n_sets < 1 || n_total < 0) return SQH_EINVAL;
    if (h_total) *h_total = 0;
    return run(c, d_xy, n_total, n_sets, d_set_off, d_out, d_out_off, out_cap, h_total, d_ws, ws_bytes,
               static_cast<hipStream_t>(stream));
}

int sqh_get_trace(const sqh_ctx* c, uint64_t* out, int max_entries)
{
    if (!c || !out || max_entries < 0) return SQH_EINVAL;
    if (!c->trace) return 0;
    const int n = std::min(max_entries, c->grid * 8);
    for (int i = 0; i < n; ++i) out[i] = c->hinfo->trace[i / 8][i % 8];
    return n;
}

int sqh_get_stats(const sqh_ctx* c, sqh_stats* out)
{
    if (!c || !out) return SQH_EINVAL;
    *out = c->stats;
    return SQH_OK;
}

const char* sqh_strerror(int code)
{
    switch (code) {
    case SQH_OK: return "ok";
    case SQH_EINVAL: return "invalid argument (null pointer, size out of range or non-finite coordinate)";
    case SQH_ENOMEM: return "workspace too small";
    case SQH_ECAPACITY: return "hull larger than the output capacity";
    case SQH_EDEVICE: return "HIP runtime error or device fault report";
    case SQH_EBUSY: return "engine has no room for the request";
    case SQH_ENOTFOUND: return "no finished request";
    default: return "unknown error";
    }
}

}  // extern "C"
