// Host driver and C ABI of libsqh (see include/sqh.h for the contract).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/sqh.h"
#include "sqh_kernels.hip"

using namespace sqh;

namespace {

constexpr size_t kAlign = 256;
constexpr int kTile = kRows * 64 * kWaves;  // positions per tile of the segmented kernels
constexpr int kLBWords = 4;                 // max look-back words per tile and kind (k_first)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int64_t N, nsets, scap, rcap, W, ntcap;
    size_t x[2], y[2], id[2];
    size_t gstart, sets, recs, rec_cid, segs[2], seg_cid[2], vstart[2];
    size_t bitmap, vidx, wprefix, lb, err, stats, sv, total;
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
    const int64_t items = std::max<int64_t>(std::max<int64_t>(N, L.rcap), L.W);
    L.ntcap = (items + std::min(kTile, kScanTile) - 1) / std::min(kTile, kScanTile) + 1;
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
    L.wprefix = take(sizeof(int) * (size_t)L.W);
    L.lb = take(sizeof(uint64_t) * 2 * kLBWords * (size_t)L.ntcap);
    L.err = take(sizeof(int));
    L.stats = take(sizeof(uint32_t) * 4 * kStatSlots);
    L.sv = take(sizeof(int) * 4);
    L.total = take(sizeof(int));
    L.bytes = o;
    return true;
}

}  // namespace

struct sqh_ctx {
    int device = 0;
    int cus = 0;
    int fp64 = 0;
    int grid_seed = 0, grid_split = 0, grid_first = 0, grid_pass = 0, grid_table = 0, grid_emit = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    int* pinned = nullptr;  // host readback buffer
    sqh_stats stats{};
};

namespace {

template <class K>
int coop_grid(K kernel, int cus)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kernel), kBlock, 0) !=
        hipSuccess)
        return 0;
    return std::max(1, nb) * cus;
}

template <class K, class... Args>
hipError_t coop_launch(K kernel, int grid, hipStream_t s, Args... args)
{
    void* argv[] = {static_cast<void*>(&args)...};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kernel), dim3(std::max(1, grid)),
                                      dim3(kBlock), argv, 0, s);
}

int grid_for(int cap, int64_t items, int tile)
{
    const int64_t nt = (items + tile - 1) / tile;
    return (int)std::max<int64_t>(1, std::min<int64_t>(cap, nt));
}

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
    float* X[2] = {reinterpret_cast<float*>(ws + L.x[0]), reinterpret_cast<float*>(ws + L.x[1])};
    float* Y[2] = {reinterpret_cast<float*>(ws + L.y[0]), reinterpret_cast<float*>(ws + L.y[1])};
    int* I[2] = {reinterpret_cast<int*>(ws + L.id[0]), reinterpret_cast<int*>(ws + L.id[1])};
    int* gstart = reinterpret_cast<int*>(ws + L.gstart);
    SetInfo* sets = reinterpret_cast<SetInfo*>(ws + L.sets);
    Seg* recs = reinterpret_cast<Seg*>(ws + L.recs);
    int* rec_cid = reinterpret_cast<int*>(ws + L.rec_cid);
    Seg* segs[2] = {reinterpret_cast<Seg*>(ws + L.segs[0]), reinterpret_cast<Seg*>(ws + L.segs[1])};
    int* seg_cid[2] = {reinterpret_cast<int*>(ws + L.seg_cid[0]), reinterpret_cast<int*>(ws + L.seg_cid[1])};
    int* vstart[2] = {reinterpret_cast<int*>(ws + L.vstart[0]), reinterpret_cast<int*>(ws + L.vstart[1])};
    uint64_t* bitmap = reinterpret_cast<uint64_t*>(ws + L.bitmap);
    int* vidx = reinterpret_cast<int*>(ws + L.vidx);
    int* wprefix = reinterpret_cast<int*>(ws + L.wprefix);
    uint64_t* lb = reinterpret_cast<uint64_t*>(ws + L.lb);
    int* err = reinterpret_cast<int*>(ws + L.err);
    uint32_t* stats = reinterpret_cast<uint32_t*>(ws + L.stats);
    int* sv = reinterpret_cast<int*>(ws + L.sv);  // {S0, V0, S1, V1}
    int* total = reinterpret_cast<int*>(ws + L.total);
    const size_t lb_bytes = sizeof(uint64_t) * 2 * kLBWords * (size_t)L.ntcap;
    const int n = (int)N, G = (int)nsets, ntcap = (int)L.ntcap, fp64 = ctx->fp64;
    int* pin = ctx->pinned;

    ctx->stats = sqh_stats{};
    ctx->stats.points = N;
    HIP_OK(hipEventRecord(ctx->ev0, st));
    HIP_OK(hipMemsetAsync(err, 0, sizeof(int), st));
    HIP_OK(hipMemsetAsync(stats, 0, sizeof(uint32_t) * 4 * kStatSlots, st));
    HIP_OK(hipMemsetAsync(bitmap, 0, sizeof(uint64_t) * (size_t)L.W, st));
    HIP_OK(hipMemsetAsync(recs, 0, sizeof(Seg) * (size_t)(4 * nsets), st));
    if (d_set_off) {
        k_prep_sets<<<(G + 1 + 255) / 256, 256, 0, st>>>(d_set_off, G, N, gstart, err);
    } else {
        k_single_set<<<1, 64, 0, st>>>(gstart, n);
    }
    HIP_OK(hipGetLastError());

    // seed: lexmin / lexmax per set
    HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
    {
        PolSeed pol{reinterpret_cast<const float2*>(d_xy), gstart, sets, err};
        HIP_OK(coop_launch(k_tiles<PolSeed>, grid_for(ctx->grid_seed, N, kTile), st, pol, (const int*)nullptr, n,
                           (const int*)nullptr, G, ntcap, lb, err, stats));
    }
    HIP_OK(hipMemcpyAsync(pin, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (pin[0] & (kErrNonFinite | kErrBounds)) return SQH_EINVAL;
    if (pin[0]) return SQH_EDEVICE;

    // first split: side counts and farthest point per side
    HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
    {
        PolSplit pol{reinterpret_cast<const float2*>(d_xy), gstart, sets, bitmap, vidx, fp64};
        HIP_OK(coop_launch(k_tiles<PolSplit>, grid_for(ctx->grid_split, N, kTile), st, pol, (const int*)nullptr, n,
                           (const int*)nullptr, G, ntcap, lb, err, stats));
    }
    // first compaction into four child segments per set
    HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
    {
        PolFirst pol{reinterpret_cast<const float2*>(d_xy), gstart, sets, X[0], Y[0], I[0], recs, rec_cid, bitmap,
                     vidx, fp64};
        HIP_OK(coop_launch(k_tiles<PolFirst>, grid_for(ctx->grid_first, N, kTile), st, pol, (const int*)nullptr, n,
                           (const int*)nullptr, G, ntcap, lb, err, stats));
    }
    HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
    HIP_OK(coop_launch(k_table, grid_for(ctx->grid_table, 4 * nsets, kScanTile), st, (const Seg*)recs,
                       (const int*)rec_cid, (const int*)nullptr, 0, (int)(4 * nsets), segs[0], seg_cid[0], vstart[0],
                       sv, ntcap, lb, err));

    int cur = 0;
    for (int pass = 0;; ++pass) {
        HIP_OK(hipMemcpyAsync(pin, sv + 2 * cur, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        const int S = pin[0], V = pin[1];
        if (S <= 0) break;
        ctx->stats.passes += 1;
        ctx->stats.survivors_total += V;
        ctx->stats.max_segments = std::max<int64_t>(ctx->stats.max_segments, S);
        const int nxt = cur ^ 1;
        HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
        {
            PolPass pol{segs[cur], seg_cid[cur], vstart[cur], X[cur], Y[cur], I[cur], X[nxt], Y[nxt], I[nxt],
                        recs, rec_cid, bitmap, vidx, fp64};
            HIP_OK(coop_launch(k_tiles<PolPass>, grid_for(ctx->grid_pass, V, kTile), st, pol,
                               (const int*)(sv + 2 * cur + 1), 0, (const int*)(sv + 2 * cur), 0, ntcap, lb, err,
                               stats));
        }
        HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
        HIP_OK(coop_launch(k_table, grid_for(ctx->grid_table, 2 * (int64_t)S, kScanTile), st, (const Seg*)recs,
                           (const int*)rec_cid, (const int*)(sv + 2 * cur), 2, 0, segs[nxt], seg_cid[nxt],
                           vstart[nxt], sv + 2 * nxt, ntcap, lb, err));
        cur = nxt;
    }

    HIP_OK(hipMemsetAsync(lb, 0, lb_bytes, st));
    const int W = (int)((N + 63) / 64);
    HIP_OK(coop_launch(k_emit, grid_for(ctx->grid_emit, W, kScanTile), st, (const uint64_t*)bitmap, (const int*)vidx,
                       W, d_out, out_cap, wprefix, total, ntcap, lb, err));
    if (d_out_off) {
        k_out_offsets<<<(G + 1 + 255) / 256, 256, 0, st>>>(gstart, G, n, bitmap, wprefix, total, d_out_off);
        HIP_OK(hipGetLastError());
    }
    HIP_OK(hipEventRecord(ctx->ev1, st));
    HIP_OK(hipMemcpyAsync(pin, total, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(pin + 1, err, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(pin + 2, stats, sizeof(uint32_t) * 4 * kStatSlots, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const int64_t h = pin[0];
    const int e = pin[1];
    const uint32_t* sp = reinterpret_cast<const uint32_t*>(pin + 2);
    for (int i = 0; i < kStatSlots; ++i) {
        ctx->stats.orient_evals += sp[4 * i + 0];
        ctx->stats.orient_exact += sp[4 * i + 1];
        ctx->stats.cmp_exact += sp[4 * i + 2];
    }
    ctx->stats.hull_size = h;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) == hipSuccess) ctx->stats.ms_total = ms;
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
    c->grid_seed = coop_grid(k_tiles<PolSeed>, c->cus);
    c->grid_split = coop_grid(k_tiles<PolSplit>, c->cus);
    c->grid_first = coop_grid(k_tiles<PolFirst>, c->cus);
    c->grid_pass = coop_grid(k_tiles<PolPass>, c->cus);
    c->grid_table = coop_grid(k_table, c->cus);
    c->grid_emit = coop_grid(k_emit, c->cus);
    if (!c->grid_seed || !c->grid_split || !c->grid_first || !c->grid_pass || !c->grid_table || !c->grid_emit ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->pinned), 4096, hipHostMallocDefault) != hipSuccess) {
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
    if (c->pinned) (void)hipHostFree(c->pinned);
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
