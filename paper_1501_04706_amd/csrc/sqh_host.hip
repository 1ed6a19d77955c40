// Host driver and C ABI of libsqh (see include/sqh.h for the contract).
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <stddef.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <new>
#include <vector>
#include <deque>
#include <mutex>

#include "../../include/sqh.h"
#include "sqh_kernels.hip"
#include "sqh_stream.hip"
#include "sqh_engine.hip"
#include "sqh_diag.hip"

using namespace sqh;

namespace {

constexpr size_t kAlign = 256;
// Streaming passes enqueued per call: at most kStreamPassLaunches (each does
// nothing once the segment table no longer qualifies); a context enqueues as
// many as the previous call of the same size class needed when the
// streaming kernels finished that call, else all of them, plus one on few
// workgroups in case this call needs one more (a call that needs more than
// it got is finished by the passes kernel).
constexpr int kStreamPassLaunches = 8;
constexpr int kMaxLaunches = 16;
constexpr int kMaxGrid = kMaxChunks;  // workgroups of the persistent kernel (upper bound)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    int64_t N, nsets, scap, rcap, W;
    size_t x[2], y[2], id[2];
    size_t gstart, sets, recs, rec_cid, segs[2], seg_cid[2], vstart[2];
    size_t bitmap, vidx, vlist, wprefix, slots, ctab, bar, err, stats, sv, info;
    size_t ext, xy2, ids2, gs2, shist, stot, sws;
    int64_t vcap;
    size_t bytes;
};

// The status block read back after every call: the error word, the
// counters, the set and vertex counts and the info block are consecutive
// takes of every layout below; offsets from the error word.
struct StatusOffsets {
    size_t stats, info, bytes;
};
StatusOffsets status_offsets()
{
    StatusOffsets so;
    so.stats = align_up(sizeof(int));
    const size_t sv = so.stats + align_up(sizeof(uint32_t) * 4 * kStatSlots);
    so.info = sv + align_up(sizeof(int) * 4);
    so.bytes = so.info + sizeof(HullInfo);
    return so;
}

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
    L.slots = take(sizeof(ChunkSlot<8>) * (size_t)kMaxGrid);
    L.ctab = take(sizeof(Pair) * (size_t)kMaxGrid);
    L.bar = take(sizeof(GridBar));
    L.err = take(sizeof(int));
    L.stats = take(sizeof(uint32_t) * 4 * kStatSlots);
    L.sv = take(sizeof(int) * 4);
    L.info = take(sizeof(HullInfo));
    // pre-filter of a single hull: corners, the kept subset and its indices
    L.ext = take(sizeof(uint64_t) * 8 * (size_t)kMaxGrid);
    L.xy2 = take(sizeof(float2) * (size_t)std::max<int64_t>(N, 1));
    L.ids2 = take(sizeof(int) * (size_t)std::max<int64_t>(N, 1));
    L.gs2 = take(sizeof(int) * 2);
    // sorted-chain variant: bucket counts per workgroup and totals
    L.shist = take(sizeof(int) * (size_t)kSortBuckets * (size_t)kMaxGrid);
    L.stot = take(sizeof(int) * (size_t)kSortBuckets);
    // streaming path of one large set: partial results and pass state
    // (the streaming pass's records: one per tile of kPTile points and per segment)
    L.sws = take(N >= kStreamMin ? sizeof(StreamWs) + sizeof(PassRec) * (size_t)(N / kPTile + kSPassMaxS + 2) : 0);
    L.bytes = o;
    return true;
}

}  // namespace

// ---- allocation-free entry point: a file-scope device scratch array ------
//
// sqh_hull_noalloc runs single hulls of at most SQH_NOALLOC_MAX_POINTS points
// in this array instead of a caller workspace. In host code `g_scratch` only
// names the symbol; its device address (one copy per device) is looked up
// once per device with hipGetSymbolAddress while sqh_create has that device
// current, and only that address is ever passed to kernels.
constexpr size_t kScratchBytes = size_t(40) << 20;
static __device__ __align__(256) unsigned char g_scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchSlot {
    std::once_flag once;
    void* ptr = nullptr;
    int rc = SQH_EDEVICE;
};
ScratchSlot g_scratch_slot[kMaxDevices];

// Called with `device` current.
void scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    ScratchSlot& s = g_scratch_slot[device];
    std::call_once(s.once, [&s]() {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_scratch)) == hipSuccess && p) {
            s.ptr = p;
            s.rc = SQH_OK;
        }
    });
}

struct TuneEntry {
    int log2n;       // problem class: floor(log2(max(n_total, 1)))
    int grid;        // workgroups of the persistent kernel
    int tail;        // tail threshold (points) below which workgroup 0 finishes alone
    int stream = 1;  // 1: large single hulls take the streaming path; 0: the persistent kernel
    int sgrid = 0;   // workgroups of the streaming kernels (0: twice the co-resident grid, at most kMaxSGrid)
};

struct sqh_ctx {
    int device = 0;
    int cus = 0;
    int fp64 = 0;
    int line = 1;      // the streaming path may use the static line filter
    int max_grid = 0;  // co-resident workgroups of k_hull
    int trace = 0;     // SQH_TRACE=1: per-workgroup timestamps in the info block
    hipEvent_t ev0 = nullptr, evk = nullptr, ev1 = nullptr;
    unsigned char* hstatus = nullptr;  // pinned host copy of the status block (status_offsets)
    HullInfo* hinfo = nullptr;   // ... its info block
    uint32_t* hstats = nullptr;  // ... its counters
    int* herr = nullptr;         // ... its error word
    sqh_stats stats{};
    static constexpr int kMaxTune = 40;
    TuneEntry tune[kMaxTune];
    int ntune = 0;
    int engine_grid = 0;  // workgroups of an engine step (0: all but 1/8 of the co-resident ones)
    int prefilter = 0;    // SQH_PREFILTER_*
    int variant = 0;      // SQH_VARIANT_*
    int stream = 1;       // large single hulls take the streaming path (SQH_STREAM=0 turns it off)
    int spass_used[64];   // per size class: streaming passes the last call ran (-1: none yet)
    // per-launch timing (sqh_set_launch_timing): events before and after
    // each kernel of the last call, and the kernels' names
    static constexpr int kMaxTimed = 24;
    int ltiming = 0;
    char lonly[32] = {};  // time only the launches of this kernel ("": all)
    int nl = 0;
    hipEvent_t lev[2 * kMaxTimed] = {};
    const char* lname[kMaxTimed] = {};
    sqh_ctx() { for (int& v : spass_used) v = -1; }
};

struct sqh_graph {
    sqh_ctx* ctx = nullptr;
    HullArgs args{};
    int64_t N = 0, out_cap = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

#define HIP_OK(expr)                                       \
    do {                                                   \
        if ((expr) != hipSuccess) return SQH_EDEVICE;      \
    } while (0)

int log2_class(int64_t n)
{
    int k = 0;
    while (k < 62 && (int64_t(1) << (k + 1)) <= std::max<int64_t>(n, 1)) ++k;
    return k;
}

// Launch shape for a problem of n_total points: the tuned entry of the
// nearest problem class, else all co-resident workgroups and the built-in
// tail threshold.
TuneEntry pick_tuning(const sqh_ctx* ctx, int64_t n_total)
{
    TuneEntry t{log2_class(n_total), ctx->max_grid, kTailPoints};
    int best = 1 << 30;
    for (int i = 0; i < ctx->ntune; ++i) {
        const int d = std::abs(ctx->tune[i].log2n - t.log2n);
        if (d < best) {
            best = d;
            t.grid = ctx->tune[i].grid;
            t.tail = ctx->tune[i].tail;
            t.stream = ctx->tune[i].stream;
            t.sgrid = ctx->tune[i].sgrid;
        }
    }
    t.grid = std::max(1, std::min(t.grid, ctx->max_grid));
    return t;
}

// Validate the call and fill the kernel arguments over the caller's workspace.
int setup(sqh_ctx* ctx, const float* d_xy, int64_t N, int64_t nsets, const int64_t* d_set_off, int32_t* d_out,
          int64_t* d_out_off, int64_t out_cap, void* d_ws, size_t ws_bytes, const TuneEntry& tu, HullArgs& a,
          int& reset_grid)
{
    Layout L;
    if (!make_layout(N, nsets, L)) return SQH_EINVAL;
    if (!d_ws || ws_bytes < L.bytes) return SQH_ENOMEM;
    if (out_cap < 0) return SQH_EINVAL;
    if (N > 0 && !d_xy) return SQH_EINVAL;
    if (out_cap > 0 && !d_out) return SQH_EINVAL;
    if (tu.grid < 1 || tu.grid > ctx->max_grid || tu.grid > kMaxGrid || tu.tail < 0) return SQH_EINVAL;
    HIP_OK(hipSetDevice(ctx->device));

    char* ws = static_cast<char*>(d_ws);
    auto at = [&](size_t off) { return static_cast<void*>(ws + off); };
    a = HullArgs{};
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
    a.timing = ctx->trace == 1 ? 2 : (ctx->trace == 2 ? 3 : 1);
    a.tail_points = tu.tail;
    a.prefilter = nsets == 1 ? ctx->prefilter : 0;
    a.sorted = nsets == 1 && ctx->variant == SQH_VARIANT_SORTED ? 1 : 0;
    a.shist = static_cast<int*>(at(L.shist));
    a.stot = static_cast<int*>(at(L.stot));
    a.ext = static_cast<uint64_t*>(at(L.ext));
    a.xy2 = static_cast<float2*>(at(L.xy2));
    a.ids2 = static_cast<int*>(at(L.ids2));
    a.gs2 = static_cast<int*>(at(L.gs2));
    a.sws = at(L.sws);
    a.sdone = N >= kStreamMin ? static_cast<StreamWs*>(a.sws)->done : nullptr;
    // one large set in plain mode, 16-byte aligned input: the streaming path
    a.stream = (ctx->stream && tu.stream && nsets == 1 && N >= kStreamMin && !a.prefilter && !a.sorted &&
                (reinterpret_cast<uintptr_t>(d_xy) & 15u) == 0)
                   ? 1
                   : 0;
    a.start = a.stream ? static_cast<StreamWs*>(a.sws)->state : nullptr;
    a.spasses = kStreamPassLaunches;
    a.line_ok = ctx->line;
    const int64_t work = std::max<int64_t>(std::max<int64_t>(a.W, 4 * nsets), nsets + 1);
    reset_grid = (int)std::min<int64_t>(2048, std::max<int64_t>(1, (work + 255) / 256));
    return SQH_OK;
}

// The cooperative launches of one call after the workspace reset: the
// pre-filter where it runs, then the persistent kernel (the instance that
// reads the pre-filter's subset only where the pre-filter runs), or for the
// sorted-chain variant its first phases, k_sort and its passes.
inline bool pre_runs(const HullArgs& a) { return a.prefilter && a.G == 1 && a.N > 0; }

// One launch of a call: cooperative launches take `grid` workgroups of
// kBlock threads; the streaming kernels, which never wait for another
// workgroup, are ordinary launches of 2 * grid workgroups of kSBlock threads
// (ordinary launches start without the cooperative launch's queue round trip).
struct Launch {
    const void* f;
    int coop;
    int light;  // a streaming pass launched on few workgroups (in case one more is needed)
};
constexpr int kLightGrid = 64;

// The streaming path ends with k_stail; the passes kernel follows it in the
// same sequence when `fallback` is set (graphs), else only when the hull is
// not complete after it (sqh_hull checks the device's flag).
inline int call_launches(const HullArgs& a, Launch (&L)[kMaxLaunches], bool fallback = true)
{
    int n = 0;
    auto add = [&](const void* f, int coop, int light = 0) {
        L[n].f = f; L[n].coop = coop; L[n].light = light; ++n;
    };
    if (a.stream) {
        add(reinterpret_cast<const void*>(k_sseed), 0);
        add(reinterpret_cast<const void*>(k_ssplit), 0);
        add(reinterpret_cast<const void*>(k_sfirst<true>), 0);
        add(reinterpret_cast<const void*>(k_sfirst<false>), 0);
        for (int i = 0; i < a.spasses; ++i) add(reinterpret_cast<const void*>(k_spass), 0);
        if (!fallback && a.spasses < kStreamPassLaunches) add(reinterpret_cast<const void*>(k_spass), 0, 1);
        add(reinterpret_cast<const void*>(k_stail), 0);
        if (fallback) add(reinterpret_cast<const void*>(k_hull<kHullPasses>), 1);
        return n;
    }
    if (pre_runs(a)) add(reinterpret_cast<const void*>(k_prefilter), 1);
    if (a.sorted && a.G == 1) {
        add(reinterpret_cast<const void*>(k_hull<kHullFirst>), 1);
        add(reinterpret_cast<const void*>(k_sort), 1);
        add(reinterpret_cast<const void*>(k_hull<kHullPasses>), 1);
    } else {
        add(pre_runs(a) ? reinterpret_cast<const void*>(k_hull<kHullPre>)
                        : reinterpret_cast<const void*>(k_hull<kHullPlain>),
            1);
    }
    return n;
}
// Streaming kernels: a tuned grid applies to all of them; by default the
// first compaction runs two workgroups per co-resident one (its tiles wait
// on a reservation round trip, which a second workgroup per compute unit
// hides) and the others one (fewer partials for the last workgroup to
// reduce: 35 us instead of 48 for the seed of 20M points).
inline dim3 launch_grid(const Launch& l, int grid, int sgrid)
{
    if (l.f == reinterpret_cast<const void*>(k_stail)) return dim3(1);
    if (l.light) return dim3(kLightGrid);
    if (l.coop) return dim3(grid);
    if (sgrid > 0) return dim3(std::min(sgrid, kMaxSGrid));
    const bool first = l.f == reinterpret_cast<const void*>(k_sfirst<true>) ||
                       l.f == reinterpret_cast<const void*>(k_sfirst<false>);
    return dim3(std::min(first ? 2 * grid : grid, kMaxSGrid));
}
inline dim3 launch_block(const Launch& l)
{
    return dim3(l.coop || l.f == reinterpret_cast<const void*>(k_stail) ? kBlock : kSBlock);
}

const char* kernel_name(const void* f)
{
    struct { const void* f; const char* name; } const names[] = {
        {reinterpret_cast<const void*>(k_sseed), "k_sseed"},
        {reinterpret_cast<const void*>(k_ssplit), "k_ssplit"},
        {reinterpret_cast<const void*>(k_sfirst<true>), "k_sfirst<line>"},
        {reinterpret_cast<const void*>(k_sfirst<false>), "k_sfirst<semistatic>"},
        {reinterpret_cast<const void*>(k_spass), "k_spass"},
        {reinterpret_cast<const void*>(k_stail), "k_stail"},
        {reinterpret_cast<const void*>(k_hull<kHullPlain>), "k_hull<plain>"},
        {reinterpret_cast<const void*>(k_hull<kHullPre>), "k_hull<prefiltered>"},
        {reinterpret_cast<const void*>(k_hull<kHullFirst>), "k_hull<first>"},
        {reinterpret_cast<const void*>(k_hull<kHullPasses>), "k_hull<passes>"},
        {reinterpret_cast<const void*>(k_prefilter), "k_prefilter"},
        {reinterpret_cast<const void*>(k_sort), "k_sort"},
    };
    for (const auto& e : names)
        if (e.f == f) return e.name;
    return "?";
}

// Per-launch timing: an event before and one after each timed kernel.
inline bool timed(const sqh_ctx* ctx, const char* name)
{
    return ctx->ltiming && ctx->nl < sqh_ctx::kMaxTimed && (!ctx->lonly[0] || strcmp(ctx->lonly, name) == 0);
}
inline int time_open(sqh_ctx* ctx, const char* name, hipStream_t st)
{
    if (timed(ctx, name)) HIP_OK(hipEventRecord(ctx->lev[2 * ctx->nl], st));
    return SQH_OK;
}
inline int time_close(sqh_ctx* ctx, const char* name, hipStream_t st)
{
    if (timed(ctx, name)) {
        HIP_OK(hipEventRecord(ctx->lev[2 * ctx->nl + 1], st));
        ctx->lname[ctx->nl++] = name;
    }
    return SQH_OK;
}

// Enqueue the workspace reset and the launches, bracketed by events.
int enqueue(sqh_ctx* ctx, HullArgs& a, int reset_grid, int grid, int sgrid, hipStream_t st, bool fallback = true)
{
    ctx->nl = 0;
    HIP_OK(hipEventRecord(ctx->ev0, st));
    if (time_open(ctx, "k_reset", st) != SQH_OK) return SQH_EDEVICE;
    k_reset<<<reset_grid, 256, 0, st>>>(a);
    HIP_OK(hipGetLastError());
    if (time_close(ctx, "k_reset", st) != SQH_OK) return SQH_EDEVICE;
    HIP_OK(hipEventRecord(ctx->evk, st));
    void* argv[] = {static_cast<void*>(&a)};
    Launch L[kMaxLaunches];
    const int nf = call_launches(a, L, fallback);
    for (int i = 0; i < nf; ++i) {
        if (time_open(ctx, kernel_name(L[i].f), st) != SQH_OK) return SQH_EDEVICE;
        const dim3 gd = launch_grid(L[i], grid, sgrid);
        if (L[i].coop) HIP_OK(hipLaunchCooperativeKernel(L[i].f, gd, launch_block(L[i]), argv, 0, st));
        else HIP_OK(hipLaunchKernel(L[i].f, gd, launch_block(L[i]), argv, 0, st));
        if (time_close(ctx, kernel_name(L[i].f), st) != SQH_OK) return SQH_EDEVICE;
    }
    HIP_OK(hipEventRecord(ctx->ev1, st));
    return SQH_OK;
}

void phase_times(const HullInfo& hi, sqh_stats& S);

// Read the status words back (synchronising the stream), fill the context's
// counters and map the device status to a return code.
int collect(sqh_ctx* ctx, const HullArgs& a, int64_t N, int64_t out_cap, int64_t* h_total, hipStream_t st,
            bool timed)
{
    const size_t info_bytes = ctx->trace ? sizeof(HullInfo) : offsetof(HullInfo, trace);
    const StatusOffsets so = status_offsets();
    const char* d0 = reinterpret_cast<const char*>(a.err);
    if (reinterpret_cast<const char*>(a.stats) == d0 + so.stats && reinterpret_cast<const char*>(a.info) == d0 + so.info) {
        // one copy of the whole block (each copy is a launch on the stream)
        HIP_OK(hipMemcpyAsync(ctx->hstatus, a.err, so.info + info_bytes, hipMemcpyDeviceToHost, st));
    } else {
        HIP_OK(hipMemcpyAsync(ctx->hinfo, a.info, info_bytes, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(ctx->hstats, a.stats, sizeof(uint32_t) * 4 * kStatSlots, hipMemcpyDeviceToHost, st));
        HIP_OK(hipMemcpyAsync(ctx->herr, a.err, sizeof(int), hipMemcpyDeviceToHost, st));
    }
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
    phase_times(hi, S);
    const int64_t h = hi.h_total;
    S.hull_size = h;
    S.prefilter_points = hi.prefilter_n;
    S.sorted_points = hi.sort_n;
    S.sort_violations = hi.sort_bad;
    S.stream_path = a.stream ? (hi.stream_done ? 1 : 2) : 0;
    S.line_filter = a.stream ? hi.stream_line : 0;
    if (timed) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) == hipSuccess) S.ms_total = ms;
        if (hipEventElapsedTime(&ms, ctx->evk, ctx->ev1) == hipSuccess) S.ms_kernel = ms;
    }
    if (h_total) *h_total = h;
    if (e & (kErrNonFinite | kErrBounds)) return SQH_EINVAL;
    if (e) return SQH_EDEVICE;
    return h > out_cap ? SQH_ECAPACITY : SQH_OK;
}

// Device timestamps (100 MHz constant clock) taken by workgroup 0 at phase
// ends, as phase durations.
void phase_times(const HullInfo& hi, sqh_stats& S)
{
    if (hi.nstamps <= 1) return;
    const double tick_ms = 1e-5;
    auto dt = [&](int i) { return (double)(hi.stamp[i] - hi.stamp[i - 1]) * tick_ms; };
    for (int i = 1; i < hi.nstamps && i < kMaxStamps; ++i) {
        const int tag = hi.stamp_tag[i];
        if (tag == 5) S.ms_prefilter += dt(i);
        else if (tag == 6) S.ms_sort += dt(i);
        else if (tag == 1) S.ms_seed += dt(i);
        else if (tag == 2) S.ms_split += dt(i);
        else if (tag == 3) S.ms_first += dt(i);
        else if (tag == 4) S.ms_emit += dt(i);
        else if (tag >= 100) {
            S.ms_pass += dt(i);
            if (tag - 100 < SQH_MAX_TIMED_PASSES) S.pass_ms[tag - 100] = dt(i);
        }
    }
}

int run_tuned(sqh_ctx* ctx, const float* d_xy, int64_t N, int64_t nsets, const int64_t* d_set_off, int32_t* d_out,
              int64_t* d_out_off, int64_t out_cap, int64_t* h_total, void* d_ws, size_t ws_bytes, hipStream_t st,
              const TuneEntry& tu)
{
    HullArgs a;
    int reset_grid = 1;
    int rc = setup(ctx, d_xy, N, nsets, d_set_off, d_out, d_out_off, out_cap, d_ws, ws_bytes, tu, a, reset_grid);
    if (rc != SQH_OK) return rc;
    if (!a.stream) {
        rc = enqueue(ctx, a, reset_grid, tu.grid, tu.sgrid, st);
        if (rc != SQH_OK) return rc;
        return collect(ctx, a, N, out_cap, h_total, st, true);
    }
    // streaming path: the passes kernel only if the streaming kernels left work
    const int cls = std::min(log2_class(N), 63);
    a.spasses = ctx->spass_used[cls] < 0 ? kStreamPassLaunches : ctx->spass_used[cls];
    rc = enqueue(ctx, a, reset_grid, tu.grid, tu.sgrid, st, false);
    if (rc != SQH_OK) return rc;
    rc = collect(ctx, a, N, out_cap, h_total, st, true);
    const HullInfo& hi = *ctx->hinfo;
    const bool done = hi.stream_done != 0 || *ctx->herr != 0;
    ctx->spass_used[cls] = hi.stream_done != 0 ? std::min(hi.spass_n, kStreamPassLaunches) : kStreamPassLaunches;
    if (done) return rc;
    void* argv[] = {static_cast<void*>(&a)};
    if (time_open(ctx, "k_hull<passes>", st) != SQH_OK) return SQH_EDEVICE;
    HIP_OK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_hull<kHullPasses>), dim3(tu.grid),
                                      dim3(kBlock), argv, 0, st));
    if (time_close(ctx, "k_hull<passes>", st) != SQH_OK) return SQH_EDEVICE;
    HIP_OK(hipEventRecord(ctx->ev1, st));
    return collect(ctx, a, N, out_cap, h_total, st, true);
}

int run(sqh_ctx* ctx, const float* d_xy, int64_t N, int64_t nsets, const int64_t* d_set_off, int32_t* d_out,
        int64_t* d_out_off, int64_t out_cap, int64_t* h_total, void* d_ws, size_t ws_bytes, hipStream_t st)
{
    return run_tuned(ctx, d_xy, N, nsets, d_set_off, d_out, d_out_off, out_cap, h_total, d_ws, ws_bytes, st,
                     pick_tuning(ctx, N));
}

// Minimal reader for the tuning format written by sqh_get_tuning:
//   {"entries": [{"log2n": K, "grid": G, "tail": T}, ...]}
// Keys may appear in any order inside an entry; unknown keys are ignored.
bool read_int_key(const char* obj, const char* end, const char* key, long& v)
{
    char pat[32];
    snprintf(pat, sizeof pat, "\"%s\"", key);
    const size_t plen = strlen(pat);
    for (const char* p = obj; p + plen <= end; ++p) {
        if (strncmp(p, pat, plen) != 0) continue;
        p += plen;
        while (p < end && (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')) ++p;
        if (p >= end || *p != ':') return false;
        ++p;
        char* q = nullptr;
        v = strtol(p, &q, 10);
        return q != p && q <= end;
    }
    return false;
}

}  // namespace

// ------------------------------------------------------------ engine --

namespace {

// Device arena of a serving engine with K slots (multiple of 64), R request
// entries and two staging halves of SC points (admissions fill one half while
// a step reads the other).
struct EngLayout {
    int64_t K, R, SC, scap, rcap;
    size_t x[2], y[2], id[2], segs[2], seg_cid[2], vstart[2];
    size_t bitmap, vidx, hout, recs, rec_cid, sets, gstart, sbase, bad, res_base, res_n, res_alive, res_h;
    size_t stage, vlist, slots, ctab, bar, err, stats, sv, info;
    size_t bytes;
};

bool make_eng_layout(int64_t K, int64_t R, int64_t SC, EngLayout& L)
{
    if (K < 64 || K % 64 || K > ((int64_t)INT32_MAX & ~63LL) - 64 || R < 1 || R > (1 << 20) || SC < 1 || SC > K)
        return false;
    L.K = K;
    L.R = R;
    L.SC = SC;
    // every segment holds a point, a pass leaves at most 2/3 of its points
    // in segments, and a new set adds at most 4 segments
    L.scap = (2 * K) / 3 + 4 * R + 64;
    L.rcap = std::max<int64_t>(4 * R, 2 * L.scap) + 8;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
    for (int b = 0; b < 2; ++b) {
        L.x[b] = take(sizeof(float) * (size_t)K);
        L.y[b] = take(sizeof(float) * (size_t)K);
        L.id[b] = take(sizeof(int) * (size_t)K);
        L.segs[b] = take(sizeof(Seg) * (size_t)L.scap);
        L.seg_cid[b] = take(sizeof(int) * (size_t)L.scap);
        L.vstart[b] = take(sizeof(int) * (size_t)(L.scap + 1));
    }
    L.bitmap = take(sizeof(uint64_t) * (size_t)(K / 64));
    L.vidx = take(sizeof(int) * (size_t)K);
    L.hout = take(sizeof(int) * (size_t)K);
    L.recs = take(sizeof(Seg) * (size_t)L.rcap);
    L.rec_cid = take(sizeof(int) * (size_t)L.rcap);
    L.sets = take(sizeof(SetInfo) * (size_t)R);
    L.gstart = take(sizeof(int) * (size_t)(R + 1));
    L.sbase = take(sizeof(int) * (size_t)R);
    L.bad = take(sizeof(int) * (size_t)R);
    L.res_base = take(sizeof(int) * (size_t)R);
    L.res_n = take(sizeof(int) * (size_t)R);
    L.res_alive = take(sizeof(int) * (size_t)R);
    L.res_h = take(sizeof(int) * (size_t)R);
    L.stage = take(sizeof(float2) * (size_t)(2 * SC));  // two halves: one per step in flight
    L.vlist = take(sizeof(int2));
    L.slots = take(sizeof(ChunkSlot<8>) * (size_t)kMaxGrid);
    L.ctab = take(sizeof(Pair) * (size_t)kMaxGrid);
    L.bar = take(sizeof(GridBar));
    L.err = take(sizeof(int));
    L.stats = take(sizeof(uint32_t) * 4 * kStatSlots);
    L.sv = take(sizeof(int) * 4);
    L.info = take(sizeof(HullInfo));
    L.bytes = o;
    return true;
}

struct EngReq {
    uint64_t tag;
    int64_t base, n, alloc, stage_at;
};

struct EngDone {
    uint64_t tag;
    int status;
    std::vector<int32_t> hull;
};

}  // namespace

struct sqh_engine {
    sqh_ctx* ctx = nullptr;
    char* arena = nullptr;
    EngLayout L{};
    int cur = 0;    // survivor buffer holding the resident segments
    int side = 0;   // staging half that admissions fill
    bool broken = false;
    bool inflight = false;
    bool admitted = false;  // admissions since the last launch (ev_admit is recorded)
    std::map<int64_t, int64_t> free_ranges;  // first slot -> length (64-aligned)
    std::vector<EngReq> staged;     // admitted, waiting for the next launch
    std::vector<EngReq> resident;   // segments in the table
    std::vector<EngReq> step_all;   // launched step: all requests, by first slot
    std::vector<EngReq> step_new;   // launched step: its new requests
    int64_t stage_used = 0;
    std::deque<EngDone> done;
    int* h_up = nullptr;     // pinned: gstart (R+1), sbase (R), res_base (R), res_n (R)
    int* h_down = nullptr;   // pinned: res_alive (R), res_h (R), bad (R), err
    int32_t* h_bounce = nullptr;
    int64_t bounce_cap = 0;
    HullInfo* h_info = nullptr;
    hipEvent_t ev_admit = nullptr, ev_done = nullptr;
    hipStream_t step_stream = nullptr;
    int64_t steps = 0;
};

namespace {

int64_t up_points(const sqh_engine* e)
{
    int64_t n = 0;
    for (const auto& q : e->step_new) n += q.n;
    return n;
}

bool eng_alloc(sqh_engine* e, int64_t n, int64_t& base)
{
    const int64_t need = (n + 63) & ~63LL;
    for (auto it = e->free_ranges.begin(); it != e->free_ranges.end(); ++it) {
        if (it->second >= need) {
            base = it->first;
            const int64_t rest = it->second - need;
            e->free_ranges.erase(it);
            if (rest > 0) e->free_ranges[base + need] = rest;
            return true;
        }
    }
    return false;
}

void eng_free(sqh_engine* e, int64_t base, int64_t alloc)
{
    auto it = e->free_ranges.emplace(base, alloc).first;
    auto next = std::next(it);
    if (next != e->free_ranges.end() && it->first + it->second == next->first) {
        it->second += next->second;
        e->free_ranges.erase(next);
    }
    if (it != e->free_ranges.begin()) {
        auto prev = std::prev(it);
        if (prev->first + prev->second == it->first) {
            prev->second += it->second;
            e->free_ranges.erase(it);
        }
    }
}

}  // namespace

// Structure-of-arrays input: the interleaved copy at the front of the
// workspace (8 bytes per point, rounded up to the workspace alignment).
inline size_t soa_copy_bytes(int64_t n) { return ((size_t)n * sizeof(float2) + kAlign - 1) / kAlign * kAlign; }

__global__ __launch_bounds__(256) void k_interleave(const float* x, const float* y, float2* xy, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        xy[i] = make_float2(x[i], y[i]);
}

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
    // co-resident workgroups: the smallest over every cooperative kernel
    int per_cu = 1 << 30;
    {
        const void* coop[] = {reinterpret_cast<const void*>(k_hull<kHullPlain>),
                              reinterpret_cast<const void*>(k_hull<kHullPre>),
                              reinterpret_cast<const void*>(k_hull<kHullFirst>),
                              reinterpret_cast<const void*>(k_hull<kHullPasses>),
                              reinterpret_cast<const void*>(k_prefilter), reinterpret_cast<const void*>(k_sort)};
        for (const void* f : coop) {
            int k = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, f, kBlock, 0) != hipSuccess) k = 0;
            per_cu = std::min(per_cu, k);
        }
    }
    if (per_cu < 1) {
        delete c;
        return SQH_EDEVICE;
    }
    c->max_grid = std::min(kMaxGrid, per_cu * c->cus);
    scratch_init(device);  // the device is current here
    {
        const char* t = getenv("SQH_TRACE");
        c->trace = t ? atoi(t) : 0;  // 1: seed and split, 2: first compaction and first pass
        const char* st = getenv("SQH_STREAM");
        c->stream = st ? (atoi(st) != 0) : 1;
    }
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->evk) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->hstatus), status_offsets().bytes, hipHostMallocDefault) !=
            hipSuccess) {
        sqh_destroy(c);
        return SQH_EDEVICE;
    }
    {
        const StatusOffsets so = status_offsets();
        c->herr = reinterpret_cast<int*>(c->hstatus);
        c->hstats = reinterpret_cast<uint32_t*>(c->hstatus + so.stats);
        c->hinfo = reinterpret_cast<HullInfo*>(c->hstatus + so.info);
    }
    *out = c;
    return SQH_OK;
}

void sqh_destroy(sqh_ctx* c)
{
    if (!c) return;
    for (hipEvent_t& e : c->lev)
        if (e) (void)hipEventDestroy(e);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->evk) (void)hipEventDestroy(c->evk);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->hstatus) (void)hipHostFree(c->hstatus);
    delete c;
}

int sqh_set_prefilter(sqh_ctx* c, int mode)
{
    if (!c || mode < SQH_PREFILTER_NONE || mode > SQH_PREFILTER_OCTAGON) return SQH_EINVAL;
    c->prefilter = mode;
    return SQH_OK;
}

int sqh_set_variant(sqh_ctx* c, int variant)
{
    if (!c || (variant != SQH_VARIANT_PARTITION && variant != SQH_VARIANT_SORTED)) return SQH_EINVAL;
    c->variant = variant;
    return SQH_OK;
}

int sqh_set_precision(sqh_ctx* c, int mode)
{
    if (!c || (mode != SQH_FP32_FILTER && mode != SQH_FP64_ONLY && mode != SQH_FP32_SEMISTATIC)) return SQH_EINVAL;
    c->fp64 = mode == SQH_FP64_ONLY;
    c->line = mode == SQH_FP32_FILTER;
    return SQH_OK;
}

int sqh_set_streaming(sqh_ctx* c, int on)
{
    if (!c) return SQH_EINVAL;
    c->stream = on != 0;
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

size_t sqh_workspace_bytes_soa(int64_t n)
{
    Layout L;
    if (!make_layout(n, 1, L)) return 0;
    return soa_copy_bytes(n) + L.bytes;
}

int sqh_hull_soa(sqh_ctx* c, const float* d_x, const float* d_y, int64_t n, int32_t* d_out, int64_t out_cap,
                 int64_t* h_count, void* d_ws, size_t ws_bytes, void* stream)
{
    if (!c || !h_count || n < 0 || (n > 0 && (!d_x || !d_y))) return SQH_EINVAL;
    *h_count = 0;
    const size_t need = sqh_workspace_bytes_soa(n);
    if (need == 0) return SQH_EINVAL;
    if (!d_ws || ws_bytes < need) return SQH_ENOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    float2* xy = static_cast<float2*>(d_ws);
    const size_t cb = soa_copy_bytes(n);
    if (n > 0) {
        const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
        k_interleave<<<grid, 256, 0, st>>>(d_x, d_y, xy, n);
        HIP_OK(hipGetLastError());
    }
    return run(c, reinterpret_cast<const float*>(xy), n, 1, nullptr, d_out, nullptr, out_cap, h_count,
               static_cast<unsigned char*>(d_ws) + cb, ws_bytes - cb, st);
}

int sqh_hull_noalloc(sqh_ctx* c, const float* d_xy, int64_t n, int32_t* d_out, int64_t out_cap, int64_t* h_count,
                     void* stream)
{
    if (!c || !h_count || n < 0) return SQH_EINVAL;
    *h_count = 0;
    if (n > SQH_NOALLOC_MAX_POINTS) return SQH_ENOMEM;
    if (c->device < 0 || c->device >= kMaxDevices) return SQH_EDEVICE;
    const ScratchSlot& sl = g_scratch_slot[c->device];
    if (sl.rc != SQH_OK) return SQH_EDEVICE;
    Layout L;
    if (!make_layout(n, 1, L) || L.bytes > kScratchBytes) return SQH_ENOMEM;
    return run(c, d_xy, n, 1, nullptr, d_out, nullptr, out_cap, h_count, sl.ptr, kScratchBytes,
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

int sqh_autotune(sqh_ctx* c, const float* d_xy, const int64_t* d_set_off, int64_t n_sets, int64_t n_total,
                 int32_t* d_out, int64_t* d_out_off, int64_t out_cap, void* d_ws, size_t ws_bytes, void* stream,
                 int reps)
{
    if (!c || n_sets < 1 || n_total < 0 || reps < 1 || reps > 100) return SQH_EINVAL;
    if (n_sets > 1 && (!d_set_off || !d_out_off)) return SQH_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int cls = log2_class(n_total);
    const int m = c->max_grid;
    const int grids[4] = {m, std::max(1, (3 * m) / 4), std::max(1, m / 2), std::max(1, m / 4)};
    const int tails[3] = {0, 1 << 13, 1 << 16};
    // candidates: the persistent kernel at every grid x tail; for one large
    // set also the streaming path at 1024, 512 and 256 workgroups
    TuneEntry cand[16];
    int nc = 0;
    for (int gi = 0; gi < 4; ++gi) {
        if (gi > 0 && grids[gi] == grids[gi - 1]) continue;
        for (int ti = 0; ti < 3; ++ti) {
            cand[nc] = TuneEntry{cls, grids[gi], tails[ti]};
            cand[nc++].stream = 0;
        }
    }
    if (n_sets == 1 && n_total >= kStreamMin && c->stream) {
        for (const int sg : {kMaxSGrid, kMaxSGrid / 2, kMaxSGrid / 4}) {
            cand[nc] = TuneEntry{cls, m, kTailPoints};
            cand[nc].stream = 1;
            cand[nc++].sgrid = sg;
        }
    }
    TuneEntry best{cls, m, kTailPoints};
    double best_ms = 1e300;
    int64_t h = 0;
    for (int ci = 0; ci < nc; ++ci) {
        const TuneEntry& tu = cand[ci];
        int rc = run_tuned(c, d_xy, n_total, n_sets, d_set_off, d_out, d_out_off, out_cap, &h, d_ws, ws_bytes, st,
                           tu);  // warm-up
        if (rc != SQH_OK) return rc;
        double t[100];
        for (int r = 0; r < reps; ++r) {
            rc = run_tuned(c, d_xy, n_total, n_sets, d_set_off, d_out, d_out_off, out_cap, &h, d_ws, ws_bytes, st,
                           tu);
            if (rc != SQH_OK) return rc;
            t[r] = c->stats.ms_total;
        }
        std::sort(t, t + reps);
        const double med = t[reps / 2];
        if (med < best_ms) {
            best_ms = med;
            best = tu;
        }
    }
    int slot = -1;
    for (int i = 0; i < c->ntune; ++i)
        if (c->tune[i].log2n == cls) slot = i;
    if (slot < 0) {
        if (c->ntune >= sqh_ctx::kMaxTune) return SQH_ENOMEM;
        slot = c->ntune++;
    }
    c->tune[slot] = best;
    return SQH_OK;
}

int sqh_get_tuning(const sqh_ctx* c, char* buf, size_t len)
{
    if (!c) return SQH_EINVAL;
    char tmp[96 * sqh_ctx::kMaxTune + 64];
    int n = snprintf(tmp, sizeof tmp, "{\"entries\": [");
    for (int i = 0; i < c->ntune; ++i)
        n += snprintf(tmp + n, sizeof tmp - n,
                      "%s{\"log2n\": %d, \"grid\": %d, \"tail\": %d, \"stream\": %d, \"sgrid\": %d}",
                      i ? ", " : "", c->tune[i].log2n, c->tune[i].grid, c->tune[i].tail, c->tune[i].stream,
                      c->tune[i].sgrid);
    n += snprintf(tmp + n, sizeof tmp - n, "]");
    if (c->engine_grid > 0) n += snprintf(tmp + n, sizeof tmp - n, ", \"engine_grid\": %d", c->engine_grid);
    n += snprintf(tmp + n, sizeof tmp - n, "}");
    if (buf && len > 0) {
        const size_t k = std::min<size_t>(len - 1, (size_t)n);
        memcpy(buf, tmp, k);
        buf[k] = 0;
    }
    return n + 1;
}

int sqh_set_tuning(sqh_ctx* c, const char* json)
{
    if (!c || !json) return SQH_EINVAL;
    TuneEntry t[sqh_ctx::kMaxTune];
    int nt = 0;
    const char* p = strstr(json, "\"entries\"");
    if (!p) return SQH_EINVAL;
    p = strchr(p, '[');
    if (!p) return SQH_EINVAL;
    const char* close = strchr(p, ']');
    if (!close) return SQH_EINVAL;
    for (const char* o = strchr(p, '{'); o && o < close; o = strchr(o + 1, '{')) {
        const char* e = strchr(o, '}');
        if (!e || e > close) return SQH_EINVAL;
        long k = 0, g = 0, tl = 0, sm = 1, sg = 0;
        if (!read_int_key(o, e, "log2n", k) || !read_int_key(o, e, "grid", g) || !read_int_key(o, e, "tail", tl))
            return SQH_EINVAL;
        (void)read_int_key(o, e, "stream", sm);  // optional keys
        (void)read_int_key(o, e, "sgrid", sg);
        if (k < 0 || k > 62 || g < 1 || g > c->max_grid || tl < 0 || tl > INT32_MAX) return SQH_EINVAL;
        if ((sm != 0 && sm != 1) || sg < 0 || sg > kMaxSGrid) return SQH_EINVAL;
        if (nt >= sqh_ctx::kMaxTune) return SQH_EINVAL;
        t[nt] = TuneEntry{(int)k, (int)g, (int)tl};
        t[nt].stream = (int)sm;
        t[nt++].sgrid = (int)sg;
    }
    long eg = 0;
    const char* after = close + 1;
    if (read_int_key(after, after + strlen(after), "engine_grid", eg) && (eg < 1 || eg > c->max_grid))
        return SQH_EINVAL;
    memcpy(c->tune, t, sizeof(TuneEntry) * nt);
    c->ntune = nt;
    c->engine_grid = (int)eg;
    return SQH_OK;
}

int sqh_graph_create(sqh_ctx* c, const float* d_xy, const int64_t* d_set_off, int64_t n_sets, int64_t n_total,
                     int32_t* d_out, int64_t* d_out_off, int64_t out_cap, void* d_ws, size_t ws_bytes,
                     sqh_graph** out)
{
    if (!out) return SQH_EINVAL;
    *out = nullptr;
    if (!c || n_sets < 1 || n_total < 0) return SQH_EINVAL;
    if (n_sets > 1 && (!d_set_off || !d_out_off)) return SQH_EINVAL;
    sqh_graph* g = new (std::nothrow) sqh_graph();
    if (!g) return SQH_ENOMEM;
    g->ctx = c;
    g->N = n_total;
    g->out_cap = out_cap;
    const TuneEntry tu = pick_tuning(c, n_total);
    int reset_grid = 1;
    int rc = setup(c, d_xy, n_total, n_sets, d_set_off, d_out, d_out_off, out_cap, d_ws, ws_bytes, tu, g->args,
                   reset_grid);
    if (rc != SQH_OK) {
        delete g;
        return rc;
    }
    // a chain of kernel nodes: the workspace reset, then the cooperative
    // launches of the call, each marked cooperative so that every
    // workgroup is resident at once
    void* argv[] = {static_cast<void*>(&g->args)};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(k_reset);
    kp.gridDim = dim3(reset_grid);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = argv;
    kp.extra = nullptr;
    hipKernelNodeAttrValue coop{};
    coop.cooperative = 1;
    hipGraphNode_t prev = nullptr;
    bool ok = hipGraphCreate(&g->graph, 0) == hipSuccess &&
              hipGraphAddKernelNode(&prev, g->graph, nullptr, 0, &kp) == hipSuccess;
    Launch L[kMaxLaunches];
    const int nf = call_launches(g->args, L);
    for (int i = 0; ok && i < nf; ++i) {
        hipKernelNodeParams hp = kp;
        hp.func = const_cast<void*>(L[i].f);
        hp.gridDim = launch_grid(L[i], tu.grid, tu.sgrid);
        hp.blockDim = launch_block(L[i]);
        hipGraphNode_t node = nullptr;
        ok = hipGraphAddKernelNode(&node, g->graph, &prev, 1, &hp) == hipSuccess &&
             (!L[i].coop ||
              hipGraphKernelNodeSetAttribute(node, hipKernelNodeAttributeCooperative, &coop) == hipSuccess);
        prev = node;
    }
    ok = ok && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) == hipSuccess;
    if (!ok) {
        sqh_graph_destroy(g);
        return SQH_EDEVICE;
    }
    *out = g;
    return SQH_OK;
}

int sqh_graph_launch(sqh_graph* g, void* stream)
{
    if (!g || !g->exec) return SQH_EINVAL;
    HIP_OK(hipSetDevice(g->ctx->device));
    HIP_OK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return SQH_OK;
}

int sqh_graph_result(sqh_graph* g, int64_t* h_total, void* stream)
{
    if (!g || !g->exec) return SQH_EINVAL;
    HIP_OK(hipSetDevice(g->ctx->device));
    return collect(g->ctx, g->args, g->N, g->out_cap, h_total, static_cast<hipStream_t>(stream), false);
}

void sqh_graph_destroy(sqh_graph* g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

size_t sqh_engine_bytes(int64_t slots, int64_t max_requests, int64_t stage_points)
{
    EngLayout L;
    if (!make_eng_layout(slots, max_requests, stage_points, L)) return 0;
    return L.bytes;
}

int sqh_engine_create(sqh_ctx* c, void* d_arena, size_t arena_bytes, int64_t slots, int64_t max_requests,
                      int64_t stage_points, sqh_engine** out)
{
    if (!out) return SQH_EINVAL;
    *out = nullptr;
    if (!c || !d_arena) return SQH_EINVAL;
    EngLayout L;
    if (!make_eng_layout(slots, max_requests, stage_points, L)) return SQH_EINVAL;
    if (arena_bytes < L.bytes) return SQH_ENOMEM;
    HIP_OK(hipSetDevice(c->device));
    sqh_engine* e = new (std::nothrow) sqh_engine();
    if (!e) return SQH_ENOMEM;
    e->ctx = c;
    e->arena = static_cast<char*>(d_arena);
    e->L = L;
    e->free_ranges[0] = slots;
    const size_t up = sizeof(int) * (size_t)(4 * max_requests + 1);
    const size_t down = sizeof(int) * (size_t)(3 * max_requests + 1);
    e->bounce_cap = 1 << 20;
    if (hipHostMalloc(reinterpret_cast<void**>(&e->h_up), up, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_down), down, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_bounce), sizeof(int32_t) * (size_t)e->bounce_cap,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&e->h_info), sizeof(HullInfo), hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_admit, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&e->ev_done, hipEventDisableTiming) != hipSuccess) {
        sqh_engine_destroy(e);
        return SQH_EDEVICE;
    }
    // empty resident tables in both survivor buffers
    if (hipMemset(e->arena + L.sv, 0, sizeof(int) * 4) != hipSuccess ||
        hipMemset(e->arena + L.vstart[0], 0, sizeof(int)) != hipSuccess ||
        hipMemset(e->arena + L.vstart[1], 0, sizeof(int)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        sqh_engine_destroy(e);
        return SQH_EDEVICE;
    }
    *out = e;
    return SQH_OK;
}

void sqh_engine_destroy(sqh_engine* e)
{
    if (!e) return;
    if (e->inflight && e->ev_done) (void)hipEventSynchronize(e->ev_done);
    if (e->h_up) (void)hipHostFree(e->h_up);
    if (e->h_down) (void)hipHostFree(e->h_down);
    if (e->h_bounce) (void)hipHostFree(e->h_bounce);
    if (e->h_info) (void)hipHostFree(e->h_info);
    if (e->ev_admit) (void)hipEventDestroy(e->ev_admit);
    if (e->ev_done) (void)hipEventDestroy(e->ev_done);
    delete e;
}

int sqh_engine_admit(sqh_engine* e, const float* xy, int64_t n, uint64_t tag, int on_device, void* stream)
{
    if (!e || n < 0 || (n > 0 && !xy)) return SQH_EINVAL;
    if (e->broken) return SQH_EDEVICE;
    if (n > e->L.SC || n > e->L.K) return SQH_EINVAL;  // can never fit
    if (n == 0) {
        e->done.push_back(EngDone{tag, SQH_OK, {}});
        return SQH_OK;
    }
    const size_t in_flight = e->inflight ? e->step_all.size() : e->resident.size();
    if ((int64_t)(e->staged.size() + in_flight) >= e->L.R) return SQH_EBUSY;
    if (e->stage_used + n > e->L.SC) return SQH_EBUSY;
    int64_t base = 0;
    if (!eng_alloc(e, n, base)) return SQH_EBUSY;
    HIP_OK(hipSetDevice(e->ctx->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    float2* stage = reinterpret_cast<float2*>(e->arena + e->L.stage) + (size_t)e->side * e->L.SC + e->stage_used;
    if (hipMemcpyAsync(stage, xy, sizeof(float2) * (size_t)n,
                       on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(e->ev_admit, st) != hipSuccess) {
        eng_free(e, base, (n + 63) & ~63LL);
        return SQH_EDEVICE;
    }
    e->admitted = true;
    e->staged.push_back(EngReq{tag, base, n, (n + 63) & ~63LL, e->stage_used});
    e->stage_used += n;
    return SQH_OK;
}

int sqh_engine_launch(sqh_engine* e, int max_passes, void* stream)
{
    if (!e || max_passes < 1 || max_passes > kMaxPasses) return SQH_EINVAL;
    if (e->broken) return SQH_EDEVICE;
    if (e->inflight) return SQH_EBUSY;
    if (e->staged.empty() && e->resident.empty()) return SQH_ENOTFOUND;
    sqh_ctx* c = e->ctx;
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIP_OK(hipSetDevice(c->device));
    const EngLayout& L = e->L;
    const int64_t R = L.R;
    const int G = (int)e->staged.size();
    // all requests in slot order (new ones included) for the census
    e->step_all = e->resident;
    e->step_all.insert(e->step_all.end(), e->staged.begin(), e->staged.end());
    std::sort(e->step_all.begin(), e->step_all.end(),
              [](const EngReq& p, const EngReq& q) { return p.base < q.base; });
    e->step_new.swap(e->staged);
    e->staged.clear();
    const int nres = (int)e->step_all.size();
    int* up_gstart = e->h_up;
    int* up_sbase = e->h_up + (R + 1);
    int* up_rbase = e->h_up + (2 * R + 1);
    int* up_rn = e->h_up + (3 * R + 1);
    for (int g = 0; g < G; ++g) {
        up_gstart[g] = (int)e->step_new[g].stage_at;
        up_sbase[g] = (int)e->step_new[g].base;
    }
    up_gstart[G] = (int)e->stage_used;
    for (int r = 0; r < nres; ++r) {
        up_rbase[r] = (int)e->step_all[r].base;
        up_rn[r] = (int)e->step_all[r].n;
    }
    char* A = e->arena;
    auto at = [&](size_t off) { return static_cast<void*>(A + off); };
    if (e->admitted) HIP_OK(hipStreamWaitEvent(st, e->ev_admit, 0));  // staged points have arrived
    e->admitted = false;
    HIP_OK(hipMemcpyAsync(at(L.gstart), up_gstart, sizeof(int) * (size_t)(G + 1), hipMemcpyHostToDevice, st));
    if (G > 0) HIP_OK(hipMemcpyAsync(at(L.sbase), up_sbase, sizeof(int) * (size_t)G, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(at(L.res_base), up_rbase, sizeof(int) * (size_t)nres, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(at(L.res_n), up_rn, sizeof(int) * (size_t)nres, hipMemcpyHostToDevice, st));

    // An engine step leaves 1/8 of the compute units free by default: the
    // copies of the next step's admissions run as copy kernels, which cannot
    // start while the persistent kernel holds every compute unit.
    TuneEntry tu = pick_tuning(c, e->stage_used > 0 ? e->stage_used : 1);
    tu.grid = c->engine_grid > 0 ? std::min(c->engine_grid, c->max_grid)
                                 : std::max(1, c->max_grid - c->max_grid / 8);
    HullArgs a{};
    a.xy = reinterpret_cast<const float2*>(A + L.stage) + (size_t)e->side * L.SC;
    a.N = (int)e->stage_used;
    a.G = G;
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
    a.vcap = 0;
    a.slots = at(L.slots);
    a.ctab = static_cast<Pair*>(at(L.ctab));
    a.bar = static_cast<GridBar*>(at(L.bar));
    a.err = static_cast<int*>(at(L.err));
    a.stats = static_cast<uint32_t*>(at(L.stats));
    a.info = static_cast<HullInfo*>(at(L.info));
    a.fp64 = c->fp64;
    a.timing = 1;
    a.tail_points = tu.tail;
    a.sbase = static_cast<const int*>(at(L.sbase));
    a.cur0 = e->cur;
    a.max_passes = max_passes;
    a.nres = nres;
    a.res_base = static_cast<const int*>(at(L.res_base));
    a.res_n = static_cast<const int*>(at(L.res_n));
    a.res_alive = static_cast<int*>(at(L.res_alive));
    a.res_h = static_cast<int*>(at(L.res_h));
    a.hout = static_cast<int*>(at(L.hout));
    a.bad = static_cast<int*>(at(L.bad));

    HIP_OK(hipEventRecord(c->ev0, st));
    k_engine_reset<<<std::max(1, std::min(1024, std::max(G, nres / 256 + 1))), 256, 0, st>>>(a);
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(c->evk, st));
    void* argv[] = {static_cast<void*>(&a)};
    HIP_OK(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_engine_step), dim3(tu.grid), dim3(kBlock),
                                      argv, 0, st));
    HIP_OK(hipEventRecord(c->ev1, st));
    int* dn_alive = e->h_down;
    int* dn_h = e->h_down + R;
    int* dn_bad = e->h_down + 2 * R;
    int* dn_err = e->h_down + 3 * R;
    HIP_OK(hipMemcpyAsync(dn_alive, at(L.res_alive), sizeof(int) * (size_t)nres, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(dn_h, at(L.res_h), sizeof(int) * (size_t)nres, hipMemcpyDeviceToHost, st));
    if (G > 0) HIP_OK(hipMemcpyAsync(dn_bad, at(L.bad), sizeof(int) * (size_t)G, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(dn_err, at(L.err), sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(e->h_info, at(L.info), offsetof(HullInfo, trace), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(c->hstats, at(L.stats), sizeof(uint32_t) * 4 * kStatSlots, hipMemcpyDeviceToHost, st));
    HIP_OK(hipEventRecord(e->ev_done, st));
    // later admissions fill the other staging half
    e->side ^= 1;
    e->stage_used = 0;
    e->step_stream = st;
    e->inflight = true;
    return SQH_OK;
}

int sqh_engine_finish(sqh_engine* e)
{
    if (!e) return SQH_EINVAL;
    if (e->broken) return SQH_EDEVICE;
    if (!e->inflight) return 0;
    sqh_ctx* c = e->ctx;
    hipStream_t st = e->step_stream;
    HIP_OK(hipSetDevice(c->device));
    HIP_OK(hipEventSynchronize(e->ev_done));
    e->inflight = false;
    const EngLayout& L = e->L;
    const int64_t R = L.R;
    char* A = e->arena;
    const int G = (int)e->step_new.size();
    const int nres = (int)e->step_all.size();
    int* dn_alive = e->h_down;
    int* dn_h = e->h_down + R;
    int* dn_bad = e->h_down + 2 * R;
    int* dn_err = e->h_down + 3 * R;
    if (*dn_err & (kErrSpin | kErrBounds)) {
        e->broken = true;
        return SQH_EDEVICE;
    }
    e->cur = e->h_info->cur_out;
    ++e->steps;
    {
        sqh_stats& S = c->stats;
        S = sqh_stats{};
        S.points = up_points(e);
        S.passes = e->h_info->passes;
        phase_times(*e->h_info, S);
        for (int i = 0; i < kStatSlots; ++i) {
            S.orient_evals += c->hstats[4 * i + 0];
            S.orient_exact += c->hstats[4 * i + 1];
            S.cmp_exact += c->hstats[4 * i + 2];
        }
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess) S.ms_total = ms;
        if (hipEventElapsedTime(&ms, c->evk, c->ev1) == hipSuccess) S.ms_kernel = ms;
    }
    // bad inputs among the new requests (their sets were skipped)
    std::map<int64_t, int> bad_base;
    for (int g = 0; g < G; ++g)
        if (dn_bad[g]) bad_base[e->step_new[g].base] = 1;
    // collect finished requests: copy their hulls through the pinned bounce buffer
    int finished = 0;
    std::vector<EngReq> keep;
    std::vector<std::pair<EngReq, int>> fin;
    for (int r = 0; r < nres; ++r) {
        if (dn_alive[r]) keep.push_back(e->step_all[r]);
        else fin.push_back({e->step_all[r], dn_h[r]});
    }
    auto deliver = [&](const EngReq& q, const int32_t* h, int64_t cnt) {
        EngDone d{q.tag, SQH_OK, std::vector<int32_t>(h, h + cnt)};
        if (bad_base.count(q.base)) {
            d.status = SQH_EINVAL;
            d.hull.clear();
        }
        e->done.push_back(std::move(d));
        eng_free(e, q.base, q.alloc);
        ++finished;
    };
    size_t i0 = 0;
    while (i0 < fin.size()) {
        if (fin[i0].second > e->bounce_cap) {
            // one hull larger than the bounce buffer: copy it directly
            std::vector<int32_t> tmp((size_t)fin[i0].second);
            HIP_OK(hipMemcpy(tmp.data(), A + L.hout + sizeof(int) * (size_t)fin[i0].first.base,
                             sizeof(int) * tmp.size(), hipMemcpyDeviceToHost));
            deliver(fin[i0].first, tmp.data(), (int64_t)tmp.size());
            ++i0;
            continue;
        }
        int64_t used = 0;
        size_t i1 = i0;
        while (i1 < fin.size() && used + fin[i1].second <= e->bounce_cap) {
            const int h = fin[i1].second;
            if (h > 0)
                HIP_OK(hipMemcpyAsync(e->h_bounce + used, A + L.hout + sizeof(int) * (size_t)fin[i1].first.base,
                                      sizeof(int) * (size_t)h, hipMemcpyDeviceToHost, st));
            used += h;
            ++i1;
        }
        HIP_OK(hipStreamSynchronize(st));
        int64_t off = 0;
        for (size_t i = i0; i < i1; ++i) {
            deliver(fin[i].first, e->h_bounce + off, fin[i].second);
            off += fin[i].second;
        }
        i0 = i1;
    }
    e->resident.swap(keep);
    e->step_new.clear();
    e->step_all.clear();
    return finished;
}

int sqh_engine_step(sqh_engine* e, int max_passes, void* stream)
{
    const int rc = sqh_engine_launch(e, max_passes, stream);
    if (rc == SQH_ENOTFOUND) return 0;  // nothing resident or staged
    if (rc != SQH_OK) return rc;
    return sqh_engine_finish(e);
}

int sqh_engine_poll(sqh_engine* e, uint64_t* tag, int32_t* h_out, int64_t cap, int64_t* h)
{
    if (!e || !tag || !h || cap < 0 || (cap > 0 && !h_out)) return SQH_EINVAL;
    if (e->done.empty()) return SQH_ENOTFOUND;
    EngDone& d = e->done.front();
    *tag = d.tag;
    *h = (int64_t)d.hull.size();
    const int st = d.status;
    if (st != SQH_OK) {
        e->done.pop_front();
        return st;
    }
    if (*h > cap) return SQH_ECAPACITY;  // kept: poll again with a larger buffer
    if (*h > 0) memcpy(h_out, d.hull.data(), sizeof(int32_t) * (size_t)*h);
    e->done.pop_front();
    return SQH_OK;
}

int sqh_engine_status(const sqh_engine* e, int64_t* resident, int64_t* staged, int64_t* finished,
                      int64_t* free_slots)
{
    if (!e) return SQH_EINVAL;
    if (resident) *resident = (int64_t)(e->inflight ? e->step_all.size() : e->resident.size());
    if (staged) *staged = (int64_t)e->staged.size();
    if (finished) *finished = (int64_t)e->done.size();
    if (free_slots) {
        int64_t f = 0;
        for (const auto& kv : e->free_ranges) f += kv.second;
        *free_slots = f;
    }
    return e->broken ? SQH_EDEVICE : SQH_OK;
}

int sqh_get_trace(const sqh_ctx* c, uint64_t* out, int max_entries)
{
    if (!c || !out || max_entries < 0) return SQH_EINVAL;
    if (!c->trace) return 0;
    const int n = std::min(max_entries, c->max_grid * 8);
    for (int i = 0; i < n; ++i) out[i] = c->hinfo->trace[i / 8][i % 8];
    return n;
}

int sqh_set_launch_timing(sqh_ctx* c, int on, const char* only)
{
    if (!c || (only && strlen(only) >= sizeof c->lonly)) return SQH_EINVAL;
    if (on && !c->lev[0]) {
        (void)hipSetDevice(c->device);
        for (hipEvent_t& e : c->lev)
            if (hipEventCreate(&e) != hipSuccess) return SQH_EDEVICE;
    }
    c->ltiming = on != 0;
    snprintf(c->lonly, sizeof c->lonly, "%s", only ? only : "");
    c->nl = 0;
    return SQH_OK;
}

int sqh_get_launch_times(const sqh_ctx* c, const char** names, double* ms, int cap)
{
    if (!c || cap < 0 || (cap > 0 && (!names || !ms))) return SQH_EINVAL;
    const int n = std::min(cap, c->nl);
    for (int i = 0; i < n; ++i) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, c->lev[2 * i], c->lev[2 * i + 1]) != hipSuccess) return SQH_EDEVICE;
        names[i] = c->lname[i];
        ms[i] = t;
    }
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

// ---- test hooks ----------------------------------------------------------

namespace {
int diag_finish(hipStream_t st)
{
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    return SQH_OK;
}
}  // namespace

extern "C" {

int sqh_diag_orient(const float* d_tri, int64_t n, int fp64_only, int32_t* d_sign, float* d_vals, int32_t* d_flags,
                    void* stream)
{
    if (n < 0 || n > INT32_MAX / 6 || (n > 0 && (!d_tri || !d_sign || !d_vals || !d_flags))) return SQH_EINVAL;
    if (n == 0) return SQH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_diag_orient<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(d_tri, (int)n, fp64_only != 0, d_sign, d_vals,
                                                             d_flags);
    return diag_finish(st);
}

int sqh_diag_compare(const float* d_cases, const int32_t* d_ids, int64_t n, int fp64_only, int32_t* d_out,
                     void* stream)
{
    if (n < 0 || n > INT32_MAX / 8 || (n > 0 && (!d_cases || !d_ids || !d_out))) return SQH_EINVAL;
    if (n == 0) return SQH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_diag_compare<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(d_cases, d_ids, (int)n, fp64_only != 0, d_out);
    return diag_finish(st);
}

int sqh_diag_scan(const int32_t* d_in, int64_t n, int32_t* d_ex_a, int32_t* d_ex_b, int32_t* d_tot, void* stream)
{
    if (n < 0 || n > INT32_MAX - kBlock || (n > 0 && (!d_in || !d_ex_a || !d_ex_b || !d_tot))) return SQH_EINVAL;
    if (n == 0) return SQH_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_diag_scan<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(d_in, (int)n, d_ex_a, d_ex_b, d_tot);
    return diag_finish(st);
}

}  // extern "C"
