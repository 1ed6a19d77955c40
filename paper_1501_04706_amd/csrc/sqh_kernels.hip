// HIP kernels of libsqh (gfx950): seed, first split, first compaction,
// segmented passes, segment-table rebuild and ordered emission.
//
// Paper mapping (Zhang, Mei, Xu, Zhao, arXiv 1501.04706):
//   k_seed    section 4.3 -- leftmost / rightmost points (lexicographic here)
//   k_split   section 4.3 + 4.4.1 -- side of every point w.r.t. the line
//             through them, and the farthest point of each side
//   k_first   sections 4.4.2-4.4.4 on the two sides -- discard points inside
//             the triangle, stable partition into the two child segments,
//             and the farthest point of each child (the next pass's step
//             4.4.1, fused)
//   k_pass    the same for all segments of all sets at once
//   k_table   section 4.4.2 / 4.4.4 segment updates: the child segments of
//             every segment become the next pass's segment table
//   k_emit    the surviving heads, in ring order, are the hull
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sqh_pred.hpp"
#include "sqh_tile.hpp"
#include "sqh_types.hpp"

namespace sqh {

constexpr int kRows = 8;  // rows of 64 positions per wave: tile = 2048 positions

__device__ __forceinline__ int search_le(const int* start, int q, int lo, int hi)
{
    // largest g in [lo, hi] with start[g] <= q (start[lo] <= q is assumed)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A hull vertex gets a key: a slot of the survivor index space that no
// point and no other vertex of its set uses, increasing along the ring
// (counter-clockwise from the set's lexmin point). The emit step orders
// vertices by key.
__device__ __forceinline__ void record_vertex(uint64_t* bitmap, int* vidx, int key, int id)
{
    atomicOr((unsigned long long*)&bitmap[key >> 6], 1ull << (key & 63));
    vidx[key] = id;
}

// ============================================================ k_seed ==
struct PolSeed {
    static constexpr int NB = 2;
    static constexpr bool COUNTS = false, SCATTER = false, MULTI = true;
    static constexpr int ROWS = kRows;
    struct Ctx {
        int base;
    };
    const float2* xy;
    const int* gstart;
    SetInfo* sets;
    int* err;

    __device__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ int group_start(int g) const { return gstart[g]; }
    __device__ int group_end(int g) const { return gstart[g + 1]; }
    __device__ Ctx ctx(int g) const { return Ctx{gstart[g]}; }
    __device__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = xy[q];
        x = v.x; y = v.y; id = q - c.base;
    }
    __device__ int classify(const Ctx&, int, int q, float x, float y, int id, Cand& k, Counters&) const
    {
        if (!(isfinite(x) && isfinite(y))) {
            atomicOr(err, kErrNonFinite);
            return 0;
        }
        k.a = 0.0f; k.w = 0.0f; k.x = x; k.y = y; k.id = id; k.pos = q;
        return 3;  // candidate for both lexmin (bucket 0) and lexmax (bucket 1)
    }
    // bucket 0: lexicographically smaller wins; bucket 1: larger wins; ties
    // (coincident points): lower index. Values compare as floats (-0 == +0).
    __device__ bool beats(const Ctx&, int k, const Cand& P, const Cand& Q, Counters&) const
    {
        if (Q.pos < 0) return P.pos >= 0;
        if (P.pos < 0) return false;
        if (P.x == Q.x && P.y == Q.y) return P.id < Q.id;
        const bool less = (P.x < Q.x) || (P.x == Q.x && P.y < Q.y);
        return k == 0 ? less : !less;
    }
    __device__ Cand fetch_cand(const Ctx& c, int, int pos, Counters&) const
    {
        const float2 v = xy[pos];
        Cand k;
        k.a = 0.0f; k.w = 0.0f; k.x = v.x; k.y = v.y; k.id = pos - c.base; k.pos = pos;
        return k;
    }
    __device__ int place(const Ctx&, int, int, int) const { return 0; }
    __device__ void store(int, float, float, int) const {}
    __device__ void finalize(const Ctx&, int g, const Agg<NB>& a) const
    {
        SetInfo& s = sets[g];
        s.ax = a.best[0].x; s.ay = a.best[0].y; s.aid = a.best[0].id; s.apos = a.best[0].pos;
        s.bx = a.best[1].x; s.by = a.best[1].y; s.bid = a.best[1].id; s.bpos = a.best[1].pos;
    }
};

// =========================================================== k_split ==
struct PolSplit {
    static constexpr int NB = 2;
    static constexpr bool COUNTS = true, SCATTER = false, MULTI = false;
    static constexpr int ROWS = kRows;
    struct Ctx {
        Edge ab, ba;
        int base, skip;
    };
    const float2* xy;
    const int* gstart;
    SetInfo* sets;
    uint64_t* bitmap;
    int* vidx;
    int fp64;

    __device__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ int group_start(int g) const { return gstart[g]; }
    __device__ int group_end(int g) const { return gstart[g + 1]; }
    __device__ Ctx ctx(int g) const
    {
        const SetInfo& s = sets[g];
        Ctx c;
        c.ab = make_edge(s.ax, s.ay, s.bx, s.by);
        c.ba = make_edge(s.bx, s.by, s.ax, s.ay);
        c.base = gstart[g];
        // lexmin and lexmax coincide only if every point sits at one position
        c.skip = (s.ax == s.bx) && (s.ay == s.by);
        return c;
    }
    __device__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = xy[q];
        x = v.x; y = v.y; id = q - c.base;
    }
    // lower side: strictly right of A->B; upper side: strictly left of A->B
    // (= strictly right of B->A). Points on the line -- A, B, duplicates and
    // collinear points -- belong to neither side.
    __device__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        if (c.skip) return kNone;
        Orient32 o;
        ++ctr.orient;
        const int sg = orient_sign(c.ab, x, y, fp64 != 0, o, ctr.orient_exact);
        if (sg == 0) return kNone;
        k.a = sg < 0 ? -o.d : o.d;
        k.w = 2.0f * o.es;
        k.x = x; k.y = y; k.id = id; k.pos = q;
        return sg < 0 ? 0 : 1;
    }
    __device__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(k == 0 ? c.ab : c.ba, P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ Cand fetch_cand(const Ctx& c, int k, int pos, Counters&) const
    {
        const float2 v = xy[pos];
        const Orient32 o = orient32(c.ab, v.x, v.y);
        Cand r;
        r.a = k == 0 ? -o.d : o.d;
        r.w = 2.0f * o.es;
        r.x = v.x; r.y = v.y; r.id = pos - c.base; r.pos = pos;
        return r;
    }
    __device__ int place(const Ctx&, int, int, int) const { return 0; }
    __device__ void store(int, float, float, int) const {}
    __device__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        SetInfo& s = sets[g];
        s.n_lo = a.cnt[0];
        s.n_up = a.cnt[1];
        s.clx = a.best[0].x; s.cly = a.best[0].y; s.clid = a.best[0].id;
        s.cux = a.best[1].x; s.cuy = a.best[1].y; s.cuid = a.best[1].id;
        // vertex keys: A at the set's first slot, B right after the lower side
        record_vertex(bitmap, vidx, c.base, s.aid);
        if (!c.skip) record_vertex(bitmap, vidx, c.base + 1 + a.cnt[0], s.bid);
    }
};

// =========================================================== k_first ==
// Slot layout of set s (base = its first slot, n_s slots):
//   base                               A
//   [base+1, base+1+n_lo)              lower side's points; child (A,C_lo)
//                                      packed from the front, child (C_lo,B)
//                                      from the back
//   base+1+n_lo                        B
//   [base+2+n_lo, base+2+n_lo+n_up)    upper side: (B,C_up) front, (C_up,A) back
struct PolFirst {
    static constexpr int NB = 4;
    static constexpr bool COUNTS = true, SCATTER = true, MULTI = false;
    static constexpr int ROWS = kRows;
    struct Ctx {
        Edge ab;
        Edge e[4];  // A->C_lo, C_lo->B, B->C_up, C_up->A
        int base, n_lo, n_up, skip;
    };
    const float2* xy;
    const int* gstart;
    const SetInfo* sets;
    float* X;
    float* Y;
    int* I;
    Seg* recs;
    int* rec_cid;
    uint64_t* bitmap;
    int* vidx;
    int fp64;

    __device__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ int group_start(int g) const { return gstart[g]; }
    __device__ int group_end(int g) const { return gstart[g + 1]; }
    __device__ Ctx ctx(int g) const
    {
        const SetInfo& s = sets[g];
        Ctx c;
        c.ab = make_edge(s.ax, s.ay, s.bx, s.by);
        c.e[0] = make_edge(s.ax, s.ay, s.clx, s.cly);
        c.e[1] = make_edge(s.clx, s.cly, s.bx, s.by);
        c.e[2] = make_edge(s.bx, s.by, s.cux, s.cuy);
        c.e[3] = make_edge(s.cux, s.cuy, s.ax, s.ay);
        c.base = gstart[g];
        c.n_lo = s.n_lo;
        c.n_up = s.n_up;
        c.skip = (s.ax == s.bx) && (s.ay == s.by);
        return c;
    }
    __device__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = xy[q];
        x = v.x; y = v.y; id = q - c.base;
    }
    // Section 4.4.3: a point of segment (A,B) with farthest point C is kept
    // for child (A,C) if strictly right of A->C, for child (C,B) if strictly
    // right of C->B, and discarded otherwise (inside or on triangle ACB; the
    // paper's "and" must read "or": no point is right of both lines).
    __device__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        if (c.skip) return kNone;
        Orient32 o;
        ++ctr.orient;
        const int side = orient_sign(c.ab, x, y, fp64 != 0, o, ctr.orient_exact);
        if (side == 0) return kNone;
        const bool up = side > 0;
        const Edge& E1 = up ? c.e[2] : c.e[0];
        const Edge& E2 = up ? c.e[3] : c.e[1];
        ++ctr.orient;
        if (orient_sign(E1, x, y, fp64 != 0, o, ctr.orient_exact) < 0) {
            k = make_cand(o, x, y, id, q);
            return up ? 2 : 0;
        }
        ++ctr.orient;
        if (orient_sign(E2, x, y, fp64 != 0, o, ctr.orient_exact) < 0) {
            k = make_cand(o, x, y, id, q);
            return up ? 3 : 1;
        }
        return kNone;
    }
    __device__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(c.e[k], P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ Cand fetch_cand(const Ctx& c, int k, int pos, Counters&) const
    {
        const float2 v = xy[pos];
        return make_cand(orient32(c.e[k], v.x, v.y), v.x, v.y, pos - c.base, pos);
    }
    __device__ int place(const Ctx& c, int, int k, int rank) const
    {
        switch (k) {
        case 0: return c.base + 1 + rank;
        case 1: return c.base + c.n_lo - rank;
        case 2: return c.base + 2 + c.n_lo + rank;
        default: return c.base + 1 + c.n_lo + c.n_up - rank;
        }
    }
    __device__ void store(int dst, float x, float y, int id) const
    {
        X[dst] = x; Y[dst] = y; I[dst] = id;
    }
    __device__ void child(int slot, const Edge& E, const Cand& C, int off, int len) const
    {
        Seg r;
        r.ax = E.ox; r.ay = E.oy; r.bx = E.ex; r.by = E.ey;
        r.cx = C.x; r.cy = C.y;
        r.off = off; r.len = len;
        recs[slot] = r;
        rec_cid[slot] = C.id;
    }
    __device__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        const SetInfo& s = sets[g];
        if (c.n_lo > 0) {
            record_vertex(bitmap, vidx, c.base + 1 + a.cnt[0], s.clid);
            child(4 * g + 0, c.e[0], a.best[0], c.base + 1, a.cnt[0]);
            child(4 * g + 1, c.e[1], a.best[1], c.base + 1 + c.n_lo - a.cnt[1], a.cnt[1]);
        }
        if (c.n_up > 0) {
            record_vertex(bitmap, vidx, c.base + 2 + c.n_lo + a.cnt[2], s.cuid);
            child(4 * g + 2, c.e[2], a.best[2], c.base + 2 + c.n_lo, a.cnt[2]);
            child(4 * g + 3, c.e[3], a.best[3], c.base + 2 + c.n_lo + c.n_up - a.cnt[3], a.cnt[3]);
        }
    }
};

// ============================================================ k_pass ==
// Positions are virtual: segment g owns [vstart[g], vstart[g+1]) and its
// points sit in slots [off, off+len) of the input buffer. Children are packed
// into the parent's slots: (A,C) from the front, (C,B) from the back; C's
// key is the first slot after the (A,C) points.
struct PolPass {
    static constexpr int NB = 2;
    static constexpr bool COUNTS = true, SCATTER = true, MULTI = false;
    static constexpr int ROWS = kRows;
    struct Ctx {
        Edge e[2];  // A->C, C->B
        int off, len, vstart;
    };
    const Seg* segs;
    const int* seg_cid;
    const int* vstart;
    const float* Xi;
    const float* Yi;
    const int* Ii;
    float* Xo;
    float* Yo;
    int* Io;
    Seg* recs;
    int* rec_cid;
    uint64_t* bitmap;
    int* vidx;
    int fp64;

    __device__ int group_of(int q, int lo, int hi) const { return search_le(vstart, q, lo, hi); }
    __device__ int group_start(int g) const { return vstart[g]; }
    __device__ int group_end(int g) const { return vstart[g + 1]; }
    __device__ Ctx ctx(int g) const
    {
        const Seg s = segs[g];
        Ctx c;
        c.e[0] = make_edge(s.ax, s.ay, s.cx, s.cy);
        c.e[1] = make_edge(s.cx, s.cy, s.bx, s.by);
        c.off = s.off;
        c.len = s.len;
        c.vstart = vstart[g];
        return c;
    }
    __device__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const int p = c.off + (q - c.vstart);
        x = Xi[p]; y = Yi[p]; id = Ii[p];
    }
    __device__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        Orient32 o;
        const int p = c.off + (q - c.vstart);
        ++ctr.orient;
        if (orient_sign(c.e[0], x, y, fp64 != 0, o, ctr.orient_exact) < 0) {
            k = make_cand(o, x, y, id, p);
            return 0;
        }
        ++ctr.orient;
        if (orient_sign(c.e[1], x, y, fp64 != 0, o, ctr.orient_exact) < 0) {
            k = make_cand(o, x, y, id, p);
            return 1;
        }
        return kNone;
    }
    __device__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(c.e[k], P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ Cand fetch_cand(const Ctx& c, int k, int pos, Counters&) const
    {
        const float x = Xi[pos], y = Yi[pos];
        return make_cand(orient32(c.e[k], x, y), x, y, Ii[pos], pos);
    }
    __device__ int place(const Ctx& c, int, int k, int rank) const
    {
        return k == 0 ? c.off + rank : c.off + c.len - 1 - rank;
    }
    __device__ void store(int dst, float x, float y, int id) const
    {
        Xo[dst] = x; Yo[dst] = y; Io[dst] = id;
    }
    __device__ void child(int slot, const Edge& E, const Cand& C, int off, int len) const
    {
        Seg r;
        r.ax = E.ox; r.ay = E.oy; r.bx = E.ex; r.by = E.ey;
        r.cx = C.x; r.cy = C.y;
        r.off = off; r.len = len;
        recs[slot] = r;
        rec_cid[slot] = C.id;
    }
    __device__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        record_vertex(bitmap, vidx, c.off + a.cnt[0], seg_cid[g]);
        child(2 * g + 0, c.e[0], a.best[0], c.off, a.cnt[0]);
        child(2 * g + 1, c.e[1], a.best[1], c.off + c.len - a.cnt[1], a.cnt[1]);
    }
};

template <class Pol>
__global__ __launch_bounds__(kBlock) void k_tiles(Pol pol, const int* Pp, int Pc, const int* Gp, int Gc,
                                                  int nt_cap, uint64_t* lb, int* err, uint32_t* stats)
{
    __shared__ TileShared<Pol> sh;
    const int P = Pp ? *Pp : Pc;
    const int G = Gp ? *Gp : Gc;
    constexpr int T = Pol::ROWS * 64 * kWaves;
    const int nt = (P + T - 1) / T;
    if (nt > nt_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, kErrBounds);
        return;
    }
    Counters ctr = {0u, 0u, 0u};
    for (int t = blockIdx.x; t < nt; t += gridDim.x) process_tile(pol, t, P, G, lb, err, sh, ctr);
    flush_counters(stats, ctr);
}

template __global__ void k_tiles<PolSeed>(PolSeed, const int*, int, const int*, int, int, uint64_t*, int*, uint32_t*);
template __global__ void k_tiles<PolSplit>(PolSplit, const int*, int, const int*, int, int, uint64_t*, int*, uint32_t*);
template __global__ void k_tiles<PolFirst>(PolFirst, const int*, int, const int*, int, int, uint64_t*, int*, uint32_t*);
template __global__ void k_tiles<PolPass>(PolPass, const int*, int, const int*, int, int, uint64_t*, int*, uint32_t*);

// ================================================== ordered scans ==
// Exclusive scan of (a, b) pairs over items with one-word decoupled look-back
// (no groups). Used to rebuild the segment table and to rank hull vertices.
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

struct Pair {
    int a, b;
};

__device__ __forceinline__ Pair wave_incl_scan(Pair v)
{
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int oa = __shfl_up(v.a, d), ob = __shfl_up(v.b, d);
        if (lane >= d) { v.a += oa; v.b += ob; }
    }
    return v;
}

// Block-wide exclusive scan of one pair per thread; returns the block total
// in *tot. Uses sh[kWaves].
__device__ __forceinline__ Pair block_excl_scan(Pair v, Pair* sh, Pair* tot)
{
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const Pair inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    Pair off = {0, 0}, all = {0, 0};
#pragma unroll
    for (int u = 0; u < kWaves; ++u) {
        if (u < w) { off.a += sh[u].a; off.b += sh[u].b; }
        all.a += sh[u].a; all.b += sh[u].b;
    }
    *tot = all;
    __syncthreads();
    return Pair{off.a + inc.a - v.a, off.b + inc.b - v.b};
}

// prefix of tile t's predecessors (window look-back by one wave)
__device__ Pair scan_look_back(const uint64_t* lb, int t, int* err)
{
    const int lane = lane_id();
    Pair acc = {0, 0};
    int base = t - 1, spins = 0;
    while (true) {
        const int j = base - lane;
        uint64_t wv = 0;
        bool inc_ok = false, agg_ok = false;
        if (j >= 0) {
            wv = ld_word(lb + 2 * (size_t)j + 1);
            inc_ok = word_ok(wv);
            if (!inc_ok) {
                wv = ld_word(lb + 2 * (size_t)j);
                agg_ok = word_ok(wv);
            }
        }
        const uint64_t incm = __ballot(inc_ok);
        const uint64_t rdym = __ballot(inc_ok || agg_ok || j < 0);
        const int first_inc = incm ? (__ffsll((unsigned long long)incm) - 1) : 64;
        const uint64_t need = first_inc < 64 ? mask_le(first_inc) : ~0ull;
        if ((rdym & need) != need) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(err, kErrSpin);
                return acc;
            }
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        int a = 0, b = 0;
        if (lane <= first_inc && j >= 0) { a = (int)word_hi(wv); b = (int)word_lo(wv); }
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) { a += __shfl_xor(a, m); b += __shfl_xor(b, m); }
        acc.a += a; acc.b += b;
        if (first_inc < 64 || base - 63 <= 0) break;
        base -= 64;
    }
    return acc;
}

// Tile prefix with publication; all threads get the result.
__device__ __forceinline__ Pair tile_prefix(uint64_t* lb, int t, Pair tot, Pair* shp, int* err)
{
    if (threadIdx.x < 64) {
        Pair pre = {0, 0};
        if (t == 0) {
            if (threadIdx.x == 0) st_word(lb + 1, pack2(tot.a, tot.b));
        } else {
            if (threadIdx.x == 0) st_word(lb + 2 * (size_t)t, pack2(tot.a, tot.b));
            pre = scan_look_back(lb, t, err);
            if (threadIdx.x == 0) st_word(lb + 2 * (size_t)t + 1, pack2(pre.a + tot.a, pre.b + tot.b));
        }
        if (threadIdx.x == 0) *shp = pre;
    }
    __syncthreads();
    const Pair r = *shp;
    __syncthreads();
    return r;
}

// Segment-table rebuild: the child records recs[0..M) (M = mul * *nprev, or
// Mc if nprev is null) in ring order; active ones (len > 0) are compacted
// into segs with vstart = running sum of len. out_sv = {S, V}.
__global__ __launch_bounds__(kBlock) void k_table(const Seg* recs, const int* rec_cid, const int* nprev, int mul,
                                                  int Mc, Seg* segs, int* seg_cid, int* vstart, int* out_sv,
                                                  int nt_cap, uint64_t* lb, int* err)
{
    __shared__ Pair shw[kWaves];
    __shared__ Pair shp;
    const int M = nprev ? mul * (*nprev) : Mc;
    const int nt = (M + kScanTile - 1) / kScanTile;
    if (nt > nt_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, kErrBounds);
        return;
    }
    if (M == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { out_sv[0] = 0; out_sv[1] = 0; vstart[0] = 0; }
        return;
    }
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int i0 = t * kScanTile + (int)threadIdx.x * kScanItems;
        Pair mine = {0, 0};
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = i0 + k;
            if (i < M) {
                const int len = recs[i].len;
                if (len > 0) { mine.a += 1; mine.b += len; }
            }
        }
        Pair tot;
        const Pair ex = block_excl_scan(mine, shw, &tot);
        const Pair pre = tile_prefix(lb, t, tot, &shp, err);
        Pair at = {pre.a + ex.a, pre.b + ex.b};
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = i0 + k;
            if (i < M) {
                const Seg r = recs[i];
                if (r.len > 0) {
                    segs[at.a] = r;
                    seg_cid[at.a] = rec_cid[i];
                    vstart[at.a] = at.b;
                    at.a += 1;
                    at.b += r.len;
                }
            }
        }
        if (t == nt - 1 && threadIdx.x == 0) {
            out_sv[0] = pre.a + tot.a;
            out_sv[1] = pre.b + tot.b;
            vstart[pre.a + tot.a] = pre.b + tot.b;
        }
    }
}

// Ordered emission: vertex keys are the set bits of bitmap[0..W); the rank of
// a key among all set bits is its output position (keys increase along each
// set's ring and sets are stored in order). wprefix[w] = set bits before word w.
__global__ __launch_bounds__(kBlock) void k_emit(const uint64_t* bitmap, const int* vidx, int W, int32_t* out,
                                                 int64_t cap, int* wprefix, int* total, int nt_cap, uint64_t* lb,
                                                 int* err)
{
    __shared__ Pair shw[kWaves];
    __shared__ Pair shp;
    const int nt = (W + kScanTile - 1) / kScanTile;
    if (nt > nt_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, kErrBounds);
        return;
    }
    if (W == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *total = 0;
        return;
    }
    for (int t = blockIdx.x; t < nt; t += gridDim.x) {
        const int i0 = t * kScanTile + (int)threadIdx.x * kScanItems;
        uint64_t wd[kScanItems];
        Pair mine = {0, 0};
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = i0 + k;
            wd[k] = i < W ? bitmap[i] : 0ull;
            mine.a += __popcll(wd[k]);
        }
        Pair tot;
        const Pair ex = block_excl_scan(mine, shw, &tot);
        const Pair pre = tile_prefix(lb, t, tot, &shp, err);
        int rank = pre.a + ex.a;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            const int i = i0 + k;
            if (i < W) {
                wprefix[i] = rank;
                uint64_t bits = wd[k];
                while (bits) {
                    const int b = __ffsll((unsigned long long)bits) - 1;
                    bits &= bits - 1;
                    if (rank < cap) out[rank] = vidx[i * 64 + b];
                    ++rank;
                }
            }
        }
        if (t == nt - 1 && threadIdx.x == 0) *total = pre.a + tot.a;
    }
}

// Output offsets of a batch: out_off[s] = vertices with key < set_off[s].
__global__ void k_out_offsets(const int* gstart, int nsets, int N, const uint64_t* bitmap, const int* wprefix,
                              const int* total, int64_t* out_off)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nsets) return;
    const int key = gstart[s];
    int64_t v;
    if (key >= N) {
        v = *total;
    } else {
        const int w = key >> 6;
        v = wprefix[w] + __popcll(bitmap[w] & mask_lt(key & 63));
    }
    out_off[s] = v;
}

// int64 set offsets -> int32 group starts, with validation.
__global__ void k_prep_sets(const int64_t* set_off, int nsets, int64_t n_total, int* gstart, int* err)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > nsets) return;
    const int64_t v = set_off[s];
    bool bad = v < 0 || v > n_total;
    if (s == 0 && v != 0) bad = true;
    if (s == nsets && v != n_total) bad = true;
    if (s > 0 && set_off[s - 1] > v) bad = true;
    if (bad) atomicOr(err, kErrBounds);
    gstart[s] = bad ? 0 : (int)v;
}

__global__ void k_single_set(int* gstart, int n)
{
    if (threadIdx.x == 0) { gstart[0] = 0; gstart[1] = n; }
}

}  // namespace sqh
