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
#include <type_traits>

#include "sqh_pred.hpp"
#include "sqh_chunk.hpp"
#include "sqh_types.hpp"

namespace sqh {

constexpr int kRows = 8;  // rows of 64 positions per wave: tile = 2048 positions

__device__ __forceinline__ int search_le(const int* start, int q, int lo, int hi)
{
    // largest g in [lo, hi] with start[g] <= q (start[lo] <= q is assumed)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (gld(start + mid) <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A hull vertex gets a key: a slot of the survivor index space that no
// point and no other vertex of its set uses, increasing along the ring
// (counter-clockwise from the set's lexmin point). The emit step orders
// vertices by key.
struct HullInfo;
__device__ void note_vertex(HullInfo* info, int2* vlist, int key, int id);
// vlist == nullptr: no vertex list (the emission ranks the bitmap)
__device__ __forceinline__ void record_vertex(uint64_t* bitmap, int* vidx, int2* vlist, HullInfo* info, int key,
                                              int id)
{
    atomicOr((unsigned long long*)&bitmap[key >> 6], 1ull << (key & 63));
    gst(vidx + key, id);
    if (vlist) note_vertex(info, vlist, key, id);
}

// ============================================================ k_seed ==
template <bool IDS>
struct PolSeedT {
    static constexpr int NB = 2;
    static constexpr bool COUNTS = false, SCATTER = false, MULTI = true, MIDDLE = false;
    static constexpr int ROWS = kRows;
    struct Ctx {
        int base;
    };
    const float2* xy;
    const int* gstart;
    SetInfo* sets;
    int* err;
    const int* ids;  // IDS: each position's input index (a pre-filtered subset)
    int* bad;  // null, or one flag per set raised by a non-finite coordinate
    int G;

    __device__ __forceinline__ int num_groups() const { return G; }
    __device__ __forceinline__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ __forceinline__ int group_start(int g) const { return gld(gstart + g); }
    __device__ __forceinline__ int group_end(int g) const { return gld(gstart + g + 1); }
    __device__ __forceinline__ Ctx ctx(int g) const { return Ctx{gld(gstart + g)}; }
    __device__ __forceinline__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = gld(xy + q);
        x = v.x; y = v.y;
        if constexpr (IDS) id = gld(ids + q);
        else id = q - c.base;
    }
    __device__ __forceinline__ int classify(const Ctx&, int g, int q, float x, float y, int id, Cand& k, Counters&) const
    {
        if (!(isfinite(x) && isfinite(y))) {
            atomicOr(err, kErrNonFinite);
            if (bad) bad[g] = 1;
            return 0;
        }
        k.a = 0.0f; k.w = 0.0f; k.x = x; k.y = y; k.id = id;
        return 3;  // candidate for both lexmin (bucket 0) and lexmax (bucket 1)
    }
    // bucket 0: lexicographically smaller wins; bucket 1: larger wins; ties
    // (coincident points): lower index. Values compare as floats (-0 == +0).
    __device__ __forceinline__ int beats_fast(const Ctx&, int k, const Cand& P, const Cand& Q) const
    {
        const bool less = (P.x < Q.x) | ((P.x == Q.x) & (P.y < Q.y));
        const bool more = (P.x > Q.x) | ((P.x == Q.x) & (P.y > Q.y));
        const bool eq = (P.x == Q.x) & (P.y == Q.y);
        const bool w = (k == 0 ? less : more) | (eq & (P.id < Q.id));
        const bool r = (Q.id < 0) ? (P.id >= 0) : ((P.id >= 0) & w);
        return r ? 1 : 0;
    }
    __device__ __forceinline__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters&) const
    {
        return beats_fast(c, k, P, Q) > 0;
    }
    __device__ __forceinline__ int place(const Ctx&, int, int, int) const { return 0; }
    __device__ __forceinline__ void store(int, float, float, int) const {}
    __device__ __forceinline__ void finalize(const Ctx&, int g, const Agg<NB>& a) const
    {
        SetInfo s = gld(sets + g);
        s.ax = a.best[0].x; s.ay = a.best[0].y; s.aid = a.best[0].id;
        s.bx = a.best[1].x; s.by = a.best[1].y; s.bid = a.best[1].id;
        gst(sets + g, s);
    }
};
using PolSeed = PolSeedT<false>;

// ====================================================== pre-filter ==
// The paper's first mode (section 4.2) drops the points inside the
// quadrilateral of the extreme points in x and y before the first split;
// the octagon adds the extremes of x + y and x - y.
//
// Corner k is, among the points whose projection on direction k is extreme,
// the one of lowest index; the diagonal projections are the float32 sums
// fl(x + y) and fl(x - y), and -0 counts as +0. Directions, counter-clockwise
// from -x:
//   0 min x   1 min x + y   2 min y   3 max x - y
//   4 max x   5 max x + y   6 max y   7 min x - y
// Neither the rounding nor the tie rule matters for the hull. The corners
// are input points; a point strictly left of every edge of the closed
// polygon through them sees each edge turn by a positive angle, so its
// winding number is positive and it lies in the interior of the corners'
// convex hull, hence of the input's: it is no hull vertex. A point at a
// corner's position is on an edge that starts there, so it is never
// certified inside; if all corners coincide there is no edge and every
// point is kept. The subset (points not certified inside, with their input
// indices) therefore holds every hull vertex and every copy of one, and its
// hull, tie rules included, is the input's. "Strictly left" is certified by
// the float32 orientation filter; an overflow in it makes the bound
// infinite or NaN, which certifies nothing.

// order-preserving map of a float32 onto uint32 (for non-NaN values)
__device__ __forceinline__ uint32_t ord32(float f)
{
    const uint32_t u = __float_as_uint(f);
    return u ^ ((uint32_t)((int32_t)u >> 31) | 0x80000000u);
}

// Directions 3, 4, 5, 6 take the largest projection, the others the
// smallest. Across lanes and workgroups an extreme is carried as one 64-bit
// key: high word the projection's order, low word the index (smallest-key
// directions) or its complement (largest-key directions), so that the
// extreme key names the lowest index among the extreme projections.
constexpr uint32_t kExtMax = 0x78u;

__device__ __forceinline__ bool ext_is_max(int k) { return (kExtMax >> k) & 1u; }
__device__ __forceinline__ uint64_t ext_none(int k) { return ext_is_max(k) ? 0ull : ~0ull; }
__device__ __forceinline__ uint64_t ext_key(int k, float v, int id)
{
    if (id < 0) return ext_none(k);
    const uint32_t o = ord32(v + 0.0f);  // -0 -> +0
    return ((uint64_t)o << 32) | (ext_is_max(k) ? ~(uint32_t)id : (uint32_t)id);
}
__device__ __forceinline__ uint64_t ext_pick(int k, uint64_t a, uint64_t b)
{
    return ext_is_max(k) ? (a > b ? a : b) : (a < b ? a : b);
}
__device__ __forceinline__ int ext_index(int k, uint64_t key)
{
    const uint32_t lo = (uint32_t)key;
    return (int)(ext_is_max(k) ? ~lo : lo);
}

// One lane's extremes: its points come in increasing index order, so a
// strict comparison keeps the lowest index among equal projections.
struct ExtLane {
    float v[8];
    int id[8];
    __device__ __forceinline__ void init()
    {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = ext_is_max(k) ? -INFINITY : INFINITY;
            id[k] = -1;
        }
    }
    __device__ __forceinline__ void add(float x, float y, int q)
    {
        const float s = x + y, d = x - y;
        const float pr[8] = {x, s, y, d, x, s, y, d};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool t = ext_is_max(k) ? (pr[k] > v[k]) : (pr[k] < v[k]);
            v[k] = t ? pr[k] : v[k];
            id[k] = t ? q : id[k];
        }
    }
};

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// The polygon's non-degenerate edges, wave-uniform (n = 0: all corners
// coincide, every point is kept).
//
// Line test (|coordinates| <= 2^60): edge o -> o + (dx, dy) (dx, dy rounded)
// as t = fma(nx, px, fma(ny, py, c)), nx = -dy, ny = dx, c = fl(fl(dy ox) -
// fl(dx oy)). With D = |dx| My + |dy| Mx, where Mx, My bound |x|, |y| over
// the input (the extremes in x and y), the rounding of the differences, of
// c and of both fma's moves t from the exact orientation of (o, e, p) by at
// most 9 u D (1 + 10 u) plus 5 * 2^-150 in the subnormal range (u = 2^-24),
// so t > m = 2^-19 D + 2^-140 (32 u D) proves the orientation positive. The
// bound on the coordinates keeps every term below 2^123 (no overflow).
// Larger coordinates use the float32 orientation filter, whose overflow
// gives an infinite or NaN bound and certifies nothing.
constexpr float kLineCoordMax = 0x1p60f;
constexpr float kLineRel = 0x1p-19f;

struct KeepEdges {
    float nx[8], ny[8], c[8], m[8];
    int n;
    bool line;  // the line test applies (else the orientation filter)
};

// edges in LDS for the orientation filter: ox, oy, dx, dy per edge
struct KeepLds {
    float e[4][8];
};

// corners cx, cy in direction order (the quadrilateral uses the even ones)
__device__ __forceinline__ void keep_build(KeepEdges& E, KeepLds& L, const float (&cx)[8], const float (&cy)[8],
                                           bool quad)
{
    const float Mx = fmaxf(fabsf(cx[0]), fabsf(cx[4]));  // min x, max x
    const float My = fmaxf(fabsf(cy[2]), fabsf(cy[6]));  // min y, max y
    E.line = fmaxf(Mx, My) <= kLineCoordMax;
    E.n = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) E.nx[i] = E.ny[i] = E.c[i] = E.m[i] = 0.0f;
    const bool w0 = threadIdx.x == 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (quad && (i & 1)) continue;
        const int j = quad ? ((i + 2) & 7) : ((i + 1) & 7);
        if (cx[i] == cx[j] && cy[i] == cy[j]) continue;  // zero-length edge
        const float dx = cx[j] - cx[i], dy = cy[j] - cy[i];
        const float cc = dy * cx[i] - dx * cy[i];
        const float mm = (fabsf(dx) * My + fabsf(dy) * Mx) * kLineRel + kFilterTau;
        // (placed with selects so that the arrays stay in registers)
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            if (t == E.n) {
                E.nx[t] = -dy;
                E.ny[t] = dx;
                E.c[t] = cc;
                E.m[t] = mm;
                if (w0) {
                    L.e[0][t] = cx[i];
                    L.e[1][t] = cy[i];
                    L.e[2][t] = dx;
                    L.e[3][t] = dy;
                }
            }
        }
        ++E.n;
    }
}

// keep p: not certified strictly left of every edge
__device__ __forceinline__ bool keep_point(const KeepEdges& E, const KeepLds& L, float px, float py, Counters& ctr)
{
    if (E.n == 0) return true;
    bool in = true;
    if (E.line) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < E.n) in = in && fmaf(E.nx[i], px, fmaf(E.ny[i], py, E.c[i])) > E.m[i];
        }
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (i < E.n) {
                const float P = L.e[2][i] * (py - L.e[1][i]);
                const float Q = L.e[3][i] * (px - L.e[0][i]);
                const float d = P - Q;
                const float es = (fabsf(P) + fabsf(Q)) * kFilterScale + kFilterTau;
                in = in && d > es;
            }
        }
    }
    ctr.orient += (uint32_t)E.n;
    return !in;
}

// =========================================================== k_split ==
template <bool IDS>
struct PolSplitT {
    static constexpr int NB = 2;
    static constexpr bool COUNTS = true, SCATTER = false, MULTI = false, MIDDLE = false;
    static constexpr int ROWS = kRows;
    struct Ctx {
        float ax, ay, bx, by;   // A->B and B->A are rebuilt where used
        int base, sbase, skip;  // first read position, first slot (vertex keys)
        __device__ __forceinline__ Edge ab() const { return make_edge(ax, ay, bx, by); }
        __device__ __forceinline__ Edge ba() const { return make_edge(bx, by, ax, ay); }
    };
    const float2* xy;
    const int* gstart;
    const int* sbase;
    const int* bad;  // null, or sets to skip (non-finite input)
    const int* ids;  // IDS: each position's input index (a pre-filtered subset)
    SetInfo* sets;
    uint64_t* bitmap;
    int* vidx;
    int2* vlist;
    HullInfo* info;
    int fp64;
    int G;

    __device__ __forceinline__ int num_groups() const { return G; }
    __device__ __forceinline__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ __forceinline__ int group_start(int g) const { return gld(gstart + g); }
    __device__ __forceinline__ int group_end(int g) const { return gld(gstart + g + 1); }
    __device__ __forceinline__ Ctx ctx(int g) const
    {
        const SetInfo s = gld(sets + g);
        Ctx c;
        c.ax = s.ax; c.ay = s.ay; c.bx = s.bx; c.by = s.by;
        c.base = gld(gstart + g);
        c.sbase = gld(sbase + g);
        // lexmin and lexmax coincide only if every point sits at one position
        c.skip = ((s.ax == s.bx) && (s.ay == s.by)) || (bad && gld(bad + g));
        return c;
    }
    __device__ __forceinline__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = gld(xy + q);
        x = v.x; y = v.y;
        if constexpr (IDS) id = gld(ids + q);
        else id = q - c.base;
    }
    // lower side: strictly right of A->B; upper side: strictly left of A->B
    // (= strictly right of B->A). Points on the line -- A, B, duplicates and
    // collinear points -- belong to neither side.
    __device__ __forceinline__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        if (c.skip) return kNone;
        ++ctr.orient;
        const Orient32 o = orient32p(c.ax, c.ay, c.bx, c.by, x, y);
        int sg = fast_sign(o, fp64 != 0);
        settle_p(sg, sg == 0, c.ax, c.ay, c.bx, c.by, x, y, ctr.orient_exact);
        k.a = sg < 0 ? -o.d : o.d;
        k.w = 2.0f * o.es;
        k.x = x; k.y = y; k.id = id;
        return sg < 0 ? 0 : (sg > 0 ? 1 : kNone);
    }
    __device__ __forceinline__ int beats_fast(const Ctx&, int, const Cand& P, const Cand& Q) const
    {
        return sqh::beats_fast(P, Q, fp64 != 0);
    }
    __device__ __forceinline__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(k == 0 ? c.ab() : c.ba(), P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ __forceinline__ int place(const Ctx&, int, int, int) const { return 0; }
    __device__ __forceinline__ void store(int, float, float, int) const {}
    __device__ __forceinline__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        SetInfo s = gld(sets + g);
        s.n_lo = a.cnt[0];
        s.n_up = a.cnt[1];
        s.clx = a.best[0].x; s.cly = a.best[0].y; s.clid = a.best[0].id;
        s.cux = a.best[1].x; s.cuy = a.best[1].y; s.cuid = a.best[1].id;
        gst(sets + g, s);
        // vertex keys: A at the set's first slot, B right after the lower side
        record_vertex(bitmap, vidx, vlist, info, c.sbase, s.aid);
        if (!c.skip) record_vertex(bitmap, vidx, vlist, info, c.sbase + 1 + a.cnt[0], s.bid);
    }
};
using PolSplit = PolSplitT<false>;

// =========================================================== k_first ==
// Slot layout of set s (base = its first slot, n_s slots):
//   base                               A
//   [base+1, base+1+n_lo)              lower side's points; child (A,C_lo)
//                                      packed from the front, child (C_lo,B)
//                                      from the back
//   base+1+n_lo                        B
//   [base+2+n_lo, base+2+n_lo+n_up)    upper side: (B,C_up) front, (C_up,A) back
template <bool IDS>
struct PolFirstT {
    static constexpr int NB = 4;
    static constexpr bool COUNTS = true, SCATTER = true, MULTI = false, MIDDLE = false;
    static constexpr int ROWS = kRows;
    // A, B, C_lo, C_up as loaded; the edges A->B, A->C_lo, C_lo->B, B->C_up
    // and C_up->A are rebuilt where used
    struct Ctx {
        float ax, ay, bx, by, lx, ly, ux, uy;
        int base, sbase, n_lo, n_up, skip;  // first read position, first slot
        __device__ __forceinline__ Edge ab() const { return make_edge(ax, ay, bx, by); }
        __device__ __forceinline__ Edge edge(int k) const
        {
            switch (k) {
            case 0: return make_edge(ax, ay, lx, ly);
            case 1: return make_edge(lx, ly, bx, by);
            case 2: return make_edge(bx, by, ux, uy);
            default: return make_edge(ux, uy, ax, ay);
            }
        }
    };
    const float2* xy;
    const int* gstart;
    const int* sbase;
    const int* bad;
    const int* ids;  // IDS: each position's input index (a pre-filtered subset)
    const SetInfo* sets;
    float* X;
    float* Y;
    int* I;
    Seg* recs;
    int* rec_cid;
    uint64_t* bitmap;
    int* vidx;
    int2* vlist;
    HullInfo* info;
    int fp64;
    int G;

    __device__ __forceinline__ int num_groups() const { return G; }
    __device__ __forceinline__ int group_of(int q, int lo, int hi) const { return search_le(gstart, q, lo, hi); }
    __device__ __forceinline__ int group_start(int g) const { return gld(gstart + g); }
    __device__ __forceinline__ int group_end(int g) const { return gld(gstart + g + 1); }
    __device__ __forceinline__ Ctx ctx(int g) const
    {
        const SetInfo s = gld(sets + g);
        Ctx c;
        c.ax = s.ax; c.ay = s.ay; c.bx = s.bx; c.by = s.by;
        c.lx = s.clx; c.ly = s.cly; c.ux = s.cux; c.uy = s.cuy;
        c.base = gld(gstart + g);
        c.sbase = gld(sbase + g);
        c.n_lo = s.n_lo;
        c.n_up = s.n_up;
        c.skip = ((s.ax == s.bx) && (s.ay == s.by)) || (bad && gld(bad + g));
        return c;
    }
    __device__ __forceinline__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const float2 v = gld(xy + q);
        x = v.x; y = v.y;
        if constexpr (IDS) id = gld(ids + q);
        else id = q - c.base;
    }
    // Section 4.4.3: a point of segment (A,B) with farthest point C is kept
    // for child (A,C) if strictly right of A->C, for child (C,B) if strictly
    // right of C->B, and discarded otherwise (inside or on triangle ACB; the
    // paper's "and" must read "or": no point is right of both lines).
    __device__ __forceinline__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        if (c.skip) return kNone;
        const bool f64 = fp64 != 0;
        ctr.orient += 3;
        const Orient32 o = orient32p(c.ax, c.ay, c.bx, c.by, x, y);
        int side = fast_sign(o, f64);
        settle_p(side, side == 0, c.ax, c.ay, c.bx, c.by, x, y, ctr.orient_exact);
        const bool up = side > 0;
        // lower side: A->C_lo, C_lo->B; upper side: B->C_up, C_up->A; the
        // two edges share the apex C
        const float sx = up ? c.bx : c.ax, sy = up ? c.by : c.ay;  // first edge's start
        const float mx = up ? c.ux : c.lx, my = up ? c.uy : c.ly;  // apex
        const float tx = up ? c.ax : c.bx, ty = up ? c.ay : c.by;  // second edge's end
        const Orient32 o1 = orient32p(sx, sy, mx, my, x, y);
        const Orient32 o2 = orient32p(mx, my, tx, ty, x, y);
        int s1 = fast_sign(o1, f64), s2 = fast_sign(o2, f64);
        settle_p(s1, side != 0 && s1 == 0, sx, sy, mx, my, x, y, ctr.orient_exact);
        settle_p(s2, side != 0 && s1 >= 0 && s2 == 0, mx, my, tx, ty, x, y, ctr.orient_exact);
        const bool in1 = s1 < 0, in2 = !in1 && s2 < 0;
        k = make_cand(in1 ? o1 : o2, x, y, id);
        const int b = up ? 2 : 0;
        return side == 0 ? kNone : (in1 ? b : (in2 ? b + 1 : kNone));
    }
    __device__ __forceinline__ int beats_fast(const Ctx&, int, const Cand& P, const Cand& Q) const
    {
        return sqh::beats_fast(P, Q, fp64 != 0);
    }
    __device__ __forceinline__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(c.edge(k), P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ __forceinline__ int place(const Ctx& c, int, int k, int rank) const
    {
        switch (k) {
        case 0: return c.sbase + 1 + rank;
        case 1: return c.sbase + c.n_lo - rank;
        case 2: return c.sbase + 2 + c.n_lo + rank;
        default: return c.sbase + 1 + c.n_lo + c.n_up - rank;
        }
    }
    __device__ __forceinline__ void store(int dst, float x, float y, int id) const
    {
        gst(X + dst, x); gst(Y + dst, y); gst(I + dst, id);
    }
    __device__ __forceinline__ void child(int slot, const Edge& E, const Cand& C, int off, int len) const
    {
        Seg r;
        r.ax = E.ox; r.ay = E.oy; r.bx = E.ex; r.by = E.ey;
        r.cx = C.x; r.cy = C.y;
        r.off = off; r.len = len;
        gst(recs + slot, r);
        gst(rec_cid + slot, C.id);
    }
    __device__ __forceinline__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        const SetInfo s = gld(sets + g);
        if (c.n_lo > 0) {
            record_vertex(bitmap, vidx, vlist, info, c.sbase + 1 + a.cnt[0], s.clid);
            child(4 * g + 0, c.edge(0), a.best[0], c.sbase + 1, a.cnt[0]);
            child(4 * g + 1, c.edge(1), a.best[1], c.sbase + 1 + c.n_lo - a.cnt[1], a.cnt[1]);
        }
        if (c.n_up > 0) {
            record_vertex(bitmap, vidx, vlist, info, c.sbase + 2 + c.n_lo + a.cnt[2], s.cuid);
            child(4 * g + 2, c.edge(2), a.best[2], c.sbase + 2 + c.n_lo, a.cnt[2]);
            child(4 * g + 3, c.edge(3), a.best[3], c.sbase + 2 + c.n_lo + c.n_up - a.cnt[3], a.cnt[3]);
        }
    }
};
using PolFirst = PolFirstT<false>;

// ============================================================ k_pass ==
// Positions are virtual: segment g owns [vstart[g], vstart[g+1]) and its
// points sit in slots [off, off+len) of the input buffer. Children are packed
// into the parent's slots: (A,C) from the front, (C,B) from the back; C's
// key is the first slot after the (A,C) points.
struct PolPass {
    static constexpr int NB = 2;
    // MIDDLE: groups are never empty, so rows holding whole groups take the
    // lane-parallel path
    static constexpr bool COUNTS = true, SCATTER = true, MULTI = false, MIDDLE = true;
    static constexpr int ROWS = kRows;
    // A, C, B as loaded; the edges A->C and C->B are rebuilt where used
    // (cheaper than keeping them live across the streaming loop)
    struct Ctx {
        float ax, ay, cx, cy, bx, by;
        int off, len, vstart;
        __device__ __forceinline__ Edge edge(int k) const
        {
            return k == 0 ? make_edge(ax, ay, cx, cy) : make_edge(cx, cy, bx, by);
        }
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
    int2* vlist;
    HullInfo* info;
    int fp64;
    int G;

    __device__ __forceinline__ int num_groups() const { return G; }
    __device__ __forceinline__ int group_of(int q, int lo, int hi) const { return search_le(vstart, q, lo, hi); }
    __device__ __forceinline__ int group_start(int g) const { return gld(vstart + g); }
    __device__ __forceinline__ int group_end(int g) const { return gld(vstart + g + 1); }
    __device__ __forceinline__ Ctx ctx(int g) const
    {
        const Seg s = gld(segs + g);
        Ctx c;
        c.ax = s.ax; c.ay = s.ay; c.cx = s.cx; c.cy = s.cy; c.bx = s.bx; c.by = s.by;
        c.off = s.off;
        c.len = s.len;
        c.vstart = gld(vstart + g);
        return c;
    }
    __device__ __forceinline__ void load(const Ctx& c, int, int q, float& x, float& y, int& id) const
    {
        const int p = c.off + (q - c.vstart);
        x = gld(Xi + p); y = gld(Yi + p); id = gld(Ii + p);
    }
    __device__ __forceinline__ int classify(const Ctx& c, int, int q, float x, float y, int id, Cand& k, Counters& ctr) const
    {
        const bool f64 = fp64 != 0;
        ctr.orient += 2;
        const Orient32 o1 = orient32p(c.ax, c.ay, c.cx, c.cy, x, y);  // A -> C
        const Orient32 o2 = orient32p(c.cx, c.cy, c.bx, c.by, x, y);  // C -> B
        int s1 = fast_sign(o1, f64), s2 = fast_sign(o2, f64);
        settle_p(s1, s1 == 0, c.ax, c.ay, c.cx, c.cy, x, y, ctr.orient_exact);
        settle_p(s2, s1 >= 0 && s2 == 0, c.cx, c.cy, c.bx, c.by, x, y, ctr.orient_exact);
        const bool in1 = s1 < 0, in2 = !in1 && s2 < 0;
        k = make_cand(in1 ? o1 : o2, x, y, id);
        return in1 ? 0 : (in2 ? 1 : kNone);
    }
    __device__ __forceinline__ int beats_fast(const Ctx&, int, const Cand& P, const Cand& Q) const
    {
        return sqh::beats_fast(P, Q, fp64 != 0);
    }
    __device__ __forceinline__ bool beats(const Ctx& c, int k, const Cand& P, const Cand& Q, Counters& ctr) const
    {
        return sqh::beats(c.edge(k), P, Q, fp64 != 0, ctr.cmp_exact);
    }
    __device__ __forceinline__ int place(const Ctx& c, int, int k, int rank) const
    {
        return k == 0 ? c.off + rank : c.off + c.len - 1 - rank;
    }
    __device__ __forceinline__ void store(int dst, float x, float y, int id) const
    {
        gst(Xo + dst, x); gst(Yo + dst, y); gst(Io + dst, id);
    }
    __device__ __forceinline__ void child(int slot, const Edge& E, const Cand& C, int off, int len) const
    {
        Seg r;
        r.ax = E.ox; r.ay = E.oy; r.bx = E.ex; r.by = E.ey;
        r.cx = C.x; r.cy = C.y;
        r.off = off; r.len = len;
        gst(recs + slot, r);
        gst(rec_cid + slot, C.id);
    }
    __device__ __forceinline__ void finalize(const Ctx& c, int g, const Agg<NB>& a) const
    {
        record_vertex(bitmap, vidx, vlist, info, c.off + a.cnt[0], gld(seg_cid + g));
        child(2 * g + 0, c.edge(0), a.best[0], c.off, a.cnt[0]);
        child(2 * g + 1, c.edge(1), a.best[1], c.off + c.len - a.cnt[1], a.cnt[1]);
    }
};

// ================================================== persistent hull kernel ==
//
// One cooperative launch computes all hulls of a call: seed, first split,
// first compaction, the segmented passes until no segment has points, and
// the ordered emission. One 1024-thread workgroup runs per compute unit;
// workgroups meet at grid barriers between steps. Loop bounds are read by
// every workgroup after a barrier, so all of them take the same path. Once
// few points are left, workgroup 0 finishes the remaining passes alone
// (no grid barriers).

// Grid barrier. Arrival counters are split over kBarSub sub-counters to cut
// same-address atomic serialisation; each workgroup issues one release fence
// before arriving and one acquire fence after leaving, and spins with
// relaxed loads. The last arriver of a sub-counter acquires (so later
// arrivals carry the earlier ones' writes) before arriving at the top
// counter with a release (which also orders its reset of the sub-counter
// before the next generation); the last top arriver publishes the new
// generation with a release store. Bounded spin: on timeout the error flag is raised and the
// workgroup continues.
constexpr int kBarSub = 16;
struct GridBar {
    unsigned int gen;
    unsigned int top;
    unsigned int pad[14];
    unsigned int sub[kBarSub][16];  // one 64-byte line per sub-counter
    unsigned int emit_mode;         // broadcast from workgroup 0 (see k_hull)
    unsigned int pad2[15];
};

__device__ __forceinline__ void spin_gen(GridBar* bar, unsigned int g, int* err)
{
    int spins = 0;
    while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins > kSpinLimit) {
            atomicOr(err, kErrSpin);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

__device__ __forceinline__ void grid_sync(GridBar* bar, int* err)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int nb = gridDim.x, i = blockIdx.x % kBarSub;
        const unsigned int nsub = (nb - i + kBarSub - 1) / kBarSub;
        const unsigned int ntop = nb < (unsigned)kBarSub ? nb : (unsigned)kBarSub;
        const unsigned int g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned int a = __hip_atomic_fetch_add(&bar->sub[i][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == nsub - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(&bar->sub[i][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // release: the reset happens before the last top arriver's
            // acquire, hence before the new generation and the next arrivals
            const unsigned int t = __hip_atomic_fetch_add(&bar->top, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ntop - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&bar->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                spin_gen(bar, g, err);
            }
        } else {
            spin_gen(bar, g, err);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__device__ __forceinline__ int ld_flag(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Pair {
    int a, b;
};

// Block-wide exclusive scan of one pair per thread; *tot receives the block
// total. `red` holds kWaves pairs.
__device__ __forceinline__ Pair block_excl_scan(Pair v, Pair* red, Pair* tot)
{
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const Pair inc = {wave_incl_sum(v.a), wave_incl_sum(v.b)};
    __syncthreads();
    if (lane == 63) red[w] = inc;
    __syncthreads();
    Pair off = {0, 0}, all = {0, 0};
#pragma unroll
    for (int u = 0; u < kWaves; ++u) {
        if (u < w) { off.a += red[u].a; off.b += red[u].b; }
        all.a += red[u].a; all.b += red[u].b;
    }
    *tot = all;
    return Pair{off.a + inc.a - v.a, off.b + inc.b - v.b};
}

constexpr int kMaxChunks = 256;  // workgroups of the persistent grid (upper bound: one per CU)
constexpr int kMaxInfoPasses = 256;
constexpr int kMaxPasses = 1 << 16;
constexpr int kMaxStamps = 1024;
constexpr int kTailPoints = 1 << 13;   // default: passes over at most this many points ...
constexpr int kTailSegs = 256;         // ... and segments run on one workgroup (no grid barriers)
constexpr int kSmallHull = 2048;       // single hulls up to this size are emitted by one workgroup

// info block written for the host
struct HullInfo {
    int h_total;
    int passes;
    int first_v;
    int vcount;
    int vcap;     // capacity of the vertex list
    int cur_out;  // engine: survivor buffer holding the segments left after the step
    int pass_traced;  // timing 3: the first grid pass has been traced
    int prefilter_n;  // points kept by the pre-filter (+ corners), -1 if it did not run
    int keep_n;       // pre-filter: kept points appended so far
    int sort_n;       // sorted-chain variant: points sorted (-1: no sort)
    int sort_bad;     // sorted-chain variant: neighbours out of order after the sort
    int stream_done;  // streaming path: the hull is complete before the passes kernel
    int spass_n;      // streaming path: passes run by k_spass
    int stream_line;  // streaming path: the static line filter was used
    int pass_s[kMaxInfoPasses];
    int pass_v[kMaxInfoPasses];
    int nstamps;
    int stamp_tag[kMaxStamps];
    unsigned long long stamp[kMaxStamps];
    unsigned long long trace[kMaxChunks][8];  // per-workgroup timestamps (timing == 2)
};

struct HullArgs {
    const float2* xy;
    int N, G;
    const int64_t* set_off;  // device, G + 1 (null: one set [0, N))
    int32_t* out;
    int64_t cap;
    int64_t* out_off;        // device, G + 1 (null for a single hull)
    float* X[2];
    float* Y[2];
    int* I[2];
    int* gstart;
    SetInfo* sets;
    Seg* recs;
    int* rec_cid;
    Seg* segs[2];
    int* seg_cid[2];
    int* vstart[2];
    int* sv;                 // {S0, V0, S1, V1}
    uint64_t* bitmap;
    int* vidx;
    int2* vlist;             // (key, id) of recorded vertices, first kVListCap
    int* wprefix;
    int W;
    void* slots;             // ChunkSlot<4>[gridDim.x]
    Pair* ctab;              // per-workgroup pairs (emission)
    GridBar* bar;
    int* err;
    uint32_t* stats;
    HullInfo* info;
    int fp64;
    int timing;
    int vcap;
    int tail_points;         // passes over at most this many points run on workgroup 0 alone
    // serving engine (k_engine_step); k_hull uses sbase = gstart, cur0 = 0
    const int* sbase;        // G: first slot of each new set (read positions start at gstart)
    int cur0;                // survivor buffer (0/1) holding the resident segments
    int max_passes;          // passes in this step
    int nres;                // resident sets, sorted by first slot
    const int* res_base;     // nres: first slot
    const int* res_n;        // nres: points
    int* res_alive;          // nres: set if the set still has a segment after the step
    int* res_h;              // nres: hull size of a set finished in this step
    int* hout;               // slot-indexed hull output of finished sets
    int* bad;                // G: new set had a non-finite coordinate
    // pre-filter (single hulls): 0 none, 1 quadrilateral, 2 octagon
    int prefilter;
    uint64_t* ext;           // extreme keys: 8 per workgroup
    float2* xy2;             // the kept subset: points ...
    int* ids2;               // ... and their input indices
    int* gs2;                // {0, subset size}
    // sorted-chain variant (single hulls; the host launches k_sort between
    // the first phases and the passes)
    int sorted;
    int* shist;              // kSortBuckets x workgroups
    int* stot;               // kSortBuckets
    // streaming path of one large set (k_sseed, k_ssplit, k_sfirst): partial
    // results and tile count words
    void* sws;
    unsigned int* sdone;     // the streaming kernels' completion counters (cleared by k_reset)
    const int* start;        // null, or {survivor buffer, pass} where k_hull<kHullPasses> starts
    int stream;              // 1: the streaming kernels run the first phases, k_hull<kHullPasses> the rest
    int spasses;             // streaming path: k_spass launches in this call
    int line_ok;             // streaming path: the static line filter may be used
};


__device__ __forceinline__ void stamp(const HullArgs& a, int tag)
{
    if (a.timing && blockIdx.x == 0 && threadIdx.x == 0) {
        const int k = a.info->nstamps;
        if (k < kMaxStamps) {
            a.info->stamp[k] = wall_clock64();
            a.info->stamp_tag[k] = tag;
            a.info->nstamps = k + 1;
        }
    }
}

// Per-workgroup timestamps: timing 2 traces the seed (slots 0-3) and the
// first split (4-7); timing 3 the first compaction (0-3) and the first pass
// (4-7): start of A, end of A, after the barrier, end of B(C).
__device__ __forceinline__ void trace(const HullArgs& a, int mode, int slot)
{
    if (a.timing == mode && threadIdx.x == 0 && blockIdx.x < kMaxChunks)
        a.info->trace[blockIdx.x][slot] = wall_clock64();
}

__device__ __forceinline__ int chunk_len(int P, int nb)
{
    int ch = (P + nb - 1) / nb;
    ch = (ch + 63) & ~63;
    return ch < 64 ? 64 : ch;
}

// Chunk summaries for step BC: for chunk b, the count prefix of its first
// group from the chunks before it, and the running position in the next
// segment table (active child segments and their points finalised by chunks
// < b, and by chunk b itself). One thread per chunk, a segmented
// Hillis-Steele scan in LDS over the running group's counts.
template <int NB>
struct ScanOut {
    int prefix[NB];
    Pair tab_before;
    Pair tab_self;
};

template <int NB>
struct ScanLds {
    int cont[kMaxChunks];        // chunk continues the running group of chunk - 1
    int run[2][kMaxChunks][NB];  // running counts (double-buffered scan)
    int tab_a[kMaxChunks], tab_b[kMaxChunks];
};

// LDS of slot_scan, shared by all phases
__shared__ int g_summ[sizeof(ScanLds<4>) / sizeof(int)];

template <class Pol>
__device__ __forceinline__ void slot_scan(const ChunkSlot<Pol::NB>* slots, int b, int nonempty, ScanLds<Pol::NB>& L,
                                          ScanOut<Pol::NB>& o, Pair* red)
{
    constexpr int NB = Pol::NB;
    const int n = min(b + 1, nonempty);  // chunks 0..n-1
    const int t = (int)threadIdx.x;
    int first_cnt[NB];
    bool before = false, done = false, head = true;
    if (t < n) {
        const int lg = gld(&slots[t].last_g), fg = gld(&slots[t].first_g);
        before = gld(&slots[t].first_before) != 0;
        done = gld(&slots[t].first_done) != 0;
        const int prev_lg = t > 0 ? gld(&slots[t - 1].last_g) : -1;
        // chunk t lies inside the group running out of chunk t-1
        head = !(before && !done && lg == fg && fg == prev_lg);
        L.cont[t] = head ? 0 : 1;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            L.run[0][t][k] = gld(&slots[t].last.cnt[k]);
            first_cnt[k] = gld(&slots[t].first.cnt[k]);
        }
        L.tab_a[t] = gld(&slots[t].tab_a);
        L.tab_b[t] = gld(&slots[t].tab_b);
    }
    __syncthreads();
    // segmented inclusive scan: run[t] = counts of the group running out of
    // chunk t, accumulated since the chunk where it started
    int src = 0;
    int hd = (t < n) ? (head ? 1 : 0) : 1;  // a segment head lies within the window ending at t
    for (int d = 1; d < n; d <<= 1) {
        int v[NB];
        int nh = hd;
        if (t < n) {
#pragma unroll
            for (int k = 0; k < NB; ++k) v[k] = L.run[src][t][k];
            if (!hd && t >= d) {
#pragma unroll
                for (int k = 0; k < NB; ++k) v[k] += L.run[src][t - d][k];
                nh = L.cont[t - d] ? 0 : 1;
            }
        }
        __syncthreads();
        if (t < n) {
#pragma unroll
            for (int k = 0; k < NB; ++k) L.run[src ^ 1][t][k] = v[k];
            L.cont[t] = nh ? 0 : 1;
        }
        __syncthreads();
        hd = nh;
        src ^= 1;
    }
    // per chunk: table contribution, including the group that runs into it and ends inside
    Pair tab = {0, 0};
    int pre[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) pre[k] = 0;
    if (t < n) {
        tab.a = L.tab_a[t];
        tab.b = L.tab_b[t];
        if (t > 0 && before) {
            const int fg = gld(&slots[t].first_g);
            if (fg == gld(&slots[t - 1].last_g)) {
#pragma unroll
                for (int k = 0; k < NB; ++k) pre[k] = L.run[src][t - 1][k];
            }
        }
        if (done) {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const int tot = pre[k] + first_cnt[k];
                if (tot > 0) { tab.a += 1; tab.b += tot; }
            }
        }
    }
    if (t == b) {
#pragma unroll
        for (int k = 0; k < NB; ++k) o.prefix[k] = pre[k];
        o.tab_self = tab;
    }
    Pair total;
    const Pair ex = block_excl_scan(tab, red, &total);
    if (t == b || (t == n - 1 && b >= n)) {
        o.tab_before = ex;
        if (b >= n) o.tab_self = tab;
    }
    __syncthreads();
}

// Step A of a phase over [0, P) split into nb chunks; publishes slot b.
// mul > 0: child records recs[mul*g + k] of groups finalised here are counted.
template <class Pol>
__device__ __forceinline__ void phase_step_a(const HullArgs& a, const Pol& pol, int P, int nb, int b, int mul,
                                             ChunkShared<Pol>& sh, Pair* red, Counters& ctr, int& glo, int& ghi)
{
    auto* slots = reinterpret_cast<ChunkSlot<Pol::NB>*>(a.slots);
    const int CH = chunk_len(P, nb);
    const int cb = (int)min((long long)b * CH, (long long)P), ce = min(cb + CH, P);
    const int G = pol.num_groups();
    glo = 0;
    ghi = -1;
    if (threadIdx.x == 0) {
        sh.carry_g = -1;
        agg_clear(sh.carry);
        sh.first_done = 0;
    }
    __syncthreads();
    if (cb >= ce) return;
    glo = pol.group_of(cb, 0, G - 1);
    ghi = pol.group_of(ce - 1, glo, G - 1);
    process_chunk<Pol, kModeAgg>(pol, cb, ce, glo, ghi, sh, ctr);
    Pair tab = {0, 0};
    if (mul > 0) {
        // groups that start and end inside the chunk were finalised in this step
        const int ga = pol.group_start(glo) >= cb ? glo : glo + 1;
        const int gb = pol.group_end(ghi) <= ce ? ghi : ghi - 1;
        Pair mine = {0, 0};
        for (int i = mul * ga + (int)threadIdx.x; i < mul * (gb + 1); i += kBlock) {
            const int len = gld(&a.recs[i].len);
            if (len > 0) { mine.a += 1; mine.b += len; }
        }
        block_excl_scan(mine, red, &tab);
    }
    if (threadIdx.x == 0) {
        ChunkSlot<Pol::NB> s;
        s.last_g = sh.carry_g;
        s.first_g = glo;
        s.first_before = pol.group_start(glo) < cb;
        s.first_done = sh.first_done;
        s.tab_a = tab.a;
        s.tab_b = tab.b;
        s.last = sh.carry;
        s.first = sh.first_total;
        s.pad[0] = s.pad[1] = 0;
        gst(slots + b, s);
    }
}

// Step B of a reduction phase: finalise the chunk's first group if it ends
// here (prefix from the chunks before).
template <class Pol>
__device__ __forceinline__ void phase_step_b(const HullArgs& a, const Pol& pol, int P, int nb, int b,
                                             ChunkShared<Pol>& sh, Counters& ctr)
{
    auto* slots = reinterpret_cast<ChunkSlot<Pol::NB>*>(a.slots);
    const int CH = chunk_len(P, nb);
    const int cb = (int)min((long long)b * CH, (long long)P), ce = min(cb + CH, P);
    if (cb >= ce) return;
    chunk_first_group(pol, b, cb, CH, slots, nullptr, sh, ctr);
}

// Steps B and C of a compaction phase: finalise the chunk's first group if
// it ends here, compact the child records of the groups finalised by this
// chunk into the next segment table, then write the chunk's points to their
// child segments.
// The new table is written after tb.a entries holding tb.b positions
// (segments already in the table stay in place).
template <class Pol>
__device__ __forceinline__ void phase_step_bc(const HullArgs& a, const Pol& pol, int P, int nb, int b, int mul,
                                              int glo, int ghi, Seg* segs, int* seg_cid, int* vstart, int* sv,
                                              Pair tb, ChunkShared<Pol>& sh, Pair* red, Counters& ctr)
{
    auto* slots = reinterpret_cast<ChunkSlot<Pol::NB>*>(a.slots);
    const int CH = chunk_len(P, nb);
    const int cb = (int)min((long long)b * CH, (long long)P), ce = min(cb + CH, P);
    const int nonempty = (P + CH - 1) / CH;
    __shared__ ScanOut<Pol::NB> so;
    slot_scan<Pol>(slots, b, nonempty, *reinterpret_cast<ScanLds<Pol::NB>*>(g_summ), so, red);
    Pair at = {tb.a + so.tab_before.a, tb.b + so.tab_before.b};
    if (b >= nonempty) {
        // empty chunk: only the last workgroup has a job, the table totals
        if (b == nb - 1 && threadIdx.x == 0) {
            const Pair tot = {at.a + so.tab_self.a, at.b + so.tab_self.b};
            sv[0] = tot.a;
            sv[1] = tot.b;
            vstart[tot.a] = tot.b;
        }
        return;
    }
    chunk_first_group(pol, b, cb, CH, slots, so.prefix, sh, ctr);
    // records of the groups finalised by this chunk
    const int ga = (pol.group_start(glo) >= cb || sh.first_done) ? glo : glo + 1;
    const int gb = pol.group_end(ghi) <= ce ? ghi : ghi - 1;
    for (int i0 = mul * ga; i0 < mul * (gb + 1); i0 += kBlock) {
        const int i = i0 + (int)threadIdx.x;
        Seg r;
        r.len = 0;
        if (i < mul * (gb + 1)) r = gld(a.recs + i);
        const Pair v = {r.len > 0 ? 1 : 0, r.len > 0 ? r.len : 0};
        Pair tot;
        const Pair ex = block_excl_scan(v, red, &tot);
        if (r.len > 0) {
            const int pos = at.a + ex.a;
            gst(segs + pos, r);
            gst(seg_cid + pos, gld(a.rec_cid + i));
            gst(vstart + pos, at.b + ex.b);
        }
        at.a += tot.a;
        at.b += tot.b;
        __syncthreads();
    }
    if (b == nb - 1 && threadIdx.x == 0) {
        sv[0] = at.a;
        sv[1] = at.b;
        vstart[at.a] = at.b;
    }
    process_chunk<Pol, kModeScatter>(pol, cb, ce, glo, ghi, sh, ctr);
}

// A reduction phase on the whole grid, or (SINGLE) on workgroup 0 alone,
// whose one chunk holds every group whole, so that step A finalises them all.
template <class Pol, bool SINGLE = false>
__device__ __forceinline__ void phase_reduce(const HullArgs& a, const Pol& pol, int P, ChunkShared<Pol>& sh,
                                             Pair* red, Counters& ctr)
{
    const int nb = SINGLE ? 1 : (int)gridDim.x, b = SINGLE ? 0 : (int)blockIdx.x;
    int glo, ghi;
    if (SINGLE) {
        phase_step_a(a, pol, P, nb, b, 0, sh, red, ctr, glo, ghi);
        __syncthreads();
        return;
    }
    const int t0 = Pol::COUNTS ? 4 : 0;
    trace(a, 2, t0 + 0);
    phase_step_a(a, pol, P, nb, b, 0, sh, red, ctr, glo, ghi);
    trace(a, 2, t0 + 1);
    grid_sync(a.bar, a.err);
    trace(a, 2, t0 + 2);
    phase_step_b(a, pol, P, nb, b, sh, ctr);
    trace(a, 2, t0 + 3);
    grid_sync(a.bar, a.err);
}

// A compaction phase: on the whole grid, or (SINGLE) on workgroup 0 alone.
template <class Pol, bool SINGLE>
__device__ __forceinline__ void phase_compact(const HullArgs& a, const Pol& pol, int P, int mul, Seg* segs,
                                              int* seg_cid, int* vstart, int* sv, Pair tb, ChunkShared<Pol>& sh,
                                              Pair* red, Counters& ctr)
{
    const int nb = SINGLE ? 1 : (int)gridDim.x, b = SINGLE ? 0 : (int)blockIdx.x;
    int glo, ghi;
    // trace: the first compaction in slots 0-3, the first grid pass in 4-7
    const int t0 = (Pol::NB == 4) ? 0 : 4;
    const bool tr = a.timing == 3 && !SINGLE && (Pol::NB == 4 || !a.info->pass_traced);
    if (tr) trace(a, 3, t0 + 0);
    phase_step_a(a, pol, P, nb, b, mul, sh, red, ctr, glo, ghi);
    if (tr) trace(a, 3, t0 + 1);
    if (SINGLE) __syncthreads();
    else grid_sync(a.bar, a.err);
    if (tr) trace(a, 3, t0 + 2);
    phase_step_bc(a, pol, P, nb, b, mul, glo, ghi, segs, seg_cid, vstart, sv, tb, sh, red, ctr);
    if (tr) trace(a, 3, t0 + 3);
    if (SINGLE) __syncthreads();
    else grid_sync(a.bar, a.err);
    if (tr && Pol::NB == 2 && b == 0 && threadIdx.x == 0 && a.timing == 3) a.info->pass_traced = 1;
}

template <class Pol, bool SINGLE>
__device__ __forceinline__ void run_pass(const HullArgs& a, int cur, int S, int V, ChunkShared<PolPass>& sh,
                                         Pair* red, Counters& ctr)
{
    const int nxt = cur ^ 1;
    // the vertex list only serves the one-workgroup emission of a single hull
    int2* vl = (a.vcap > 0 && a.G == 1) ? a.vlist : nullptr;
    PolPass pol{a.segs[cur], a.seg_cid[cur], a.vstart[cur], a.X[cur], a.Y[cur], a.I[cur], a.X[nxt], a.Y[nxt],
                a.I[nxt], a.recs, a.rec_cid, a.bitmap, a.vidx, vl, a.info, a.fp64, S};
    phase_compact<PolPass, SINGLE>(a, pol, V, 2, a.segs[nxt], a.seg_cid[nxt], a.vstart[nxt], a.sv + 2 * nxt,
                                   Pair{0, 0}, sh, red, ctr);
}

__device__ __forceinline__ void note_pass(const HullArgs& a, int pass, int S, int V)
{
    if (threadIdx.x == 0) {
        if (pass == 0) a.info->first_v = V;
        if (pass < kMaxInfoPasses) { a.info->pass_s[pass] = S; a.info->pass_v[pass] = V; }
        a.info->passes = pass;
    }
}

// ---- the last passes of a single hull or batch, in LDS ------------------
//
// Once at most kTinyPoints points in at most kTinySegs segments are left,
// workgroup 0 copies them into LDS and runs every remaining pass there, one
// point per thread: each point is classified against A->C and C->B of its
// segment (section 4.4.3); a segmented scan along the points (shuffles in a
// wave, then across waves) gives every point its rank in its child and the
// last point of a segment both children's counts and farthest points
// (section 4.4.1); a block scan places the children (section 4.4.4), and the
// points move to their child in the other LDS buffer. Slot ranges and vertex
// keys follow the pass in global memory exactly (child (A,C) keeps the front
// of the parent's slots, (C,B) the back, C's key is off + |(A,C)|), so the
// emission is unchanged. Points keep no slot order inside a child here: only
// the slot ranges matter for the keys.
constexpr int kTinyPoints = 1024;  // at most this many points: the rest runs in LDS (one per thread)

struct TinySeg {
    float ax, ay, bx, by, cx, cy;  // A, B and the farthest point C
    int off, len, cid, vs;         // slot range, C's index, first point in LDS
};

// Segments are single-buffered (S <= V <= kTinyPoints: every segment holds
// a point, and a pass keeps fewer points than it reads), points
// double-buffered.
struct TinyLds {
    float x[2][kTinyPoints], y[2][kTinyPoints];
    int id[2][kTinyPoints];
    TinySeg seg[kTinyPoints + 1];  // + the sentinel: seg[S].vs = V
    float bx[kTinyPoints][2], by[kTinyPoints][2];
    int bid[kTinyPoints][2], cnt[kTinyPoints][2], pbase[kTinyPoints][2];
};

__device__ __forceinline__ Cand tiny_wave_max(const Edge& E, Cand v, bool fp64, Counters& ctr)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Cand o = shfl_xor_cand(v, m);
        if (beats(E, o, v, fp64, ctr.cmp_exact)) v = o;
    }
    return v;
}

// Workgroup 0 only. Reads the pass state of buffer `cur` (S segments, V <=
// kTinyPoints points) and runs passes `pass`, pass + 1, ... until no
// segment is left.
__device__ __forceinline__ void tiny_passes(const HullArgs& a, int cur, int pass, TinyLds& L, Pair* red,
                                            Counters& ctr)
{
    const int t = (int)threadIdx.x, lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const bool f64 = a.fp64 != 0;
    int2* vl = (a.vcap > 0 && a.G == 1) ? a.vlist : nullptr;
    int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
    // load the segment table and the points
    for (int s = t; s < S; s += kBlock) {
        const Seg g = gld(a.segs[cur] + s);
        TinySeg& q = L.seg[s];
        q.ax = g.ax; q.ay = g.ay; q.bx = g.bx; q.by = g.by; q.cx = g.cx; q.cy = g.cy;
        q.off = g.off; q.len = g.len;
        q.cid = gld(a.seg_cid[cur] + s);
        q.vs = gld(a.vstart[cur] + s);
    }
    if (t == 0) L.seg[S].vs = V;
    __syncthreads();
    if (t < V) {
        int lo = 0, hi = S - 1;  // segment of position t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (L.seg[mid].vs <= t) lo = mid;
            else hi = mid - 1;
        }
        const int p = L.seg[lo].off + (t - L.seg[lo].vs);
        L.x[0][t] = gld(a.X[cur] + p);
        L.y[0][t] = gld(a.Y[cur] + p);
        L.id[0][t] = gld(a.I[cur] + p);
    }
    __syncthreads();
    int c = 0;
    for (;; ++pass) {
        note_pass(a, pass, S, V);
        if (S <= 0) break;
        // 1. point t: its segment, its child (A,C) = 0 / (C,B) = 1 / none
        const bool valid = t < V;
        int st = S;  // lanes without a point form their own segment
        if (valid) {
            int lo = 0, hi = S - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (L.seg[mid].vs <= t) lo = mid;
                else hi = mid - 1;
            }
            st = lo;
        }
        const int vs = valid ? L.seg[st].vs : t;
        Edge e0, e1;
        float px = 0.0f, py = 0.0f;
        int pid = 0;
        {
            const TinySeg& q = L.seg[valid ? st : 0];
            e0 = make_edge(q.ax, q.ay, q.cx, q.cy);
            e1 = make_edge(q.cx, q.cy, q.bx, q.by);
        }
        if (valid) { px = L.x[c][t]; py = L.y[c][t]; pid = L.id[c][t]; }
        ctr.orient += valid ? 2 : 0;
        const Orient32 o1 = orient32(e0, px, py);
        const Orient32 o2 = orient32(e1, px, py);
        int s1 = fast_sign(o1, f64), s2 = fast_sign(o2, f64);
        settle(s1, valid && s1 == 0, e0, px, py, ctr.orient_exact);
        settle(s2, valid && s1 >= 0 && s2 == 0, e1, px, py, ctr.orient_exact);
        const bool in0 = valid && s1 < 0, in1 = valid && !(s1 < 0) && s2 < 0;
        const int k = in0 ? 0 : (in1 ? 1 : -1);
        // 2. segmented inclusive scan of (count, farthest) per child along
        // the points: within the wave by shuffles, then across waves
        const Cand cand = make_cand(in0 ? o1 : o2, px, py, pid);
        int c0 = in0 ? 1 : 0, c1 = in1 ? 1 : 0;
        Cand b0 = in0 ? cand : no_cand(), b1 = in1 ? cand : no_cand();
        const int wstart = t - lane;
        bool flag = vs >= t;  // a segment starts here (or no point)
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int oc0 = __shfl_up(c0, d), oc1 = __shfl_up(c1, d);
            const Cand ob0 = shfl_up_cand(b0, d), ob1 = shfl_up_cand(b1, d);
            const int of = __shfl_up(flag ? 1 : 0, d);
            if (lane >= d && !flag) {
                c0 += oc0;
                c1 += oc1;
                if (beats(e0, ob0, b0, f64, ctr.cmp_exact)) b0 = ob0;
                if (beats(e1, ob1, b1, f64, ctr.cmp_exact)) b1 = ob1;
                flag = of != 0;
            }
        }
        // wave totals: lane 63 holds the aggregate of the segment running
        // out of the wave, since its start or the wave's start (flag false)
        __shared__ int wc[kWaves][2], wflag[kWaves], wseg[kWaves];
        __shared__ Cand wb[kWaves][2];
        if (lane == 63) {
            wc[w][0] = c0; wc[w][1] = c1;
            wb[w][0] = b0; wb[w][1] = b1;
            wflag[w] = flag ? 1 : 0;
            wseg[w] = st;
        }
        __syncthreads();
        if (w == 0 && lane < kWaves) {
            // R[v] = wflag[v] ? own[v] : R[v-1] (+) own[v] (the same segment)
            const int v = lane;
            int r0 = wc[v][0], r1 = wc[v][1];
            Cand q0 = wb[v][0], q1 = wb[v][1];
            bool f = wflag[v] != 0 || v == 0;
            const int sv = wseg[v];
            Edge f0 = e0, f1 = e1;
            if (sv < S) {
                const TinySeg& q = L.seg[sv];
                f0 = make_edge(q.ax, q.ay, q.cx, q.cy);
                f1 = make_edge(q.cx, q.cy, q.bx, q.by);
            }
            for (int d = 1; d < kWaves; d <<= 1) {
                const int o0 = __shfl_up(r0, d), o1 = __shfl_up(r1, d);
                const Cand p0 = shfl_up_cand(q0, d), p1 = shfl_up_cand(q1, d);
                const int of = __shfl_up(f ? 1 : 0, d);
                if (v >= d && !f) {
                    r0 += o0;
                    r1 += o1;
                    if (beats(f0, p0, q0, f64, ctr.cmp_exact)) q0 = p0;
                    if (beats(f1, p1, q1, f64, ctr.cmp_exact)) q1 = p1;
                    f = of != 0;
                }
            }
            wc[v][0] = r0; wc[v][1] = r1;
            wb[v][0] = q0; wb[v][1] = q1;
        }
        __syncthreads();
        if (w > 0 && valid && vs < wstart) {
            // the segment started in an earlier wave: add what came before
            c0 += wc[w - 1][0];
            c1 += wc[w - 1][1];
            if (beats(e0, wb[w - 1][0], b0, f64, ctr.cmp_exact)) b0 = wb[w - 1][0];
            if (beats(e1, wb[w - 1][1], b1, f64, ctr.cmp_exact)) b1 = wb[w - 1][1];
        }
        // the last point of a segment holds its totals
        if (valid && t == L.seg[st + 1].vs - 1) {
            L.cnt[st][0] = c0; L.cnt[st][1] = c1;
            L.bx[st][0] = b0.x; L.by[st][0] = b0.y; L.bid[st][0] = b0.id;
            L.bx[st][1] = b1.x; L.by[st][1] = b1.y; L.bid[st][1] = b1.id;
        }
        const int rank = k == 0 ? c0 - 1 : c1 - 1;  // earlier points of the same child
        __syncthreads();
        // 3. children of segment t: their points' base and their table index
        // (S <= kTinyPoints = kBlock: one thread per segment)
        TinySeg mine = {};
        int n0 = 0, n1 = 0;
        if (t < S) {
            mine = L.seg[t];
            n0 = L.cnt[t][0];
            n1 = L.cnt[t][1];
        }
        Pair tot;
        const Pair ex = block_excl_scan(Pair{n0 + n1, (n0 > 0) + (n1 > 0)}, red, &tot);
        if (t < S) {
            L.pbase[t][0] = ex.a;
            L.pbase[t][1] = ex.a + n0;
            // C is a vertex: its key is the first slot after the (A,C) points
            record_vertex(a.bitmap, a.vidx, vl, a.info, mine.off + n0, mine.cid);
        }
        __syncthreads();
        // 4. move every kept point to its child
        if (k >= 0) {
            const int dst = L.pbase[st][k] + rank;
            L.x[c ^ 1][dst] = px;
            L.y[c ^ 1][dst] = py;
            L.id[c ^ 1][dst] = pid;
        }
        __syncthreads();
        // 5. the child table replaces the parents: (A,C) keeps the front of
        // the parent's slots, (C,B) the back
        if (t < S) {
            int j = ex.b;
            if (n0 > 0) {
                TinySeg& q = L.seg[j++];
                q.ax = mine.ax; q.ay = mine.ay; q.bx = mine.cx; q.by = mine.cy;
                q.cx = L.bx[t][0]; q.cy = L.by[t][0]; q.cid = L.bid[t][0];
                q.off = mine.off; q.len = n0; q.vs = ex.a;
            }
            if (n1 > 0) {
                TinySeg& q = L.seg[j];
                q.ax = mine.cx; q.ay = mine.cy; q.bx = mine.bx; q.by = mine.by;
                q.cx = L.bx[t][1]; q.cy = L.by[t][1]; q.cid = L.bid[t][1];
                q.off = mine.off + mine.len - n1; q.len = n1; q.vs = ex.a + n0;
            }
        }
        if (t == 0) L.seg[tot.b].vs = tot.a;
        __syncthreads();
        stamp(a, 100 + pass);
        S = tot.b;
        V = tot.a;
        c ^= 1;
    }
    if (t == 0) {
        a.sv[2 * cur] = 0;
        a.sv[2 * cur + 1] = 0;
    }
}

// Ordered emission of a single hull with few vertices by one workgroup: the
// rank of a vertex is the number of vertices with a smaller key.
__device__ __forceinline__ void emit_small(const HullArgs& a, int h, int2* lds)
{
    for (int i = (int)threadIdx.x; i < h; i += kBlock) lds[i] = gld(a.vlist + i);
    __syncthreads();
    for (int i = (int)threadIdx.x; i < h; i += kBlock) {
        const int key = lds[i].x;
        int rank = 0;
        for (int j = 0; j < h; ++j) rank += lds[j].x < key;
        if (rank < a.cap) gst(a.out + rank, lds[i].y);
    }
    if (threadIdx.x == 0) {
        a.info->h_total = h;
        if (a.out_off) {  // a batched call on one set
            a.out_off[0] = 0;
            a.out_off[1] = h;
        }
    }
    __syncthreads();
}

// Ordered emission on the whole grid: vertex keys are the set bits of the
// bitmap; the rank of a key among all keys is its output position (keys
// increase along each set's ring and sets are stored in order).
// W: bitmap words holding the keys
__device__ __forceinline__ void emit_grid(const HullArgs& a, Pair* red, int W)
{
    const int nb = (int)gridDim.x, b = (int)blockIdx.x;
    const int gtid = b * kBlock + (int)threadIdx.x, gstride = nb * kBlock;
    const int CHw = (W + nb - 1) / nb;
    const int wb = min(b * CHw, W), we = min(wb + CHw, W);
    Pair mine = {0, 0};
    for (int i = wb + (int)threadIdx.x; i < we; i += kBlock) mine.a += __popcll(gld(a.bitmap + i));
    Pair tot;
    block_excl_scan(mine, red, &tot);
    if (threadIdx.x == 0) a.ctab[b] = tot;
    grid_sync(a.bar, a.err);
    Pair pre = {0, 0};
    for (int c = (int)threadIdx.x; c < b; c += kBlock) pre.a += gld(&a.ctab[c].a);
    Pair ptot;
    block_excl_scan(pre, red, &ptot);
    int at = ptot.a;
    __syncthreads();
    for (int i0 = wb; i0 < we; i0 += kBlock) {
        const int i = i0 + (int)threadIdx.x;
        const uint64_t word = i < we ? gld(a.bitmap + i) : 0ull;
        Pair t;
        const Pair ex = block_excl_scan(Pair{(int)__popcll(word), 0}, red, &t);
        if (i < we) {
            int rank = at + ex.a;
            gst(a.wprefix + i, rank);
            uint64_t bits = word;
            while (bits) {
                const int bit = __ffsll((unsigned long long)bits) - 1;
                bits &= bits - 1;
                if (rank < a.cap) gst(a.out + rank, gld(a.vidx + i * 64 + bit));
                ++rank;
            }
        }
        at += t.a;
        __syncthreads();
    }
    if (b == nb - 1 && threadIdx.x == 0) a.info->h_total = at;
    if (a.out_off) {
        grid_sync(a.bar, a.err);
        const int h = ld_flag(&a.info->h_total);
        for (int s = gtid; s <= a.G; s += gstride) {
            const int key = a.gstart[s];
            int64_t v;
            if (key >= a.N) v = h;
            else v = a.wprefix[key >> 6] + __popcll(a.bitmap[key >> 6] & mask_lt(key & 63));
            a.out_off[s] = v;
        }
    }
}

constexpr int kSmallInput = 1 << 15;  // single hulls up to this size run on one workgroup

// Seed, first split and first compaction (on the grid, or SINGLE on
// workgroup 0 alone). False if the input was rejected (non-finite).
template <bool SINGLE, bool IDS>
__device__ __forceinline__ bool first_phases(const HullArgs& a, const float2* in_xy, int* in_gstart,
                                             const int* in_ids, int in_n, ChunkShared<PolFirst>& sh, Pair* red,
                                             Counters& ctr)
{
    using Seed = PolSeedT<IDS>;
    using Split = PolSplitT<IDS>;
    using First = PolFirstT<IDS>;
    // ---- seed: lexmin / lexmax of every set
    {
        Seed pol{in_xy, in_gstart, a.sets, a.err, in_ids, nullptr, a.G};
        phase_reduce<Seed, SINGLE>(a, pol, in_n, *reinterpret_cast<ChunkShared<Seed>*>(&sh), red, ctr);
    }
    stamp(a, 1);
    // flags raised before the barrier decide the path; every workgroup sees them
    if (ld_flag(a.err) & (kErrNonFinite | kErrBounds)) return false;
    // ---- first split: side counts and farthest point of each side
    {
        Split pol{in_xy, in_gstart, in_gstart, nullptr, in_ids, a.sets, a.bitmap, a.vidx, a.vlist, a.info, a.fp64,
                  a.G};
        phase_reduce<Split, SINGLE>(a, pol, in_n, *reinterpret_cast<ChunkShared<Split>*>(&sh), red, ctr);
    }
    stamp(a, 2);
    // ---- first compaction into four child segments per set
    {
        First pol{in_xy,  in_gstart, in_gstart, nullptr, in_ids, a.sets,  a.X[0], a.Y[0], a.I[0],
                  a.recs, a.rec_cid, a.bitmap,  a.vidx,  a.vlist, a.info, a.fp64, a.G};
        phase_compact<First, SINGLE>(a, pol, in_n, 4, a.segs[0], a.seg_cid[0], a.vstart[0], a.sv, Pair{0, 0},
                                     *reinterpret_cast<ChunkShared<First>*>(&sh), red, ctr);
    }
    stamp(a, 3);
    return true;
}

// The remaining passes on workgroup 0 alone, the last ones in LDS.
__device__ __forceinline__ void tail_passes(const HullArgs& a, int cur, int pass, TinyLds& tiny,
                                            ChunkShared<PolPass>& shQ, Pair* red, Counters& ctr)
{
    for (int p = pass;; ++p) {
        const int S2 = ld_flag(a.sv + 2 * cur), V2 = ld_flag(a.sv + 2 * cur + 1);
        if (S2 > 0 && V2 <= kTinyPoints) {
            tiny_passes(a, cur, p, tiny, red, ctr);
            break;
        }
        note_pass(a, p, S2, V2);
        if (S2 <= 0) break;
        if (p >= kMaxPasses) {
            if (threadIdx.x == 0) atomicOr(a.err, kErrBounds);
            break;
        }
        run_pass<PolPass, true>(a, cur, S2, V2, shQ, red, ctr);
        stamp(a, 100 + p);
        cur ^= 1;
    }
}

// The persistent kernel's instances:
//   kHullPlain  the whole hull, no pre-filter (built without the subset's
//               index loads)
//   kHullPre    the whole hull after k_prefilter, on its subset if it ran
//   kHullFirst  the first phases only (seed, first split, first
//               compaction), after which k_sort orders the segments
//   kHullPasses the passes and the emission only, after k_sort
// The last three may follow k_prefilter.
constexpr int kHullPlain = 0, kHullPre = 1, kHullFirst = 2, kHullPasses = 3;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_hull(HullArgs a)
{
    constexpr bool PRE = MODE != kHullPlain;
    __shared__ ChunkShared<PolFirst> sh_first;
    __shared__ Pair red[kWaves];
    // the vertex list of the one-workgroup emission and the LDS of the last
    // passes are never live together
    __shared__ uint4 lds_tail[(sizeof(TinyLds) > sizeof(int2) * kSmallHull ? sizeof(TinyLds)
                                                                          : sizeof(int2) * kSmallHull) / 16 + 1];
    int2* vl = reinterpret_cast<int2*>(lds_tail);
    TinyLds* tiny = reinterpret_cast<TinyLds*>(lds_tail);
    auto& shF = sh_first;
    auto& shS = *reinterpret_cast<ChunkShared<PolSeed>*>(&sh_first);
    auto& shP = *reinterpret_cast<ChunkShared<PolSplit>*>(&sh_first);
    auto& shQ = *reinterpret_cast<ChunkShared<PolPass>*>(&sh_first);
    Counters ctr = {0u, 0u, 0u};
    const int b = (int)blockIdx.x;
    bool tail = false;

    // ---- a single hull after the pre-filter (k_prefilter) runs on the kept
    // subset, whose indices are mapped back at the emission (only these few
    // values are redirected: the arguments stay in the kernel's argument
    // segment)
    const int n2 = (PRE && a.prefilter && a.G == 1 && a.N > 0) ? ld_flag(&a.info->prefilter_n) : -1;
    const bool sub = n2 >= 0 && n2 <= a.N;  // (the subset never exceeds the input)
    const float2* in_xy = sub ? a.xy2 : a.xy;
    int* in_gstart = sub ? a.gs2 : a.gstart;
    const int* in_ids = sub ? a.ids2 : nullptr;  // the subset's points carry their input indices
    const int in_n = sub ? n2 : a.N;

    bool run_tail = false;  // this workgroup finishes the passes alone
    int cur = 0, pass = 0;

    stamp(a, 0);
    if (ld_flag(a.err) & kErrBounds) goto done;  // set offsets rejected by k_reset
    // A single hull of few points runs on workgroup 0 alone (no grid
    // barriers); the other workgroups wait for its emission decision.
    if (MODE == kHullPasses) {
        // the first phases ran in an earlier launch; a rejected input ended there
        if (ld_flag(a.err) & (kErrNonFinite | kErrBounds)) goto done;
        if (a.start) {
            // earlier launches also ran passes, or finished the hull
            if (ld_flag(&a.info->stream_done)) goto done;
            cur = ld_flag(a.start) & 1;
            pass = ld_flag(a.start + 1);
        }
        goto passes;
    }
    if (MODE != kHullFirst && a.G == 1 && in_n <= kSmallInput) {
        tail = true;
        if (b == 0) {
            if constexpr (PRE)
                run_tail = sub ? first_phases<true, true>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr)
                               : first_phases<true, false>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr);
            else
                run_tail = first_phases<true, false>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr);
            if (!run_tail) {
                if (threadIdx.x == 0) {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                    __hip_atomic_store(&a.bar->emit_mode, 3u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                goto done;  // rejected input: no emission
            }
        }
    } else {
        bool ok;
        if constexpr (PRE)
            ok = sub ? first_phases<false, true>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr)
                     : first_phases<false, false>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr);
        else
            ok = first_phases<false, false>(a, in_xy, in_gstart, in_ids, in_n, sh_first, red, ctr);
        if (!ok || MODE == kHullFirst) goto done;
    passes:
        // ---- segmented passes over all segments of all sets
        for (;; ++pass) {
            const int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
            if (b == 0) note_pass(a, pass, S, V);
            if (S <= 0) break;
            if (pass >= kMaxPasses) {  // pass limit: report and stop
                if (b == 0 && threadIdx.x == 0) atomicOr(a.err, kErrBounds);
                break;
            }
            if ((V <= a.tail_points && S <= kTailSegs) || V <= kTinyPoints) {
                // few points left: workgroup 0 finishes the passes alone
                tail = true;
                run_tail = b == 0;
                break;
            }
            run_pass<PolPass, false>(a, cur, S, V, shQ, red, ctr);
            stamp(a, 100 + pass);
            cur ^= 1;
        }
    }
    if (run_tail) tail_passes(a, cur, pass, *tiny, shQ, red, ctr);
    // ---- ordered emission
    {
        // workgroup 0 decides: one workgroup (single hull, few vertices) or the grid
        unsigned int mode;
        if (b == 0) {
            const int h = ld_flag(&a.info->vcount);
            mode = (a.G == 1 && h <= kSmallHull && h <= a.vcap) ? 1u : 2u;
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __hip_atomic_store(&a.bar->emit_mode, mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (mode == 1u) emit_small(a, h, vl);
        } else if (tail) {
            // wait for workgroup 0's decision (it is still running the last passes)
            __shared__ unsigned int smode;
            if (threadIdx.x == 0) {
                int spins = 0;
                unsigned int m;
                while ((m = __hip_atomic_load(&a.bar->emit_mode, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) == 0u) {
                    if (++spins > kSpinLimit) {
                        atomicOr(a.err, kErrSpin);
                        m = 1u;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                smode = m;
            }
            __syncthreads();
            mode = smode;
            if (mode == 3u) goto done;  // workgroup 0 rejected the input
        } else {
            // the pass loop ended on a grid barrier: every workgroup can decide
            const int h = ld_flag(&a.info->vcount);
            mode = (a.G == 1 && h <= kSmallHull && h <= a.vcap) ? 1u : 2u;
        }
        if (mode == 2u) emit_grid(a, red, sub ? (n2 + 63) / 64 : a.W);
    }
    stamp(a, 4);
done:
    flush_counters(a.stats, ctr);
}

// The pre-filter of a single hull (cooperative launch before k_hull, same
// workspace). Each workgroup streams one contiguous chunk twice: first for
// the eight extremes, whose keys go to ext (8 per workgroup) and, after a
// grid barrier, are reduced by every workgroup; then to append the points
// that the polygon does not certify inside to (xy2, ids2), in any order
// (the subset's points carry their input indices, so no tie rule depends on
// it). The kept points are staged in LDS and placed with one atomic add per
// flush; the stage is flushed whenever the next block of rows could
// overfill it. Leaves the subset's size in gs2[1] and info->prefilter_n (-1:
// not run; a non-finite coordinate is left to k_hull's seed, which reports
// it).
constexpr int kPreRows = 8;                         // rows of loads in flight per wave (extremes)
constexpr int kKeepRows = 4;                        // the same for the keep pass
constexpr int kKeepStage = 2 * kBlock * kKeepRows;  // staged points per workgroup

__device__ __forceinline__ float rfl_f(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__global__ __launch_bounds__(kBlock) void k_prefilter(HullArgs a)
{
    __shared__ uint64_t ext_w[kWaves][8];
    __shared__ float corner_xy[2][8];
    __shared__ KeepLds keep_lds;
    __shared__ float2 st_xy[kKeepStage];
    __shared__ int st_id[kKeepStage];
    __shared__ int st_n, st_base;
    Counters ctr = {0u, 0u, 0u};
    stamp(a, 0);
    const int nb = (int)gridDim.x, b = (int)blockIdx.x, lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const int P = a.N;
    const int CH = chunk_len(P, nb);
    const int cb = (int)min((long long)b * CH, (long long)P), ce = min(cb + CH, P);
    int wb, we;
    wave_part(cb, ce, w, wb, we);
    // every wave's part has at most this many blocks of kKeepRows rows
    const int iters = (((ce - cb + 63) / 64 + kWaves - 1) / kWaves + kKeepRows - 1) / kKeepRows;

    // ---- extremes of this wave's part, then of the workgroup's chunk
    {
        ExtLane L;
        L.init();
        bool bad = false;
        for (int q0 = wb; q0 < we; q0 += 64 * kPreRows) {
            float2 v[kPreRows];
#pragma unroll
            for (int r = 0; r < kPreRows; ++r) {
                const int q = q0 + 64 * r + lane;
                v[r] = q < we ? gld(a.xy + q) : make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int r = 0; r < kPreRows; ++r) {
                const int q = q0 + 64 * r + lane;
                if (q < we) {
                    bad = bad || !(isfinite(v[r].x) && isfinite(v[r].y));
                    L.add(v[r].x, v[r].y, q);
                }
            }
        }
        if (__ballot(bad) && lane == 0) atomicOr(a.err, kErrNonFinite);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint64_t v = ext_key(k, L.v[k], L.id[k]);
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v = ext_pick(k, v, shfl_xor_u64(v, m));
            if (lane == 0) ext_w[w][k] = v;
        }
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint64_t v = lane < kWaves ? ext_w[lane][k] : ext_none(k);
#pragma unroll
            for (int m = kWaves / 2; m >= 1; m >>= 1) v = ext_pick(k, v, shfl_xor_u64(v, m));
            if (lane == 0) gst(a.ext + 8 * b + k, v);
        }
    }
    grid_sync(a.bar, a.err);
    if (ld_flag(a.err) & (kErrNonFinite | kErrBounds)) goto done;  // (the same for every workgroup)

    // ---- the corners: every workgroup reduces the keys of all workgroups
    if (w < 4) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            uint64_t v = ext_none(k);
            for (int t = (int)threadIdx.x; t < nb; t += 256) v = ext_pick(k, v, gld(a.ext + 8 * t + k));
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) v = ext_pick(k, v, shfl_xor_u64(v, m));
            if (lane == 0) ext_w[w][k] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = (int)threadIdx.x;
        uint64_t v = ext_w[0][k];
#pragma unroll
        for (int t = 1; t < 4; ++t) v = ext_pick(k, v, ext_w[t][k]);
        const float2 c = gld(a.xy + ext_index(k, v));  // N > 0: every direction has a point
        corner_xy[0][k] = c.x;
        corner_xy[1][k] = c.y;
    }
    if (threadIdx.x == 0) st_n = 0;
    __syncthreads();
    {
        float cx[8], cy[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            cx[k] = rfl_f(corner_xy[0][k]);
            cy[k] = rfl_f(corner_xy[1][k]);
        }
        KeepEdges E;
        keep_build(E, keep_lds, cx, cy, a.prefilter == 1);
        __syncthreads();  // keep_lds

        // ---- the points not certified inside, staged per workgroup
        for (int it = 0; it < iters; ++it) {
            const int q0 = wb + it * 64 * kKeepRows;
            float2 v[kKeepRows];
#pragma unroll
            for (int r = 0; r < kKeepRows; ++r) {
                const int q = q0 + 64 * r + lane;
                v[r] = q < we ? gld(a.xy + q) : make_float2(0.0f, 0.0f);
            }
#pragma unroll
            for (int r = 0; r < kKeepRows; ++r) {
                const int q = q0 + 64 * r + lane;
                const bool kp = q < we && keep_point(E, keep_lds, v[r].x, v[r].y, ctr);
                const uint64_t M = __ballot(kp);
                if (M) {
                    int off = 0;
                    if (lane == 0) off = atomicAdd(&st_n, (int)__popcll(M));
                    off = __shfl(off, 0);
                    if (kp) {
                        const int rr = off + __popcll(M & mask_lt(lane));
                        st_xy[rr] = v[r];
                        st_id[rr] = q;
                    }
                }
            }
            __syncthreads();
            const int n = st_n;
            __syncthreads();  // every wave has read n before the next appends
            // flush when the next block of rows (at most kBlock * kKeepRows
            // points) might not fit, and at the end
            if (n > kKeepStage - kBlock * kKeepRows || (it == iters - 1 && n > 0)) {
                if (threadIdx.x == 0) st_base = atomicAdd(&a.info->keep_n, n);
                __syncthreads();
                const int base = st_base;
                for (int i = (int)threadIdx.x; i < n; i += kBlock) {
                    gst(a.xy2 + base + i, st_xy[i]);
                    gst(a.ids2 + base + i, st_id[i]);
                }
                __syncthreads();
                if (threadIdx.x == 0) st_n = 0;
                __syncthreads();
            }
        }
    }
    grid_sync(a.bar, a.err);
    if (b == 0 && threadIdx.x == 0) {
        const int total = ld_flag(&a.info->keep_n);
        a.gs2[0] = 0;
        a.gs2[1] = total;
        a.info->prefilter_n = total;
    }
done:
    stamp(a, 5);
    flush_counters(a.stats, ctr);
}

// ---- the sorted-chain variant ------------------------------------------
//
// The paper sorts the points below and above the first split line by x
// (sections 3 and 4.3) and afterwards only removes points: a segment is a
// run of consecutive points between two hull vertices (section 4.4). Here
// the first compaction's segments (at most four for one set) are sorted by
// x after the first phases: ascending where the segment runs left to right
// (A.x <= B.x, the lower chain), descending where it runs right to left.
// Every later pass partitions each segment stably into its two children,
// and on an x-sorted segment the points outside (A, C) all precede C and
// those outside (C, B) all follow it, so the children come out in order and
// the pass only removes points; the hull is the same.
//
// k_sort (cooperative): an LSD radix sort of 8-bit digits over the
// order-preserving image of x (complemented on right-to-left segments),
// stable in every pass; every pass also takes the segment index as its top
// two bits, so that no point leaves its segment's range. Each pass:
// per-wave bucket counts in LDS -> per-workgroup counts (with per-wave
// prefixes kept in LDS) -> grid barrier -> exclusive scan of each bucket
// over the workgroups -> grid barrier -> bucket bases -> a stable scatter
// in which the lanes of one row take their ranks from ballots over the
// bucket bits. Four passes take the points from buffer 0 through buffer 1
// and back. Afterwards neighbours in a segment are checked (info->sort_bad
// counts pairs out of order; 0 expected).
constexpr int kSortSegs = 4;        // segments after the first compaction of one set
constexpr int kSortBuckets = 1024;  // 2 segment bits + 8 digit bits
constexpr int kSortRows = 4;        // rows of loads in flight per wave

// the segment of position q: vs[k] is segment k's first position (vs[S..4] = V)
__device__ __forceinline__ int sort_seg(int q, const int (&vs)[kSortSegs + 1])
{
    return (q >= vs[1] ? 1 : 0) + (q >= vs[2] ? 1 : 0) + (q >= vs[3] ? 1 : 0);
}

// The points of segment k occupy its slots off[k] .. off[k] + len - 1 (the
// slot ranges leave gaps for vertices); positions number them densely. The
// sort runs over positions and reads and writes the matching slots.
__device__ __forceinline__ int sort_slot(int q, int sg, const int (&vs)[kSortSegs + 1], const int (&off)[kSortSegs])
{
    return off[sg] + (q - vs[sg]);
}

__device__ __forceinline__ uint32_t sort_key(float x, int s, uint32_t desc)
{
    const uint32_t o = ord32(x + 0.0f);  // -0 -> +0
    return ((desc >> s) & 1u) ? ~o : o;
}

// lanes of this wave whose bucket equals this lane's (among valid lanes)
__device__ __forceinline__ uint64_t sort_match(int bucket, bool valid, int nbits)
{
    uint64_t m = __ballot(valid);
    for (int i = 0; i < nbits; ++i) {
        const bool bit = (bucket >> i) & 1;
        const uint64_t bb = __ballot(bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(kBlock) void k_sort(HullArgs a)
{
    __shared__ int wtab[kWaves][kSortBuckets];  // per-wave counts, then write offsets
    __shared__ Pair red[kWaves];
    __shared__ int sbad;
    Counters ctr = {0u, 0u, 0u};
    const int nb = (int)gridDim.x, b = (int)blockIdx.x, lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const int t = (int)threadIdx.x;
    stamp(a, 0);
    int S = 0, V = 0;
    if (!(ld_flag(a.err) & (kErrNonFinite | kErrBounds))) {
        S = ld_flag(a.sv);
        V = ld_flag(a.sv + 1);
    }
    if (S > 0 && S <= kSortSegs && V > 0) {
        int vs[kSortSegs + 1], off[kSortSegs];
        uint32_t desc = 0;
#pragma unroll
        for (int k = 0; k <= kSortSegs; ++k) vs[k] = k <= S ? gld(a.vstart[0] + k) : V;
#pragma unroll
        for (int k = 0; k < kSortSegs; ++k) {
            off[k] = 0;
            if (k < S) {
                const Seg g = gld(a.segs[0] + k);
                desc |= (g.ax > g.bx ? 1u : 0u) << k;
                off[k] = g.off;
            }
        }
        const int CH = chunk_len(V, nb);
        const int cb = (int)min((long long)b * CH, (long long)V), ce = min(cb + CH, V);
        int wb, we;
        wave_part(cb, ce, w, wb, we);
        for (int ps = 0; ps < 4; ++ps) {
            const int src = ps & 1, dst = src ^ 1;
            const int shift = 8 * ps;
            constexpr int nbits = 10, nbk = kSortBuckets;
            // 1. per-wave counts of this wave's part
            for (int i = t; i < kWaves * nbk; i += kBlock) wtab[i / nbk][i % nbk] = 0;
            __syncthreads();
            for (int q0 = wb; q0 < we; q0 += 64 * kSortRows) {
                float xr[kSortRows];
#pragma unroll
                for (int r = 0; r < kSortRows; ++r) {  // loads first
                    const int q = q0 + 64 * r + lane;
                    xr[r] = q < we ? gld(a.X[src] + sort_slot(q, sort_seg(q, vs), vs, off)) : 0.0f;
                }
#pragma unroll
                for (int r = 0; r < kSortRows; ++r) {
                    const int q = q0 + 64 * r + lane;
                    const bool valid = q < we;
                    int bucket = 0;
                    if (valid) {
                        const int sg = sort_seg(q, vs);
                        bucket = (int)((sort_key(xr[r], sg, desc) >> shift) & 255u) | (sg << 8);
                    }
                    const uint64_t m = sort_match(bucket, valid, nbits);
                    if (valid && (m >> lane) == 1ull) wtab[w][bucket] += __popcll(m);  // the group's last lane
                }
            }
            __syncthreads();
            // 2. per bucket: prefixes over the waves (kept), the workgroup's count
            for (int j = t; j < nbk; j += kBlock) {
                int run = 0;
#pragma unroll
                for (int v = 0; v < kWaves; ++v) {
                    const int c = wtab[v][j];
                    wtab[v][j] = run;
                    run += c;
                }
                gst(a.shist + j * nb + b, run);
            }
            grid_sync(a.bar, a.err);
            // 3. per bucket: exclusive scan over the workgroups, and the total
            for (int j = b; j < nbk; j += nb) {
                const int c = t < nb ? gld(a.shist + j * nb + t) : 0;
                Pair tot;
                const Pair ex = block_excl_scan(Pair{c, 0}, red, &tot);
                if (t < nb) gst(a.shist + j * nb + t, ex.a);
                if (t == 0) gst(a.stot + j, tot.a);
                __syncthreads();
            }
            grid_sync(a.bar, a.err);
            // 4. bucket bases (every workgroup), then this wave's write offsets
            {
                const int c = t < nbk ? gld(a.stot + t) : 0;
                Pair tot;
                const Pair ex = block_excl_scan(Pair{c, 0}, red, &tot);
                const int mine = t < nbk ? ex.a + gld(a.shist + t * nb + b) : 0;
                __syncthreads();
                if (t < nbk) {
#pragma unroll
                    for (int v = 0; v < kWaves; ++v) wtab[v][t] += mine;
                }
                __syncthreads();
            }
            // 5. stable scatter, row by row
            for (int q0 = wb; q0 < we; q0 += 64 * kSortRows) {
                float xr[kSortRows], yr[kSortRows];
                int ir[kSortRows];
#pragma unroll
                for (int r = 0; r < kSortRows; ++r) {  // loads first
                    const int q = q0 + 64 * r + lane;
                    xr[r] = yr[r] = 0.0f;
                    ir[r] = 0;
                    if (q < we) {
                        const int sl = sort_slot(q, sort_seg(q, vs), vs, off);
                        xr[r] = gld(a.X[src] + sl);
                        yr[r] = gld(a.Y[src] + sl);
                        ir[r] = gld(a.I[src] + sl);
                    }
                }
#pragma unroll
                for (int r = 0; r < kSortRows; ++r) {
                    const int q = q0 + 64 * r + lane;
                    const bool valid = q < we;
                    int bucket = 0;
                    if (valid) {
                        const int sg = sort_seg(q, vs);
                        bucket = (int)((sort_key(xr[r], sg, desc) >> shift) & 255u) | (sg << 8);
                    }
                    const uint64_t m = sort_match(bucket, valid, nbits);
                    int pos = 0;
                    if (valid) pos = wtab[w][bucket] + __popcll(m & mask_lt(lane));
                    if (valid && (m >> lane) == 1ull) wtab[w][bucket] += __popcll(m);
                    if (valid) {
                        const int dl = sort_slot(pos, sort_seg(pos, vs), vs, off);
                        gst(a.X[dst] + dl, xr[r]);
                        gst(a.Y[dst] + dl, yr[r]);
                        gst(a.I[dst] + dl, ir[r]);
                    }
                }
            }
            grid_sync(a.bar, a.err);
        }
        // 6. check: neighbours inside a segment in key order
        if (t == 0) sbad = 0;
        __syncthreads();
        int bad = 0;
        for (int q = cb + t; q < ce; q += kBlock) {
            if (q == 0) continue;
            const int sg = sort_seg(q, vs);
            if (sort_seg(q - 1, vs) != sg) continue;
            const int sl = sort_slot(q, sg, vs, off);  // (q - 1 is the slot before)
            if (sort_key(gld(a.X[0] + sl), sg, desc) < sort_key(gld(a.X[0] + sl - 1), sg, desc)) ++bad;
        }
        if (bad) atomicAdd(&sbad, bad);
        __syncthreads();
        if (t == 0 && sbad) atomicAdd(&a.info->sort_bad, sbad);
        if (b == 0 && t == 0) a.info->sort_n = V;
    }
    stamp(a, 6);
    flush_counters(a.stats, ctr);
}

// Per-call initialisation (a normal launch before k_hull): barrier state,
// error word, counters, info block, the vertex bitmap, the first child
// records, and the set starts (validated).
__global__ void k_reset(HullArgs a)
{
    const int gtid = (int)(blockIdx.x * blockDim.x + threadIdx.x), gstride = (int)(gridDim.x * blockDim.x);
    if (gtid == 0) {
        a.bar->gen = 0;
        a.bar->top = 0;
        a.bar->emit_mode = 0;
        *a.err = 0;
        a.info->h_total = 0;
        a.info->passes = 0;
        a.info->nstamps = 0;
        a.info->first_v = 0;
        a.info->vcount = 0;
        a.info->vcap = a.vcap;
        a.info->pass_traced = 0;
        a.info->prefilter_n = -1;
        a.info->keep_n = 0;
        a.info->sort_n = -1;
        a.info->sort_bad = 0;
        a.info->stream_done = 0;
        a.info->spass_n = 0;
        a.info->stream_line = 0;
    }
    if (gtid < kBarSub) a.bar->sub[gtid][0] = 0;
    if (a.stream && gtid < 4) a.sdone[gtid] = 0u;
    for (int i = gtid; i < 4 * kStatSlots; i += gstride) a.stats[i] = 0;
    for (int i = gtid; i < a.W; i += gstride) a.bitmap[i] = 0ull;
    for (int i = gtid; i < 4 * a.G; i += gstride) {
        a.recs[i].len = 0;
        a.rec_cid[i] = -1;
    }
    if (a.set_off) {
        for (int s = gtid; s <= a.G; s += gstride) {
            const int64_t v = a.set_off[s];
            bool bad = v < 0 || v > a.N;
            if (s == 0 && v != 0) bad = true;
            if (s == a.G && v != a.N) bad = true;
            if (s > 0 && a.set_off[s - 1] > v) bad = true;
            if (bad) atomicOr(a.err, kErrBounds);
            a.gstart[s] = bad ? 0 : (int)v;
        }
    } else if (gtid == 0) {
        a.gstart[0] = 0;
        a.gstart[1] = a.N;
    }
}

}  // namespace sqh

namespace sqh {
// Vertex list for the small-hull emission (first kVListCap vertices).
__device__ __forceinline__ void note_vertex(HullInfo* info, int2* vlist, int key, int id)
{
    const int i = atomicAdd(&info->vcount, 1);
    if (i < info->vcap) vlist[i] = make_int2(key, id);
}
}  // namespace sqh
