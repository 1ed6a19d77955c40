// Streaming path for one large point set (device code, gfx950).
//
// k_stream runs the seed, the first split and the first compaction of a
// single hull (paper sections 4.3 - 4.4) as three streams over the input,
// one grid barrier each, then leaves the segment table of the first pass in
// the workspace for k_hull<kHullPasses>, which runs the passes and the
// emission. Compared with the general persistent kernel (groups of any size,
// reduce-then-scan phases with two barriers and two reads each), every
// workgroup here walks whole tiles of 16384 points:
//   * the input is read as 16-byte loads (two points per lane), eight rows
//     of them in flight per wave;
//   * the seed and the split keep private per-lane results (the lane's
//     lexicographic extremes; side counts and farthest points) that are
//     reduced once per workgroup; after the barrier every workgroup reduces
//     the workgroups' partial results itself, so no second barrier is
//     needed;
//   * the first compaction reads the input once: tiles are taken in rounds
//     (round r gives workgroup b tile r * grid + b), each tile publishes its
//     four bucket counts as one self-validating 64-bit word, and the tile's
//     output position is the sum of the counts of all earlier tiles (the
//     earlier rounds' totals, kept by every workgroup, plus the earlier
//     tiles of its round). Points then go straight from registers to their
//     child segment, ranked inside a row by ballots so that each row writes
//     contiguous runs.
// Farthest-point candidates are kept per lane as an area interval and an
// input index; the rare comparisons the interval cannot decide fetch the
// candidate's coordinates from the input and compare exactly (the order of
// section 4.4.1 with the tie rules of the general kernel, so the result is
// the same for every tile shape).
#pragma once

namespace sqh {

// Workgroups of 512 threads, two or more per compute unit, so that one
// workgroup's loads, barriers and slot reservations overlap another's
// arithmetic.
constexpr int kSWaves = 8;
constexpr int kSBlock = kSWaves * 64;
constexpr int kMaxSGrid = 1024;               // workgroups of a streaming launch (upper bound)
constexpr int kSRows = 8;                     // rows of point pairs per wave and tile
constexpr int kSTilePairs = kSBlock * kSRows;  // pairs per workgroup tile
constexpr int kSTile = 2 * kSTilePairs;       // points per workgroup tile (8192)
constexpr int kStreamMin = 1 << 16;           // single hulls of at least this many points take this path

// Farthest-point candidate of one lane: the area interval [lo, hi] =
// [fl(a - w), fl(a + w)] of the float32 estimate a with error bound w, and
// the input index (-1: none). Rounding is monotone, so lo(P) > hi(Q) proves
// area(P) > area(Q).
struct LCand {
    float lo, hi;
    int id;
};
__device__ __forceinline__ LCand lc_none()
{
    LCand c;
    c.lo = -INFINITY; c.hi = -INFINITY; c.id = -1;
    return c;
}

// A candidate with its coordinates (for reductions and the exact order).
struct FCand {
    float lo, hi, x, y;
    int id;
    int pad[3];
};
__device__ __forceinline__ FCand fc_none()
{
    FCand c;
    c.lo = -INFINITY; c.hi = -INFINITY; c.x = 0.0f; c.y = 0.0f; c.id = -1;
    c.pad[0] = c.pad[1] = c.pad[2] = 0;
    return c;
}

// Exact order of two distinct candidates for edge E (section 4.4.1 asks for
// the farthest point; ties as in the general kernel): exact area, then among
// equal areas the point earliest along E, then the lower index.
__device__ __forceinline__ bool beats_exact_xy(const Edge& E, float px, float py, int pid, float qx, float qy, int qid)
{
    const int s = area_cmp_exact(E.ox, E.oy, E.ex, E.ey, px, py, qx, qy);
    if (s != 0) return s > 0;
    if (px == qx && py == qy) return pid < qid;
    const bool p_first = (px < qx) || (px == qx && py < qy);
    return E.fwd ? p_first : !p_first;
}

__device__ __forceinline__ bool beats_exact_xy_inl(const Edge& E, float px, float py, int pid, float qx, float qy,
                                                  int qid)
{
    const int s = area_cmp_exact_inl(E.ox, E.oy, E.ex, E.ey, px, py, qx, qy);
    if (s != 0) return s > 0;
    if (px == qx && py == qy) return pid < qid;
    const bool p_first = (px < qx) || (px == qx && py < qy);
    return E.fwd ? p_first : !p_first;
}

// settle_p without a call: the exact sign of an undecided orientation
__device__ __forceinline__ void settle_inl(int& s, bool need, float ox, float oy, float ex, float ey, float px,
                                           float py, uint32_t& n_exact)
{
    if (__ballot(need)) {
        if (need) {
            s = orient_exact_inl(ox, oy, ex, ey, px, py);
            ++n_exact;
        }
    }
}

__device__ __forceinline__ bool fc_beats(const Edge& E, const FCand& P, const FCand& Q, bool fp64, uint32_t& n_exact)
{
    if (Q.id < 0) return P.id >= 0;
    if (P.id < 0) return false;
    if (!fp64) {
        if (P.lo > Q.hi) return true;
        if (Q.lo > P.hi) return false;
    }
    ++n_exact;
    return beats_exact_xy(E, P.x, P.y, P.id, Q.x, Q.y, Q.id);
}

// Offer point (px, py, id) with interval [lo, hi] to the lane's candidate q
// when m holds. Undecided comparisons fetch q's coordinates from the input.
__device__ __forceinline__ void lc_offer(LCand& q, bool m, float lo, float hi, int id, float px, float py,
                                         const Edge& E, const float2* xy, bool fp64, uint32_t& n_exact)
{
    // an empty q loses to any point; NaN bounds (overflow) leave the
    // comparison undecided, as does the float64-only mode
    const bool win0 = m && (q.id < 0 || (!fp64 && lo > q.hi));
    const bool und = m && !win0 && (fp64 || !(q.lo > hi));
    bool win = win0;
    if (__ballot(und)) {
        if (und) {
            const float2 Q = gld(xy + q.id);
            ++n_exact;
            win = beats_exact_xy_inl(E, px, py, id, Q.x, Q.y, q.id);
        }
    }
    if (win) {
        q.lo = lo; q.hi = hi; q.id = id;
    }
}

// Filter-only offer: takes the point when its interval proves it farther;
// returns true when only the exact order can decide (q is then unchanged).
// (bitwise logic throughout: short-circuit operators would become branches)
__device__ __forceinline__ bool lc_offer_fast(LCand& q, bool m, float lo, float hi, int id, bool fp64)
{
    const bool win = m & ((q.id < 0) | (!fp64 & (lo > q.hi)));
    const bool und = m & !win & (fp64 | !(q.lo > hi));
    q.lo = win ? lo : q.lo;
    q.hi = win ? hi : q.hi;
    q.id = win ? id : q.id;
    return und;
}

// fast_sign without branches
__device__ __forceinline__ int fsign(const Orient32& o, bool fp64)
{
    const bool ok = !fp64 & (fabsf(o.d) > o.es);
    return ok ? (o.d > 0.0f ? 1 : -1) : 0;
}

__device__ __forceinline__ FCand lc_full(const LCand& q, const float2* xy)
{
    FCand c = fc_none();
    if (q.id >= 0) {
        const float2 p = gld(xy + q.id);
        c.lo = q.lo; c.hi = q.hi; c.x = p.x; c.y = p.y; c.id = q.id;
    }
    return c;
}

__device__ __forceinline__ FCand shfl_xor_fc(const FCand& c, int m)
{
    FCand r;
    r.lo = __shfl_xor(c.lo, m); r.hi = __shfl_xor(c.hi, m);
    r.x = __shfl_xor(c.x, m); r.y = __shfl_xor(c.y, m);
    r.id = __shfl_xor(c.id, m);
    r.pad[0] = r.pad[1] = r.pad[2] = 0;
    return r;
}

__device__ __forceinline__ FCand wave_max_fc(const Edge& E, FCand v, bool fp64, uint32_t& n_exact)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const FCand o = shfl_xor_fc(v, m);
        // a total order: both lanes of a pair keep the same winner
        if (fc_beats(E, o, v, fp64, n_exact)) v = o;
    }
    return v;
}

// Block-wide farthest point (result valid on every thread). `lds` holds kSWaves entries.
__device__ __forceinline__ FCand block_max_fc(const Edge& E, FCand v, FCand* lds, bool fp64, uint32_t& n_exact)
{
    const int w = (int)(threadIdx.x >> 6), lane = lane_id();
    v = wave_max_fc(E, v, fp64, n_exact);
    __syncthreads();
    if (lane == 0) lds[w] = v;
    __syncthreads();
    FCand r = lds[lane & (kSWaves - 1)];  // (kSWaves is a power of two)
#pragma unroll
    for (int m = 1; m < kSWaves; m <<= 1) {
        const FCand o = shfl_xor_fc(r, m);
        if (fc_beats(E, o, r, fp64, n_exact)) r = o;
    }
    return r;  // lanes 0..15 of every wave agree; lane 0's is used
}

// Lexicographic extreme with the lowest index among coincident points.
struct Lex {
    float x, y;
    int id;
};
__device__ __forceinline__ bool lex_beats(bool mx, const Lex& P, const Lex& Q)
{
    const bool less = (P.x < Q.x) | ((P.x == Q.x) & (P.y < Q.y));
    const bool more = (P.x > Q.x) | ((P.x == Q.x) & (P.y > Q.y));
    const bool eq = (P.x == Q.x) & (P.y == Q.y);
    return (mx ? more : less) | (eq & (P.id < Q.id));
}
__device__ __forceinline__ Lex shfl_xor_lex(const Lex& c, int m)
{
    Lex r;
    r.x = __shfl_xor(c.x, m); r.y = __shfl_xor(c.y, m); r.id = __shfl_xor(c.id, m);
    return r;
}

struct SeedPart {
    float mnx, mny;
    int mni;
    float mxx, mxy;
    int mxi;
    int bad;
    int line;        // result only: the line filter applies (see LineF)
    float ylo, yhi;  // y range (the x range is [mnx, mxx])
    float Mx, My;    // result only: bounds on |x| and |y|
};

// Static line filter for the edge o -> e (the pre-filter's line test, with
// the error bound derived there): t(p) = fma(-dy, px, fma(dx, py, c)) with
// dx, dy = fl(e - o) and c = fl(fl(dy ox) - fl(dx oy)) differs from
// orient(o, e, p) by less than m = 2^-19 (|dx| My + |dy| Mx) + 2^-140 for
// every point of the input (Mx, My bound |x|, |y| over it, at most 2^60),
// so t < -m certifies orient < 0, t > m certifies orient > 0, and
// [-t - m, -t + m] encloses the area -orient. One evaluation is two FMAs;
// the constants come from the input's extent, once per edge.
struct LineF {
    float nx, ny, c, m;
    float m2;  // 2 m: the width of every area interval of this edge
};
__device__ __forceinline__ LineF make_line(float ox, float oy, float ex, float ey, float Mx, float My)
{
    const float dx = ex - ox, dy = ey - oy;
    LineF L;
    L.nx = -dy;
    L.ny = dx;
    L.c = dy * ox - dx * oy;
    L.m = (fabsf(dx) * My + fabsf(dy) * Mx) * kLineRel + kFilterTau;
    L.m2 = 2.0f * L.m;
    return L;
}
// an edge no point is strictly right of (a side without points)
__device__ __forceinline__ LineF line_never()
{
    LineF L;
    L.nx = 0.0f; L.ny = 0.0f; L.c = INFINITY; L.m = 0.0f; L.m2 = 0.0f;
    return L;
}
__device__ __forceinline__ float line_eval(const LineF& L, float px, float py)
{
    return fmaf(L.nx, px, fmaf(L.ny, py, L.c));
}

struct SplitPart {
    int cnt[4];
    FCand c[2];
};

struct FirstPart {
    FCand c[4];
};

// Per-call state of the streaming path in the workspace.
constexpr int kSPassMaxS = 256;      // streaming passes take at most this many segments ...
constexpr int kSPassMinV = 6144;         // ... and more than this many (fewer: k_stail)
constexpr int kPRows = 8;            // rows of points per wave and tile in a streaming pass
constexpr int kPTile = kSBlock * kPRows;

// Farthest points of one segment's two children found by one workgroup.
struct PassRec {
    FCand c[2];
};

struct StreamWs {
    SeedPart seed[kMaxSGrid];
    SplitPart split[kMaxSGrid];
    FirstPart first[kMaxSGrid];
    SeedPart seed_res;    // A (mn*), B (mx*), non-finite flag
    SplitPart split_res;  // n_lo, n_up, C_lo, C_up
    unsigned int done[4];   // workgroups finished: seed, split, first compaction, streaming pass
    unsigned int pad[60];
    unsigned int cursor[4]; // first compaction: points placed so far in each child
    unsigned int pad2[60];
    int state[2];           // {survivor buffer, pass} of the next pass
    int pad3[62];
    unsigned int pcursor[kSPassMaxS][2];  // streaming pass: points placed so far per segment and child
    // followed by the streaming pass's records (PassRec), one per tile that
    // starts a workgroup's run of tiles in one segment
};
__device__ __forceinline__ PassRec* pass_recs(void* ws) { return reinterpret_cast<PassRec*>(static_cast<StreamWs*>(ws) + 1); }

// A wave holds kSRows rows of a tile: with wp0 its first pair, row r of
// lane l is pair wp0 + 64 r + l.

// Loads pair p (points 2p and 2p + 1; npf full pairs, plus one point if
// odd). Point 2p + h exists iff 2p + h < n.
__device__ __forceinline__ float4 load_pair(const float2* xy, int npf, int odd, int p)
{
    float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (p < npf) {
        v = gld(reinterpret_cast<const float4*>(xy) + p);
    } else if (odd && p == npf) {
        const float2 t = gld(xy + 2 * p);
        v.x = t.x; v.y = t.y;
    }
    return v;
}

// The contiguous range of pairs [pb, pe) that workgroup b of nb takes: an
// equal share of whole rows for every workgroup, so that none runs a tile
// more than the others.
__device__ __forceinline__ void wg_range(int n, int b, int nb, int& pb, int& pe)
{
    const int npairs = (n + 1) >> 1;
    const int per = (((npairs + nb - 1) / nb) + 63) & ~63;
    pb = min(b * per, npairs);
    pe = min(pb + per, npairs);
}

// Points this lane holds in its wave's rows of a tile (pairs p0 + 64 r).
__device__ __forceinline__ uint32_t lane_points(int n, int p0, int wave_p0)
{
    if (2 * (wave_p0 + 64 * kSRows) <= n) return 2 * kSRows;  // the wave's rows are full
    uint32_t c = 0;
#pragma unroll
    for (int r = 0; r < kSRows; ++r) c += (uint32_t)min(max(n - 2 * (p0 + 64 * r), 0), 2);
    return c;
}

// Loads this lane's pairs p0 + 64 r of one wave's rows (first pair
// wave_p0): unguarded 16-byte loads when every point exists, so that all
// loads are in flight together.
__device__ __forceinline__ void load_rows(const float2* xy, int n, int p0, int wave_p0, float4 (&v)[kSRows])
{
    if (2 * (wave_p0 + 64 * kSRows) <= n) {
        const float4* x4 = reinterpret_cast<const float4*>(xy) + p0;
#pragma unroll
        for (int r = 0; r < kSRows; ++r) v[r] = gld(x4 + 64 * r);
    } else {
#pragma unroll
        for (int r = 0; r < kSRows; ++r) v[r] = load_pair(xy, n >> 1, n & 1, p0 + 64 * r);
    }
}

// One 64-bit word per tile: bit 63 marks it written, four 15-bit counts.
__device__ __forceinline__ uint64_t pack_counts(const int (&c)[4])
{
    return (1ull << 63) | (uint64_t)c[0] | ((uint64_t)c[1] << 15) | ((uint64_t)c[2] << 30) | ((uint64_t)c[3] << 45);
}
__device__ __forceinline__ void unpack_counts(uint64_t v, int (&c)[4])
{
    c[0] = (int)(v & 0x7fff); c[1] = (int)((v >> 15) & 0x7fff);
    c[2] = (int)((v >> 30) & 0x7fff); c[3] = (int)((v >> 45) & 0x7fff);
}

// set bits of M below this lane
__device__ __forceinline__ int lanes_below(uint64_t M)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
}

// Block-wide exclusive scan of one pair per thread (kSWaves waves); *tot
// receives the block total.
__device__ __forceinline__ Pair sblock_excl_scan(Pair v, Pair* red, Pair* tot)
{
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const Pair inc = {wave_incl_sum(v.a), wave_incl_sum(v.b)};
    __syncthreads();
    if (lane == 63) red[w] = inc;
    __syncthreads();
    Pair off = {0, 0}, all = {0, 0};
#pragma unroll
    for (int u = 0; u < kSWaves; ++u) {
        if (u < w) { off.a += red[u].a; off.b += red[u].b; }
        all.a += red[u].a; all.b += red[u].b;
    }
    *tot = all;
    return Pair{off.a + inc.a - v.a, off.b + inc.b - v.b};
}

__device__ __forceinline__ int wave_sum(int v) { return wave_total(v); }

// Lower side (strictly right of A->B): edges A->C_lo (bucket 0) and C_lo->B
// (bucket 1); upper side: B->C_up (2) and C_up->A (3). Section 4.4.3 keeps
// a point for the child whose edge it is strictly right of (the paper's
// "and" reads "or": with an exact farthest point no point is right of both).
struct FirstGeo {
    float ax, ay, bx, by, lx, ly, ux, uy;
};

// Filter-only classification: 0..3, 7 (no child), or 15 when a sign needs
// the exact path.
__device__ __forceinline__ int first_fast(const FirstGeo& g, float x, float y, bool valid, bool fp64, float& a,
                                          float& w)
{
    const Orient32 o = orient32p(g.ax, g.ay, g.bx, g.by, x, y);
    const int side = fsign(o, fp64);
    const bool up = side > 0;
    const float sx = up ? g.bx : g.ax, sy = up ? g.by : g.ay;
    const float mx = up ? g.ux : g.lx, my = up ? g.uy : g.ly;
    const float tx = up ? g.ax : g.bx, ty = up ? g.ay : g.by;
    const Orient32 o1 = orient32p(sx, sy, mx, my, x, y);
    const Orient32 o2 = orient32p(mx, my, tx, ty, x, y);
    const int s1 = fsign(o1, fp64), s2 = fsign(o2, fp64);
    const bool in1 = s1 < 0, in2 = !in1 & (s2 < 0);
    a = -(in1 ? o1.d : o2.d);
    w = 2.0f * (in1 ? o1.es : o2.es);
    const int b = up ? 2 : 0;
    // undecided: the side, or the first edge's sign, or (first edge not
    // outside) the second edge's sign
    const bool und = (side == 0) | (s1 == 0) | ((s1 > 0) & (s2 == 0));
    return !valid ? 7 : (und ? 15 : (in1 ? b : (in2 ? b + 1 : 7)));
}

struct FirstLane {
    LCand q[4];
    uint32_t code_lo, code_hi;
    uint32_t n_orient_exact, n_cmp_exact;
};

// Filter-only pass over one wave's rows of a tile: codes (4 bits per point,
// 15 = settle exactly) and the lanes' candidates; returns the pending mask.
__device__ __forceinline__ uint32_t first_fast_rows(FirstLane& s, const float4 (&v)[kSRows], int p0, int n,
                                                    const FirstGeo& g, bool fp64)
{
    uint32_t pend = 0u;
#pragma unroll
    for (int rr = 0; rr < kSRows; ++rr) {
        const int id0 = 2 * (p0 + 64 * rr);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float x = h ? v[rr].z : v[rr].x, y = h ? v[rr].w : v[rr].y;
            const bool m = id0 + h < n;
            float ar, wr;
            int code = first_fast(g, x, y, m, fp64, ar, wr);
            const float lo = ar - wr, hi = ar + wr;
            bool und = code == 15;
#pragma unroll
            for (int k = 0; k < 4; ++k) und |= lc_offer_fast(s.q[k], code == k, lo, hi, id0 + h, fp64);
            code = und ? 15 : code;
            pend |= (uint32_t)und << (2 * rr + h);
            const int sh = 4 * (2 * (rr & 3) + h);
            if (rr < 4) s.code_lo |= (uint32_t)code << sh;
            else s.code_hi |= (uint32_t)code << sh;
        }
    }
    return pend;
}

// The first compaction with the line filter of the four edges A->C_lo,
// C_lo->B, B->C_up, C_up->A: a point belongs to the child whose edge it is
// strictly right of. This is the side-then-edges rule: a point right of
// A->C_lo or C_lo->B is right of A->B (A is the lexicographic minimum, so
// seen from A every point lies in a half-plane where "clockwise of" orders
// directions), likewise for the upper edges seen from B, and no point is
// right of both edges of one side (C is the farthest point). So one
// certified negative edge decides the child, four certified positive edges
// discard the point, and anything else is settled exactly.
//
// Every area interval of one edge has the same width 2m, so a lane keeps,
// per child, the centre of its candidate's interval: a point wins when its
// centre is more than 2m above, and is settled exactly when it is within
// 2m. A point is offered to every child whose edge does not certify it
// outside (not only to its own): a point that is not in child k has an
// exact area of at most 0 for k's edge, below every point of the child, so
// such a candidate only lasts where the lane has no point of the child, and
// the exact comparisons keep the order right.
struct LineCand {
    float c;  // centre of the area interval
    int id;
};
struct FirstLineLane {
    LineCand q[4];
    uint32_t code_lo, code_hi;
    uint32_t n_orient_exact, n_cmp_exact;
};

__device__ __forceinline__ uint32_t first_line_rows(FirstLineLane& s, const float4 (&v)[kSRows], int p0, int n,
                                                    const LineF (&L)[4])
{
    uint32_t pend = 0u;
#pragma unroll
    for (int rr = 0; rr < kSRows; ++rr) {
        const int id0 = 2 * (p0 + 64 * rr);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float x = h ? v[rr].z : v[rr].x, y = h ? v[rr].w : v[rr].y;
            const bool m = id0 + h < n;
            float t[4];
            bool neg[4], pos[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                t[k] = line_eval(L[k], x, y);
                neg[k] = t[k] < -L[k].m;
                pos[k] = t[k] > L[k].m;
            }
            int code = neg[0] ? 0 : (neg[1] ? 1 : (neg[2] ? 2 : (neg[3] ? 3 : 7)));
            bool und = m & !(neg[0] | neg[1] | neg[2] | neg[3]) & !(pos[0] & pos[1] & pos[2] & pos[3]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float a = -t[k];
                const float u = a - s.q[k].c;  // +inf while the lane has no candidate
                const bool mk = m & !pos[k];
                const bool win = mk & (u > L[k].m2);
                und |= mk & !win & (u >= -L[k].m2);
                s.q[k].c = win ? a : s.q[k].c;
                s.q[k].id = win ? id0 + h : s.q[k].id;
            }
            code = !m ? 7 : (und ? 15 : code);
            pend |= (uint32_t)und << (2 * rr + h);
            const int sh = 4 * (2 * (rr & 3) + h);
            if (rr < 4) s.code_lo |= (uint32_t)code << sh;
            else s.code_hi |= (uint32_t)code << sh;
        }
    }
    return pend;
}

__device__ __forceinline__ int first_classify(const FirstGeo& g, float x, float y, bool valid, bool fp64, float& a,
                                              float& w, Counters& ctr)
{
    ctr.orient += valid ? 3 : 0;
    const Orient32 o = orient32p(g.ax, g.ay, g.bx, g.by, x, y);
    int side = fast_sign(o, fp64);
    settle_inl(side, valid && side == 0, g.ax, g.ay, g.bx, g.by, x, y, ctr.orient_exact);
    const bool up = side > 0;
    const float sx = up ? g.bx : g.ax, sy = up ? g.by : g.ay;  // first edge's start
    const float mx = up ? g.ux : g.lx, my = up ? g.uy : g.ly;  // apex
    const float tx = up ? g.ax : g.bx, ty = up ? g.ay : g.by;  // second edge's end
    const Orient32 o1 = orient32p(sx, sy, mx, my, x, y);
    const Orient32 o2 = orient32p(mx, my, tx, ty, x, y);
    int s1 = fast_sign(o1, fp64), s2 = fast_sign(o2, fp64);
    const bool live = valid && side != 0;
    settle_inl(s1, live && s1 == 0, sx, sy, mx, my, x, y, ctr.orient_exact);
    settle_inl(s2, live && s1 >= 0 && s2 == 0, mx, my, tx, ty, x, y, ctr.orient_exact);
    const bool in1 = s1 < 0, in2 = !in1 && s2 < 0;
    a = -(in1 ? o1.d : o2.d);
    w = 2.0f * (in1 ? o1.es : o2.es);
    const int b = up ? 2 : 0;
    return !live ? 7 : (in1 ? b : (in2 ? b + 1 : 7));
}

__device__ __forceinline__ bool spin_word(const uint64_t* p, uint64_t& v, int* err)
{
    int spins = 0;
    while (!((v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 63)) {
        if (++spins > kSpinLimit) {
            atomicOr(err, kErrSpin);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Timestamp by any one thread (the streaming kernels' phase ends are seen by
// whichever workgroup finishes last).
__device__ __forceinline__ void stamp_here(const HullArgs& a, int tag)
{
    if (a.timing) {
        const int k = a.info->nstamps;
        if (k < kMaxStamps) {
            a.info->stamp[k] = wall_clock64();
            a.info->stamp_tag[k] = tag;
            a.info->nstamps = k + 1;
        }
    }
}

__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Values every lane holds alike, moved to scalar registers (results loaded
// through vector loads otherwise stay in vector registers).
__device__ __forceinline__ float uni(float v) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v))); }
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ SeedPart uni(const SeedPart& p)
{
    SeedPart r;
    r.mnx = uni(p.mnx); r.mny = uni(p.mny); r.mni = uni(p.mni);
    r.mxx = uni(p.mxx); r.mxy = uni(p.mxy); r.mxi = uni(p.mxi);
    r.bad = uni(p.bad); r.line = uni(p.line);
    r.ylo = uni(p.ylo); r.yhi = uni(p.yhi); r.Mx = uni(p.Mx); r.My = uni(p.My);
    return r;
}

// True on the workgroup that arrives last at counter *ctr (nb arrivals), after
// it has acquired every earlier arrival's writes.
__device__ __forceinline__ bool last_arrival(unsigned int* ctr, int nb)
{
    __shared__ int s_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned int k = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_last = k == (unsigned int)nb - 1u;
        if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_last != 0;
}

// ---- cold code: reductions (out of line, called where little is live) and
// the exact settling of the few points the filter leaves open (inline, one
// copy, run only by waves that have such a point)

// Block-wide farthest point for edge o -> e (every thread gets it).
__device__ __noinline__ FCand block_max_call(float ox, float oy, float ex, float ey, FCand v, int fp64)
{
    __shared__ FCand lds[kSWaves];
    const Edge E = make_edge(ox, oy, ex, ey);
    uint32_t n = 0;
    return block_max_fc(E, v, lds, fp64 != 0, n);
}

// Lane state of the split and its exact settling.
struct SplitLane {
    LCand q0, q1;
    int c0, c1;
    uint32_t n_orient_exact, n_cmp_exact;
};

// Points (bit i of pend: row i / 2, point i % 2 of pairs p0 + 64 r) whose side
// or farthest-point comparison the filter left open.
__device__ __forceinline__ void split_pending(SplitLane* st, uint32_t pend, int p0, float ax, float ay, float bx,
                                           float by, const float2* xy, int fp64)
{
    const bool f64 = fp64 != 0;
    const Edge eab = make_edge(ax, ay, bx, by), eba = make_edge(bx, by, ax, ay);
    SplitLane s = *st;
#pragma unroll 1
    for (int i = 0; i < 2 * kSRows; ++i) {
        const bool mine = (pend >> i) & 1u;
        if (!__ballot(mine)) continue;
        if (mine) {
            const int id = 2 * (p0 + 64 * (i >> 1)) + (i & 1);
            const float2 P = gld(xy + id);
            const Orient32 o = orient32p(ax, ay, bx, by, P.x, P.y);
            int sg = fast_sign(o, f64);
            if (sg == 0) {
                sg = orient_exact_inl(ax, ay, bx, by, P.x, P.y);
                ++s.n_orient_exact;
            }
            const float ar = sg < 0 ? -o.d : o.d, wr = 2.0f * o.es;
            const float lo = ar - wr, hi = ar + wr;
            const bool lower = sg < 0, upper = sg > 0;
            // the fast pass neither counted nor offered a pending point
            s.c0 += lower ? 1 : 0;
            s.c1 += upper ? 1 : 0;
            lc_offer(s.q0, lower, lo, hi, id, P.x, P.y, eab, xy, f64, s.n_cmp_exact);
            lc_offer(s.q1, upper, lo, hi, id, P.x, P.y, eba, xy, f64, s.n_cmp_exact);
        }
    }
    *st = s;
}



__device__ __forceinline__ void first_pending(FirstLane* st, uint32_t pend, int p0, FirstGeo g, const float2* xy,
                                           int fp64)
{
    const bool f64 = fp64 != 0;
    Edge E[4];
    E[0] = make_edge(g.ax, g.ay, g.lx, g.ly);
    E[1] = make_edge(g.lx, g.ly, g.bx, g.by);
    E[2] = make_edge(g.bx, g.by, g.ux, g.uy);
    E[3] = make_edge(g.ux, g.uy, g.ax, g.ay);
    FirstLane s = *st;
#pragma unroll 1
    for (int i = 0; i < 2 * kSRows; ++i) {
        const bool mine = (pend >> i) & 1u;
        if (!__ballot(mine)) continue;
        if (mine) {
            const int id = 2 * (p0 + 64 * (i >> 1)) + (i & 1);
            const float2 P = gld(xy + id);
            float ar, wr;
            Counters c = {0u, s.n_orient_exact, 0u};
            const int code = first_classify(g, P.x, P.y, true, f64, ar, wr, c);
            s.n_orient_exact = c.orient_exact;
            const float lo = ar - wr, hi = ar + wr;
            // the fast pass offered nothing for a pending point
#pragma unroll
            for (int k = 0; k < 4; ++k) lc_offer(s.q[k], code == k, lo, hi, id, P.x, P.y, E[k], xy, f64, s.n_cmp_exact);
            const int sh = 4 * (i & 7);
            if (i < 8) s.code_lo = (s.code_lo & ~(15u << sh)) | ((uint32_t)code << sh);
            else s.code_hi = (s.code_hi & ~(15u << sh)) | ((uint32_t)code << sh);
        }
    }
    *st = s;
}

// The pending points of first_line_rows, one at a time: the exact child,
// and the offer to it with the point's line interval.
__device__ __forceinline__ void first_pending_line(FirstLineLane* st, uint32_t pend, int p0, FirstGeo g,
                                                   const LineF (&L)[4], const float2* xy)
{
    Edge E[4];
    E[0] = make_edge(g.ax, g.ay, g.lx, g.ly);
    E[1] = make_edge(g.lx, g.ly, g.bx, g.by);
    E[2] = make_edge(g.bx, g.by, g.ux, g.uy);
    E[3] = make_edge(g.ux, g.uy, g.ax, g.ay);
    FirstLineLane s = *st;
#pragma unroll 1
    for (int i = 0; i < 2 * kSRows; ++i) {
        const bool mine = (pend >> i) & 1u;
        if (!__ballot(mine)) continue;
        if (mine) {
            const int id = 2 * (p0 + 64 * (i >> 1)) + (i & 1);
            const float2 P = gld(xy + id);
            float ar, wr;
            Counters c = {0u, s.n_orient_exact, 0u};
            const int code = first_classify(g, P.x, P.y, true, false, ar, wr, c);
            s.n_orient_exact = c.orient_exact;
            if (code < 4) {
                // one comparison, on child `code`'s edge and candidate
                // (selected, so that the exact code is inlined once)
                const bool k0 = code == 0, k1 = code == 1, k2 = code == 2;
                const LineF Lk = k0 ? L[0] : (k1 ? L[1] : (k2 ? L[2] : L[3]));
                const Edge Ek = k0 ? E[0] : (k1 ? E[1] : (k2 ? E[2] : E[3]));
                const float qc = k0 ? s.q[0].c : (k1 ? s.q[1].c : (k2 ? s.q[2].c : s.q[3].c));
                const int qid = k0 ? s.q[0].id : (k1 ? s.q[1].id : (k2 ? s.q[2].id : s.q[3].id));
                const float a = -line_eval(Lk, P.x, P.y);
                const float u = a - qc;
                bool win = u > Lk.m2;
                if (!win && u >= -Lk.m2) {
                    const float2 Q = gld(xy + qid);
                    ++s.n_cmp_exact;
                    win = beats_exact_xy_inl(Ek, P.x, P.y, id, Q.x, Q.y, qid);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const bool take = win && code == k;
                    s.q[k].c = take ? a : s.q[k].c;
                    s.q[k].id = take ? id : s.q[k].id;
                }
            }
            const int sh = 4 * (i & 7);
            if (i < 8) s.code_lo = (s.code_lo & ~(15u << sh)) | ((uint32_t)code << sh);
            else s.code_hi = (s.code_hi & ~(15u << sh)) | ((uint32_t)code << sh);
        }
    }
    *st = s;
}

// Workgroup partial of the split: side counts and farthest points.
__device__ __forceinline__ void split_wg_partial(SplitPart* out, SplitLane s, float ax, float ay, float bx, float by,
                                              const float2* xy, int fp64)
{
    __shared__ int cnt[kSWaves][2];
    const int lane = lane_id(), w = wave_index();
    const int c0 = wave_sum(s.c0), c1 = wave_sum(s.c1);
    if (lane == 0) { cnt[w][0] = c0; cnt[w][1] = c1; }
    const FCand f0 = block_max_call(ax, ay, bx, by, lc_full(s.q0, xy), fp64);
    const FCand f1 = block_max_call(bx, by, ax, ay, lc_full(s.q1, xy), fp64);
    if (threadIdx.x == 0) {
        SplitPart sp;
        sp.cnt[0] = 0; sp.cnt[1] = 0; sp.cnt[2] = 0; sp.cnt[3] = 0;
        for (int u = 0; u < kSWaves; ++u) { sp.cnt[0] += cnt[u][0]; sp.cnt[1] += cnt[u][1]; }
        sp.c[0] = f0;
        sp.c[1] = f1;
        gst(out, sp);
    }
}

// The last workgroup of the seed: A, B and the non-finite flag; the state
// of the streaming passes.
__device__ __forceinline__ void seed_finish(const HullArgs& a)
{
    __shared__ Lex s_lex[2][kSWaves];
    __shared__ int s_bad[kSWaves];
    auto* ws = static_cast<StreamWs*>(a.sws);
    const int t = (int)threadIdx.x, lane = lane_id(), w = wave_index(), nb = (int)gridDim.x;
    if (t < 2 * kSPassMaxS) (&ws->pcursor[0][0])[t] = 0u;
    if (t < 2) ws->state[t] = 0;
    Lex mn = {INFINITY, INFINITY, 0x7fffffff}, mx = {-INFINITY, -INFINITY, 0x7fffffff};
    int bad = 0;
    float ylo = INFINITY, yhi = -INFINITY;
    for (int u = t; u < nb; u += kSBlock) {
        const SeedPart sp = gld(&ws->seed[u]);
        const Lex p0 = {sp.mnx, sp.mny, sp.mni}, p1 = {sp.mxx, sp.mxy, sp.mxi};
        if (lex_beats(false, p0, mn)) mn = p0;
        if (lex_beats(true, p1, mx)) mx = p1;
        bad |= sp.bad;
        ylo = fminf(ylo, sp.ylo);
        yhi = fmaxf(yhi, sp.yhi);
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Lex o0 = shfl_xor_lex(mn, m), o1 = shfl_xor_lex(mx, m);
        if (lex_beats(false, o0, mn)) mn = o0;
        if (lex_beats(true, o1, mx)) mx = o1;
        bad |= __shfl_xor(bad, m);
        ylo = fminf(ylo, __shfl_xor(ylo, m));
        yhi = fmaxf(yhi, __shfl_xor(yhi, m));
    }
    __shared__ float s_y[2][kSWaves];
    if (lane == 0) { s_lex[0][w] = mn; s_lex[1][w] = mx; s_bad[w] = bad; s_y[0][w] = ylo; s_y[1][w] = yhi; }
    __syncthreads();
    if (t == 0) {
        Lex q0 = s_lex[0][0], q1 = s_lex[1][0];
        int qb = s_bad[0];
        float y0 = s_y[0][0], y1 = s_y[1][0];
        for (int u = 1; u < kSWaves; ++u) {
            if (lex_beats(false, s_lex[0][u], q0)) q0 = s_lex[0][u];
            if (lex_beats(true, s_lex[1][u], q1)) q1 = s_lex[1][u];
            qb |= s_bad[u];
            y0 = fminf(y0, s_y[0][u]);
            y1 = fmaxf(y1, s_y[1][u]);
        }
        SeedPart r;
        r.mnx = q0.x; r.mny = q0.y; r.mni = q0.id;
        r.mxx = q1.x; r.mxy = q1.y; r.mxi = q1.id;
        r.bad = qb;
        r.ylo = y0; r.yhi = y1;
        // the line filter needs |coordinates| <= 2^60, and pays off when the
        // input is not far from the origin compared with its extent (its
        // bound grows with the coordinates, the orientation filter's with
        // the offsets)
        r.Mx = fmaxf(fabsf(q0.x), fabsf(q1.x));
        r.My = fmaxf(fabsf(y0), fabsf(y1));
        const float ext = fmaxf(q1.x - q0.x, y1 - y0);
        r.line = (a.line_ok && !a.fp64 && !qb && fmaxf(r.Mx, r.My) <= kLineCoordMax && r.Mx <= 8.0f * ext &&
                  r.My <= 8.0f * ext) ? 1 : 0;
        gst(&ws->seed_res, r);
        a.info->stream_line = r.line;
        if (qb) atomicOr(a.err, kErrNonFinite);
        SetInfo si = {};
        si.ax = q0.x; si.ay = q0.y; si.aid = q0.id;
        si.bx = q1.x; si.by = q1.y; si.bid = q1.id;
        gst(a.sets, si);
        if (!qb && q0.x == q1.x && q0.y == q1.y) {
            // every point sits at one position: the hull is its lowest index
            record_vertex(a.bitmap, a.vidx, a.vlist, a.info, 0, q0.id);
            a.sv[0] = 0;
            a.sv[1] = 0;
            a.vstart[0][0] = 0;
        }
        stamp_here(a, 1);
    }
}

// The last workgroup of the split: side counts and farthest points over all
// workgroups, the vertex keys of A and B.
__device__ __forceinline__ void split_finish(const HullArgs& a, float ax, float ay, float bx, float by, int aid, int bid)
{
    __shared__ int cnt[kSWaves][2];
    auto* ws = static_cast<StreamWs*>(a.sws);
    const int t = (int)threadIdx.x, lane = lane_id(), w = wave_index(), nb = (int)gridDim.x;
    int c0 = 0, c1 = 0;
    FCand f0 = fc_none(), f1 = fc_none();
    {
        const Edge eab = make_edge(ax, ay, bx, by), eba = make_edge(bx, by, ax, ay);
        uint32_t nx = 0;
        for (int u = t; u < nb; u += kSBlock) {
            c0 += gld(&ws->split[u].cnt[0]);
            c1 += gld(&ws->split[u].cnt[1]);
            const FCand g0 = gld(&ws->split[u].c[0]), g1 = gld(&ws->split[u].c[1]);
            if (fc_beats(eab, g0, f0, a.fp64 != 0, nx)) f0 = g0;
            if (fc_beats(eba, g1, f1, a.fp64 != 0, nx)) f1 = g1;
        }
    }
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    if (lane == 0) { cnt[w][0] = c0; cnt[w][1] = c1; }
    f0 = block_max_call(ax, ay, bx, by, f0, a.fp64);
    f1 = block_max_call(bx, by, ax, ay, f1, a.fp64);
    if (t == 0) {
        int n_lo = 0, n_up = 0;
        for (int u = 0; u < kSWaves; ++u) { n_lo += cnt[u][0]; n_up += cnt[u][1]; }
        SplitPart r;
        r.cnt[0] = n_lo; r.cnt[1] = n_up; r.cnt[2] = 0; r.cnt[3] = 0;
        r.c[0] = f0;
        r.c[1] = f1;
        gst(&ws->split_res, r);
        // vertex keys: A at the first slot, B right after the lower side
        record_vertex(a.bitmap, a.vidx, a.vlist, a.info, 0, aid);
        record_vertex(a.bitmap, a.vidx, a.vlist, a.info, 1 + n_lo, bid);
        SetInfo si = gld(a.sets);
        si.n_lo = n_lo; si.n_up = n_up;
        si.clx = f0.x; si.cly = f0.y; si.clid = f0.id;
        si.cux = f1.x; si.cuy = f1.y; si.cuid = f1.id;
        gst(a.sets, si);
        if (n_lo == 0 && n_up == 0) {
            // collinear input: the hull is [A, B]
            a.sv[0] = 0;
            a.sv[1] = 0;
            a.vstart[0][0] = 0;
        }
        stamp_here(a, 2);
    }
}

// Workgroup partial of the first compaction (farthest point of each child).
__device__ __forceinline__ void first_wg_partial(FirstPart* out, FirstLane s, FirstGeo g, const float2* xy, int fp64)
{
    FirstPart fp;
    fp.c[0] = block_max_call(g.ax, g.ay, g.lx, g.ly, lc_full(s.q[0], xy), fp64);
    fp.c[1] = block_max_call(g.lx, g.ly, g.bx, g.by, lc_full(s.q[1], xy), fp64);
    fp.c[2] = block_max_call(g.bx, g.by, g.ux, g.uy, lc_full(s.q[2], xy), fp64);
    fp.c[3] = block_max_call(g.ux, g.uy, g.ax, g.ay, lc_full(s.q[3], xy), fp64);
    if (threadIdx.x == 0) gst(out, fp);
}

// The last workgroup of the first compaction: the farthest point of each child
// over all workgroups, the children as the first pass's segment table
// (sections 4.4.2 / 4.4.4), and the ring keys of C_lo and C_up.
__device__ __forceinline__ void first_finish(const HullArgs& a, FirstGeo g, int n_lo, int n_up, int clid, int cuid, int cnt0,
                                          int cnt1, int cnt2, int cnt3)
{
    auto* ws = static_cast<StreamWs*>(a.sws);
    const int t = (int)threadIdx.x, nb = (int)gridDim.x;
    const float ex[5] = {g.ax, g.lx, g.bx, g.ux, g.ax}, ey[5] = {g.ay, g.ly, g.by, g.uy, g.ay};
    FCand C[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const Edge E = make_edge(ex[k], ey[k], ex[k + 1], ey[k + 1]);
        uint32_t nx = 0;
        FCand f = fc_none();
        for (int u = t; u < nb; u += kSBlock) {
            const FCand g2 = gld(&ws->first[u].c[k]);
            if (fc_beats(E, g2, f, a.fp64 != 0, nx)) f = g2;
        }
        C[k] = block_max_call(ex[k], ey[k], ex[k + 1], ey[k + 1], f, a.fp64);
    }
    if (t == 0) {
        const int cnt[4] = {cnt0, cnt1, cnt2, cnt3};
        if (n_lo > 0) record_vertex(a.bitmap, a.vidx, a.vlist, a.info, 1 + cnt0, clid);
        if (n_up > 0) record_vertex(a.bitmap, a.vidx, a.vlist, a.info, 2 + n_lo + cnt2, cuid);
        const int off[4] = {1, 1 + n_lo - cnt1, 2 + n_lo, 2 + n_lo + n_up - cnt3};
        int S = 0, V = 0;
        for (int k = 0; k < 4; ++k) {
            if (cnt[k] <= 0) continue;
            Seg sg;
            sg.ax = ex[k]; sg.ay = ey[k]; sg.bx = ex[k + 1]; sg.by = ey[k + 1];
            sg.cx = C[k].x; sg.cy = C[k].y;
            sg.off = off[k];
            sg.len = cnt[k];
            gst(a.segs[0] + S, sg);
            a.seg_cid[0][S] = C[k].id;
            a.vstart[0][S] = V;
            ++S;
            V += cnt[k];
        }
        a.vstart[0][S] = V;
        a.sv[0] = S;
        a.sv[1] = V;
        stamp_here(a, 3);
    }
}

// ==================================================================== seed
// Lexicographic minimum and maximum of the input (section 4.3: the leftmost
// and rightmost points; coincident points: the lowest index) and the
// non-finite check.
__global__ __launch_bounds__(kSBlock) void k_sseed(HullArgs a)
{
    __shared__ Lex s_lex[2][kSWaves];
    __shared__ int s_bad[kSWaves];
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int t = (int)threadIdx.x, lane = lane_id(), w = wave_index();
    const int n = a.N;
    int pb, pe;
    wg_range(n, b, nb, pb, pe);
    const int nend = min(n, 2 * pe);  // points of this workgroup's range: ids below nend
    const float2* xy = a.xy;
    auto* ws = static_cast<StreamWs*>(a.sws);
    if (b == 0 && t == 0) stamp_here(a, 0);
    Lex mn = {INFINITY, INFINITY, 0x7fffffff}, mx = {-INFINITY, -INFINITY, 0x7fffffff};
    float ylo = INFINITY, yhi = -INFINITY;
    bool bad = false;
    // each wave takes every kSWaves-th block of rows of the range (waves
    // do not wait for each other here)
    for (int wp0 = pb + w * (kSRows * 64); wp0 < pe; wp0 += kSTilePairs) {
        const int p0 = wp0 + lane;
        float4 v[kSRows];
        load_rows(xy, nend, p0, wp0, v);
#pragma unroll
        for (int r = 0; r < kSRows; ++r) {
            const int id0 = 2 * (p0 + 64 * r);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float x = h ? v[r].z : v[r].x, y = h ? v[r].w : v[r].y;
                const bool m = id0 + h < nend;
                bad |= m & !((int)isfinite(x) & (int)isfinite(y));
                ylo = m ? fminf(ylo, y) : ylo;
                yhi = m ? fmaxf(yhi, y) : yhi;
                // a lane sees its points in increasing index order: strict
                // comparisons keep the lowest index among coincident points
                const bool lt = m & ((x < mn.x) | ((x == mn.x) & (y < mn.y)));
                const bool gt = m & ((x > mx.x) | ((x == mx.x) & (y > mx.y)));
                mn.x = lt ? x : mn.x; mn.y = lt ? y : mn.y; mn.id = lt ? id0 + h : mn.id;
                mx.x = gt ? x : mx.x; mx.y = gt ? y : mx.y; mx.id = gt ? id0 + h : mx.id;
            }
        }
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Lex o0 = shfl_xor_lex(mn, m), o1 = shfl_xor_lex(mx, m);
        if (lex_beats(false, o0, mn)) mn = o0;
        if (lex_beats(true, o1, mx)) mx = o1;
        ylo = fminf(ylo, __shfl_xor(ylo, m));
        yhi = fmaxf(yhi, __shfl_xor(yhi, m));
    }
    __shared__ float s_y[2][kSWaves];
    const int any_bad = __ballot(bad) != 0ull;
    if (lane == 0) { s_lex[0][w] = mn; s_lex[1][w] = mx; s_bad[w] = any_bad; s_y[0][w] = ylo; s_y[1][w] = yhi; }
    __syncthreads();
    if (t == 0) {
        Lex q0 = s_lex[0][0], q1 = s_lex[1][0];
        int qb = s_bad[0];
        float y0 = s_y[0][0], y1 = s_y[1][0];
        for (int u = 1; u < kSWaves; ++u) {
            if (lex_beats(false, s_lex[0][u], q0)) q0 = s_lex[0][u];
            if (lex_beats(true, s_lex[1][u], q1)) q1 = s_lex[1][u];
            qb |= s_bad[u];
            y0 = fminf(y0, s_y[0][u]);
            y1 = fmaxf(y1, s_y[1][u]);
        }
        SeedPart sp;
        sp.mnx = q0.x; sp.mny = q0.y; sp.mni = q0.id;
        sp.mxx = q1.x; sp.mxy = q1.y; sp.mxi = q1.id;
        sp.bad = qb; sp.line = 0;
        sp.ylo = y0; sp.yhi = y1; sp.Mx = 0.0f; sp.My = 0.0f;
        gst(&ws->seed[b], sp);
    }
    // clear the first compaction's child cursors (used after this kernel)
    if (b == 0 && t < 4) ws->cursor[t] = 0u;
    if (last_arrival(&ws->done[0], nb)) seed_finish(a);
}

// =================================================================== split
// Side of every point w.r.t. the line A->B (section 4.3) and the farthest
// point of each side (section 4.4.1). Points on the line belong to neither
// side.
__global__ __launch_bounds__(kSBlock, 4) void k_ssplit(HullArgs a)
{
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int lane = lane_id(), w = wave_index();
    const int fp64 = a.fp64;
    const int n = a.N;
    int pb, pe;
    wg_range(n, b, nb, pb, pe);
    const int nend = min(n, 2 * pe);  // points of this workgroup's range: ids below nend
    const float2* xy = a.xy;
    auto* ws = static_cast<StreamWs*>(a.sws);
    const SeedPart sr = uni(gld(&ws->seed_res));
    if (sr.bad || (sr.mnx == sr.mxx && sr.mny == sr.mxy)) return;  // finished by the seed
    const float ax = sr.mnx, ay = sr.mny, bx = sr.mxx, by = sr.mxy;
    const bool line = sr.line && !fp64;
    const LineF L = make_line(ax, ay, bx, by, sr.Mx, sr.My);
    SplitLane s;
    s.q0 = lc_none(); s.q1 = lc_none();
    s.c0 = 0; s.c1 = 0;
    s.n_orient_exact = 0u; s.n_cmp_exact = 0u;
    uint32_t n_orient = 0u;
    for (int wp0 = pb + w * (kSRows * 64); wp0 < pe; wp0 += kSTilePairs) {  // as in the seed
        const int p0 = wp0 + lane;
        float4 v[kSRows];
        load_rows(xy, nend, p0, wp0, v);
        // filter-only pass; points needing an exact decision are settled
        // afterwards, out of line (the pass neither counts nor offers them)
        uint32_t pend = 0u;
        if (line) {
#pragma unroll
            for (int r = 0; r < kSRows; ++r) {
                const int id0 = 2 * (p0 + 64 * r);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float x = h ? v[r].z : v[r].x, y = h ? v[r].w : v[r].y;
                    const bool m = id0 + h < nend;
                    const float tt = line_eval(L, x, y);
                    const bool neg = tt < -L.m, pos = tt > L.m;
                    // lower side: the area for A->B is -orient; upper: for B->A it is orient
                    const float ar = neg ? -tt : tt;
                    const float lo = ar - L.m, hi = ar + L.m;
                    const bool lower = m & neg, upper = m & pos;
                    const bool u0 = lc_offer_fast(s.q0, lower, lo, hi, id0 + h, false);
                    const bool u1 = lc_offer_fast(s.q1, upper, lo, hi, id0 + h, false);
                    const bool pd = (m & !neg & !pos) | u0 | u1;
                    s.c0 += (lower & !pd) ? 1 : 0;
                    s.c1 += (upper & !pd) ? 1 : 0;
                    pend |= (uint32_t)pd << (2 * r + h);
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < kSRows; ++r) {
                const int id0 = 2 * (p0 + 64 * r);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float x = h ? v[r].z : v[r].x, y = h ? v[r].w : v[r].y;
                    const bool m = id0 + h < nend;
                    const Orient32 o = orient32p(ax, ay, bx, by, x, y);
                    const int sg = fsign(o, fp64 != 0);
                    const float ar = sg < 0 ? -o.d : o.d, wr = 2.0f * o.es;
                    const float lo = ar - wr, hi = ar + wr;
                    const bool lower = m & (sg < 0), upper = m & (sg > 0);
                    const bool u0 = lc_offer_fast(s.q0, lower, lo, hi, id0 + h, fp64 != 0);
                    const bool u1 = lc_offer_fast(s.q1, upper, lo, hi, id0 + h, fp64 != 0);
                    const bool pd = (m & (sg == 0)) | u0 | u1;
                    s.c0 += (lower & !pd) ? 1 : 0;
                    s.c1 += (upper & !pd) ? 1 : 0;
                    pend |= (uint32_t)pd << (2 * r + h);
                }
            }
        }
        n_orient += lane_points(nend, p0, wp0);
        if (__ballot(pend != 0u)) {
            SplitLane tmp = s;
            split_pending(&tmp, pend, p0, ax, ay, bx, by, xy, fp64);
            s = tmp;
        }
    }
    split_wg_partial(&ws->split[b], s, ax, ay, bx, by, xy, fp64);
    Counters ctr = {n_orient, s.n_orient_exact, s.n_cmp_exact};
    flush_counters(a.stats, ctr);
    if (last_arrival(&ws->done[1], nb)) split_finish(a, ax, ay, bx, by, sr.mni, sr.mxi);
}

// ======================================================== first compaction
// Sections 4.4.2 - 4.4.4 on the two sides: every point of the lower side goes
// to child (A, C_lo) or (C_lo, B), every point of the upper side to (B, C_up)
// or (C_up, A), or is discarded; children are packed into the side's slots
// from the front and the back; the farthest point of each child is found on
// the way (the first pass's section 4.4.1). A tile reserves its children's
// slots with one atomic add per child (no workgroup waits for another, so
// this is an ordinary launch); the order of the points inside a child is
// therefore that of the reservations, which no later step depends on (every
// decision is geometric, with index tie-breaks). The last workgroup to finish
// writes the first pass's segment table.
// The first compaction for one filter mode (LINE: the static line filter).
template <bool LINE>
__device__ __forceinline__ void sfirst_body(const HullArgs& a)
{
    __shared__ int s_wcnt[kSWaves][4];  // per-wave child counts of the current tile
    __shared__ int s_wbase[kSWaves][4]; // ... as offsets inside the tile's reservation
    __shared__ int s_base[4];          // the tile's first rank in each child
    // the tile as each thread loaded it, for the scatter (read back only by
    // the thread that wrote it): held here rather than in registers across
    // the reservation, and rather than read again from memory
    __shared__ float4 s_tile[kSRows][kSBlock];
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int t = (int)threadIdx.x, lane = lane_id(), w = wave_index();
    const int fp64 = a.fp64;
    const int n = a.N;
    // one contiguous range of rows per workgroup; the last tile of a range
    // is partial, and its waves past the end skip it
    int pb, pe;
    wg_range(n, b, nb, pb, pe);
    const int nend = min(n, 2 * pe);  // points of this range: ids below nend
    const float2* xy = a.xy;
    float* X = a.X[0];
    float* Y = a.Y[0];
    int* I = a.I[0];
    auto* ws = static_cast<StreamWs*>(a.sws);
    const SeedPart sr = uni(gld(&ws->seed_res));
    if (sr.bad || (sr.mnx == sr.mxx && sr.mny == sr.mxy)) return;  // finished by the seed
    const SplitPart pr = gld(&ws->split_res);
    const int n_lo = uni(pr.cnt[0]), n_up = uni(pr.cnt[1]);
    if (n_lo == 0 && n_up == 0) return;  // finished by the split
    FirstGeo g;
    g.ax = sr.mnx; g.ay = sr.mny; g.bx = sr.mxx; g.by = sr.mxy;
    g.lx = uni(pr.c[0].x); g.ly = uni(pr.c[0].y); g.ux = uni(pr.c[1].x); g.uy = uni(pr.c[1].y);
    // output slot of rank R in child k: obase[k] + R (k even), obase[k] - R (k odd)
    const int obase[4] = {1, n_lo, 2 + n_lo, 1 + n_lo + n_up};
    LineF L[4];
    L[0] = n_lo > 0 ? make_line(g.ax, g.ay, g.lx, g.ly, sr.Mx, sr.My) : line_never();
    L[1] = n_lo > 0 ? make_line(g.lx, g.ly, g.bx, g.by, sr.Mx, sr.My) : line_never();
    L[2] = n_up > 0 ? make_line(g.bx, g.by, g.ux, g.uy, sr.Mx, sr.My) : line_never();
    L[3] = n_up > 0 ? make_line(g.ux, g.uy, g.ax, g.ay, sr.Mx, sr.My) : line_never();
    using Lane = std::conditional_t<LINE, FirstLineLane, FirstLane>;
    Lane s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if constexpr (LINE) {
            s.q[k].c = -INFINITY;
            s.q[k].id = -1;
        } else {
            s.q[k] = lc_none();
        }
    }
    s.n_orient_exact = 0u;
    s.n_cmp_exact = 0u;
    uint32_t wave_pts = 0u;  // points this wave classified (the same in every lane)
    for (int q = pb; q < pe; q += kSTilePairs) {
        const int wp0 = q + w * (kSRows * 64);  // this wave's first pair
        const int p0 = wp0 + lane;
        const bool live = 2 * wp0 < nend;       // uniform: the wave has points
        s.code_lo = 0x77777777u;
        s.code_hi = 0x77777777u;  // 4 bits per point i = 2 row + h: rows 0-3 / 4-7 (7: none)
        int wc[4] = {0, 0, 0, 0};
        if (live) {
            s.code_lo = 0u;
            s.code_hi = 0u;
            float4 v[kSRows];
            load_rows(xy, nend, p0, wp0, v);
#pragma unroll
            for (int rr = 0; rr < kSRows; ++rr) s_tile[rr][t] = v[rr];
            // filter-only pass; points needing an exact decision are settled
            // afterwards, one at a time
            if constexpr (LINE) {
                const uint32_t pend = first_line_rows(s, v, p0, nend, L);
                wave_pts += (uint32_t)min(nend - 2 * wp0, 2 * 64 * kSRows);
                if (__ballot(pend != 0u)) {
                    Lane tmp = s;
                    first_pending_line(&tmp, pend, p0, g, L, xy);
                    s = tmp;
                }
            } else {
                const uint32_t pend = first_fast_rows(s, v, p0, nend, g, fp64 != 0);
                wave_pts += (uint32_t)min(nend - 2 * wp0, 2 * 64 * kSRows);
                if (__ballot(pend != 0u)) {
                    Lane tmp = s;
                    first_pending(&tmp, pend, p0, g, xy, fp64);
                    s = tmp;
                }
            }
#pragma unroll
            for (int i = 0; i < 2 * kSRows; ++i) {
                const int sh = 4 * (i & 7);
                const int code = (int)(((i < 8) ? s.code_lo : s.code_hi) >> sh) & 15;
#pragma unroll
                for (int k = 0; k < 4; ++k) wc[k] += __popcll(__ballot(code == k));
            }
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 4; ++k) s_wcnt[w][k] = wc[k];
        }
        __syncthreads();
        if (t < 4) {
            // per-wave offsets inside the tile, and the tile's reservation
            int run = 0;
            for (int u = 0; u < kSWaves; ++u) {
                s_wbase[u][t] = run;
                run += s_wcnt[u][t];
            }
            s_base[t] = run > 0 ? (int)atomicAdd(&ws->cursor[t], (unsigned int)run) : 0;
        }
        __syncthreads();
        if (live) {
            // scatter: ranks inside a row from ballots, so that each row
            // writes one contiguous run per child
            float4 v[kSRows];
#pragma unroll
            for (int rr = 0; rr < kSRows; ++rr) v[rr] = s_tile[rr][t];
            int run[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) run[k] = s_base[k] + s_wbase[w][k];
#pragma unroll
            for (int rr = 0; rr < kSRows; ++rr) {
                const int id0 = 2 * (p0 + 64 * rr);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const float x = h ? v[rr].z : v[rr].x, y = h ? v[rr].w : v[rr].y;
                    const int sh = 4 * (2 * (rr & 3) + h);
                    const int code = (int)(((rr < 4) ? s.code_lo : s.code_hi) >> sh) & 15;
                    int dst = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint64_t M = __ballot(code == k);
                        const int rank = run[k] + lanes_below(M);
                        const int d = (k & 1) ? obase[k] - rank : obase[k] + rank;
                        dst = code == k ? d : dst;
                        run[k] += __popcll(M);
                    }
                    if (code < 4) {
                        gst(X + dst, x);
                        gst(Y + dst, y);
                        gst(I + dst, id0 + h);
                    }
                    // one point at a time: keeps the ballots of later points
                    // from being hoisted (their masks would all be live)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
        __syncthreads();
    }
    if constexpr (LINE) {
        // a candidate the filter did not place strictly right of its edge
        // may be no point of the child (the offers were not limited to the
        // child's points): keep it only if the exact test does; then the
        // candidates as intervals [c - m, c + m]
        const float ex[5] = {g.ax, g.lx, g.bx, g.ux, g.ax}, ey[5] = {g.ay, g.ly, g.by, g.uy, g.ay};
        FirstLane f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            int id = s.q[k].id;
            if (id >= 0 && s.q[k].c <= L[k].m) {
                const float2 P = gld(xy + id);
                ++s.n_orient_exact;
                if (orient_exact(ex[k], ey[k], ex[k + 1], ey[k + 1], P.x, P.y) >= 0) id = -1;
            }
            f.q[k].lo = s.q[k].c - L[k].m;
            f.q[k].hi = s.q[k].c + L[k].m;
            f.q[k].id = id;
        }
        first_wg_partial(&ws->first[b], f, g, xy, fp64);
    } else {
        first_wg_partial(&ws->first[b], s, g, xy, fp64);
    }
    const uint32_t n_orient = lane == 0 ? (LINE ? 4u : 3u) * (uint32_t)uni((int)wave_pts) : 0u;
    Counters ctr = {n_orient, s.n_orient_exact, s.n_cmp_exact};
    flush_counters(a.stats, ctr);
    if (last_arrival(&ws->done[2], nb)) {
        const int c0 = (int)ld_flag(reinterpret_cast<const int*>(&ws->cursor[0]));
        const int c1 = (int)ld_flag(reinterpret_cast<const int*>(&ws->cursor[1]));
        const int c2 = (int)ld_flag(reinterpret_cast<const int*>(&ws->cursor[2]));
        const int c3 = (int)ld_flag(reinterpret_cast<const int*>(&ws->cursor[3]));
        first_finish(a, g, n_lo, n_up, pr.c[0].id, pr.c[1].id, c0, c1, c2, c3);
    }
}

// One kernel per filter mode; both are launched, and the one whose mode
// the seed did not choose returns at once (one body per kernel keeps each
// within its register budget).
template <bool LINE>
__global__ __launch_bounds__(kSBlock, 4) void k_sfirst(HullArgs a)
{
    const int line = uni(gld(&reinterpret_cast<const StreamWs*>(a.sws)->seed_res.line));
    if ((line != 0 && !a.fp64) == LINE) sfirst_body<LINE>(a);
}

// ========================================================== streaming pass
// One pass of section 4.4 over a segment table of at most kSPassMaxS
// segments holding at least kSPassMinV points (the first passes of large
// hulls: few segments, millions of points). Tiles of kPTile points never
// straddle segments, so a tile's edges A->C and C->B are uniform; a tile
// reserves its slots in each child with one atomic add (child (A, C) fills
// the parent's slots from the front, (C, B) from the back); a workgroup keeps
// its lanes' farthest candidates while its tiles stay in one segment and
// then reduces them once. The last workgroup to finish writes the next
// segment table. An ordinary launch; when the table does not qualify it
// does nothing, and the passes kernel continues from the same state.
struct SSeg {
    float ax, ay, bx, by, cx, cy;  // A, B and the farthest point C
    int off, len, cid, t0;         // slots, C's index, first tile
};

__device__ __forceinline__ int pass_fast(const SSeg& g, float x, float y, bool valid, bool fp64, float& a, float& w)
{
    const Orient32 o1 = orient32p(g.ax, g.ay, g.cx, g.cy, x, y);  // A -> C
    const Orient32 o2 = orient32p(g.cx, g.cy, g.bx, g.by, x, y);  // C -> B
    const int s1 = fsign(o1, fp64), s2 = fsign(o2, fp64);
    const bool in1 = s1 < 0, in2 = !in1 & (s2 < 0);
    a = -(in1 ? o1.d : o2.d);
    w = 2.0f * (in1 ? o1.es : o2.es);
    const bool und = (s1 == 0) | ((s1 > 0) & (s2 == 0));
    return !valid ? 7 : (und ? 15 : (in1 ? 0 : (in2 ? 1 : 7)));
}

// The same with the line filters of A->C and C->B.
__device__ __forceinline__ int pass_line(const LineF& L0, const LineF& L1, float x, float y, bool valid, float& a,
                                         float& w)
{
    const float t0 = line_eval(L0, x, y), t1 = line_eval(L1, x, y);
    const bool in1 = t0 < -L0.m, pos0 = t0 > L0.m;
    const bool n1 = t1 < -L1.m, p1 = t1 > L1.m;
    const bool in2 = !in1 & pos0 & n1;
    const bool und = !in1 & !(pos0 & (n1 | p1));
    a = in1 ? -t0 : -t1;
    w = in1 ? L0.m : L1.m;
    return !valid ? 7 : (und ? 15 : (in1 ? 0 : (in2 ? 1 : 7)));
}

__device__ __forceinline__ int pass_classify(const SSeg& g, float x, float y, bool fp64, float& a, float& w,
                                             uint32_t& n_exact)
{
    const Orient32 o1 = orient32p(g.ax, g.ay, g.cx, g.cy, x, y);
    const Orient32 o2 = orient32p(g.cx, g.cy, g.bx, g.by, x, y);
    int s1 = fsign(o1, fp64), s2 = fsign(o2, fp64);
    settle_inl(s1, s1 == 0, g.ax, g.ay, g.cx, g.cy, x, y, n_exact);
    settle_inl(s2, (s1 >= 0) & (s2 == 0), g.cx, g.cy, g.bx, g.by, x, y, n_exact);
    const bool in1 = s1 < 0, in2 = !in1 & (s2 < 0);
    a = -(in1 ? o1.d : o2.d);
    w = 2.0f * (in1 ? o1.es : o2.es);
    return in1 ? 0 : (in2 ? 1 : 7);
}

// Workgroup b of nb takes tiles [tile_lo(b), tile_lo(b + 1)) of T; the
// owner of tile j is the last b with tile_lo(b) <= j.
__device__ __forceinline__ int tile_lo(int b, int nb, int T) { return (int)((long long)b * T / nb); }
__device__ __forceinline__ int tile_owner(int j, int nb, int T) { return (int)(((long long)(j + 1) * nb - 1) / T); }

__global__ __launch_bounds__(kSBlock, 4) void k_spass(HullArgs a)
{
    __shared__ SSeg s_seg[kSPassMaxS + 1];
    __shared__ int s_wcnt[kSWaves][2];
    __shared__ int s_wbase[kSWaves][2];
    __shared__ int s_base[2];
    __shared__ Pair s_red[kSWaves];
    // each thread's points of the current tile, for the scatter (read back
    // only by the thread that wrote them)
    __shared__ float s_px[kPRows][kSBlock], s_py[kPRows][kSBlock];
    __shared__ int s_pi[kPRows][kSBlock];
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    const int t = (int)threadIdx.x, lane = lane_id(), w = wave_index();
    const int fp64 = a.fp64;
    auto* ws = static_cast<StreamWs*>(a.sws);
    PassRec* recs = pass_recs(a.sws);
    if (ld_flag(a.err)) return;
    const int cur = ld_flag(&ws->state[0]) & 1, pass = ld_flag(&ws->state[1]), nxt = cur ^ 1;
    const int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
    if (S <= 0 || S > kSPassMaxS || V <= kSPassMinV || pass >= kMaxInfoPasses) return;  // uniform
    const SeedPart sr = uni(gld(&ws->seed_res));
    const bool sline = sr.line && !fp64;
    const float Mx = sr.Mx, My = sr.My;
    // the segment table and each segment's first tile
    {
        SSeg g = {};
        int nt = 0;
        if (t < S) {
            const Seg q = gld(a.segs[cur] + t);
            g.ax = q.ax; g.ay = q.ay; g.bx = q.bx; g.by = q.by; g.cx = q.cx; g.cy = q.cy;
            g.off = q.off; g.len = q.len;
            g.cid = gld(a.seg_cid[cur] + t);
            nt = (q.len + kPTile - 1) / kPTile;
        }
        Pair tot;
        const Pair ex = sblock_excl_scan(Pair{nt, 0}, s_red, &tot);
        if (t < S) {
            g.t0 = ex.a;
            s_seg[t] = g;
        }
        if (t == 0) s_seg[S].t0 = tot.a;
        __syncthreads();
    }
    const int ntiles = s_seg[S].t0;
    const int jlo = tile_lo(b, nb, ntiles), jhi = tile_lo(b + 1, nb, ntiles);
    float* Xo = a.X[nxt];
    float* Yo = a.Y[nxt];
    int* Io = a.I[nxt];
    const float* Xi = a.X[cur];
    const float* Yi = a.Y[cur];
    const int* Ii = a.I[cur];
    LCand q0 = lc_none(), q1 = lc_none();
    uint32_t n_orient = 0u, n_oexact = 0u, n_cexact = 0u;
    int s = 0;  // segment of tile j
    if (jlo < jhi) {
        int lo = 0, hi = S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_seg[mid].t0 <= jlo) lo = mid;
            else hi = mid - 1;
        }
        s = lo;
    }
    int run_j0 = jlo;  // first tile of this workgroup's run in segment s
    for (int j = jlo; j < jhi; ++j) {
        while (s_seg[s + 1].t0 <= j) {
            ++s;
            run_j0 = j;
        }
        const SSeg g = s_seg[s];
        const int q0pos = (j - g.t0) * kPTile + w * (kPRows * 64);  // this wave's first position
        const bool full = q0pos + kPRows * 64 <= g.len;             // uniform per wave
        uint32_t code = 0u;  // 4 bits per row
        {
            float x[kPRows], y[kPRows];
            int id[kPRows];
#pragma unroll
            for (int r = 0; r < kPRows; ++r) {
                const int pos = q0pos + 64 * r + lane;
                const bool m = full | (pos < g.len);
                const int p = g.off + (m ? pos : 0);
                x[r] = gld(Xi + p); y[r] = gld(Yi + p); id[r] = gld(Ii + p);
                s_px[r][t] = x[r]; s_py[r][t] = y[r]; s_pi[r][t] = id[r];
            }
            uint32_t pend = 0u;
            // the line filter where the farthest point's area is large
            // against the line bound of A->B (the areas of the children's
            // points are on that scale; the line bound grows with the
            // input's extent, the orientation filter's with the distances
            // inside the segment, which wins on short, flat segments)
            const float dxs = g.bx - g.ax, dys = g.by - g.ay;
            const float mab = (fabsf(dxs) * My + fabsf(dys) * Mx) * kLineRel;
            const float acb = fabsf(dxs * (g.cy - g.ay) - dys * (g.cx - g.ax));
            const bool line = sline && acb > 1024.0f * mab;
            if (line) {
                const LineF L0 = make_line(g.ax, g.ay, g.cx, g.cy, Mx, My);
                const LineF L1 = make_line(g.cx, g.cy, g.bx, g.by, Mx, My);
#pragma unroll
                for (int r = 0; r < kPRows; ++r) {
                    const bool m = full | (q0pos + 64 * r + lane < g.len);
                    float ar, wr;
                    int c = pass_line(L0, L1, x[r], y[r], m, ar, wr);
                    const float lo2 = ar - wr, hi2 = ar + wr;
                    bool und = c == 15;
                    und |= lc_offer_fast(q0, c == 0, lo2, hi2, id[r], false);
                    und |= lc_offer_fast(q1, c == 1, lo2, hi2, id[r], false);
                    c = und ? 15 : c;
                    pend |= (uint32_t)und << r;
                    n_orient += m ? 2u : 0u;
                    code |= (uint32_t)c << (4 * r);
                }
            } else {
#pragma unroll
                for (int r = 0; r < kPRows; ++r) {
                    const bool m = full | (q0pos + 64 * r + lane < g.len);
                    float ar, wr;
                    int c = pass_fast(g, x[r], y[r], m, fp64 != 0, ar, wr);
                    const float lo2 = ar - wr, hi2 = ar + wr;
                    bool und = c == 15;
                    und |= lc_offer_fast(q0, c == 0, lo2, hi2, id[r], fp64 != 0);
                    und |= lc_offer_fast(q1, c == 1, lo2, hi2, id[r], fp64 != 0);
                    c = und ? 15 : c;
                    pend |= (uint32_t)und << r;
                    n_orient += m ? 2u : 0u;
                    code |= (uint32_t)c << (4 * r);
                }
            }
            if (__ballot(pend != 0u)) {
                const Edge e0 = make_edge(g.ax, g.ay, g.cx, g.cy), e1 = make_edge(g.cx, g.cy, g.bx, g.by);
#pragma unroll 1
                for (int r = 0; r < kPRows; ++r) {
                    const bool mine = (pend >> r) & 1u;
                    if (!__ballot(mine)) continue;
                    if (mine) {
                        const int p = g.off + q0pos + 64 * r + lane;
                        const float px = gld(Xi + p), py = gld(Yi + p);
                        const int pid = gld(Ii + p);
                        float ar, wr;
                        const int c = pass_classify(g, px, py, fp64 != 0, ar, wr, n_oexact);
                        const float lo2 = ar - wr, hi2 = ar + wr;
                        lc_offer(q0, c == 0, lo2, hi2, pid, px, py, e0, a.xy, fp64 != 0, n_cexact);
                        lc_offer(q1, c == 1, lo2, hi2, pid, px, py, e1, a.xy, fp64 != 0, n_cexact);
                        code = (code & ~(15u << (4 * r))) | ((uint32_t)c << (4 * r));
                    }
                }
            }
        }
        int wc0 = 0, wc1 = 0;
#pragma unroll
        for (int r = 0; r < kPRows; ++r) {
            const int c = (int)(code >> (4 * r)) & 15;
            wc0 += __popcll(__ballot(c == 0));
            wc1 += __popcll(__ballot(c == 1));
        }
        if (lane == 0) { s_wcnt[w][0] = wc0; s_wcnt[w][1] = wc1; }
        __syncthreads();
        if (t < 2) {
            int run = 0;
            for (int u = 0; u < kSWaves; ++u) {
                s_wbase[u][t] = run;
                run += s_wcnt[u][t];
            }
            s_base[t] = run > 0 ? (int)atomicAdd(&ws->pcursor[s][t], (unsigned int)run) : 0;
        }
        __syncthreads();
        {
            // scatter (the tile from this thread's LDS copy)
            int run0 = s_base[0] + s_wbase[w][0], run1 = s_base[1] + s_wbase[w][1];
#pragma unroll
            for (int r = 0; r < kPRows; ++r) {
                const int c = (int)(code >> (4 * r)) & 15;
                const uint64_t M0 = __ballot(c == 0), M1 = __ballot(c == 1);
                const int dst = c == 0 ? g.off + run0 + lanes_below(M0) : g.off + g.len - 1 - (run1 + lanes_below(M1));
                if (c < 2) {
                    gst(Xo + dst, s_px[r][t]);
                    gst(Yo + dst, s_py[r][t]);
                    gst(Io + dst, s_pi[r][t]);
                }
                run0 += __popcll(M0);
                run1 += __popcll(M1);
            }
        }
        // the run of tiles in segment s ends here: reduce the candidates once
        if (j + 1 == jhi || s_seg[s + 1].t0 <= j + 1) {
            PassRec rc;
            rc.c[0] = block_max_call(g.ax, g.ay, g.cx, g.cy, lc_full(q0, a.xy), fp64);
            rc.c[1] = block_max_call(g.cx, g.cy, g.bx, g.by, lc_full(q1, a.xy), fp64);
            if (t == 0) gst(recs + run_j0, rc);
            q0 = lc_none();
            q1 = lc_none();
        }
        __syncthreads();
    }
    Counters ctr = {n_orient, n_oexact, n_cexact};
    flush_counters(a.stats, ctr);
    if (!last_arrival(&ws->done[3], nb)) return;
    // ---- the last workgroup: each segment's children (farthest points over
    // the records of the workgroups that took its tiles, counts from the
    // cursors), the vertex key of its farthest point, and the next table
    __shared__ FCand s_c[kSPassMaxS][2];
    __shared__ int s_big[kSPassMaxS];
    __shared__ int s_nbig;
    if (t == 0) s_nbig = 0;
    __syncthreads();
    if (t < S) {
        const SSeg g = s_seg[t];
        const int t1 = s_seg[t + 1].t0;
        const int bl = tile_owner(g.t0, nb, ntiles), bh = tile_owner(t1 - 1, nb, ntiles);
        if (bh - bl < 8) {
            const Edge e0 = make_edge(g.ax, g.ay, g.cx, g.cy), e1 = make_edge(g.cx, g.cy, g.bx, g.by);
            FCand v0 = fc_none(), v1 = fc_none();
            uint32_t nx = 0;
            for (int u = bl; u <= bh; ++u) {
                const PassRec r = gld(recs + max(g.t0, tile_lo(u, nb, ntiles)));
                if (fc_beats(e0, r.c[0], v0, fp64 != 0, nx)) v0 = r.c[0];
                if (fc_beats(e1, r.c[1], v1, fp64 != 0, nx)) v1 = r.c[1];
            }
            s_c[t][0] = v0;
            s_c[t][1] = v1;
        } else {
            s_big[atomicAdd(&s_nbig, 1)] = t;
        }
    }
    __syncthreads();
    for (int i = w; i < s_nbig; i += kSWaves) {
        const int s2 = s_big[i];
        const SSeg g = s_seg[s2];
        const int t1 = s_seg[s2 + 1].t0;
        const int bl = tile_owner(g.t0, nb, ntiles), bh = tile_owner(t1 - 1, nb, ntiles);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const Edge E = k == 0 ? make_edge(g.ax, g.ay, g.cx, g.cy) : make_edge(g.cx, g.cy, g.bx, g.by);
            FCand v = fc_none();
            uint32_t nx = 0;
            for (int u = bl + lane; u <= bh; u += 64) {
                const FCand o = gld(&recs[max(g.t0, tile_lo(u, nb, ntiles))].c[k]);
                if (fc_beats(E, o, v, fp64 != 0, nx)) v = o;
            }
            v = wave_max_fc(E, v, fp64 != 0, nx);
            if (lane == 0) s_c[s2][k] = v;
        }
    }
    __syncthreads();
    int n0 = 0, n1 = 0;
    SSeg g = {};
    if (t < S) {
        g = s_seg[t];
        n0 = (int)ld_flag(reinterpret_cast<const int*>(&ws->pcursor[t][0]));
        n1 = (int)ld_flag(reinterpret_cast<const int*>(&ws->pcursor[t][1]));
    }
    Pair tot;
    const Pair ex = sblock_excl_scan(Pair{(n0 > 0) + (n1 > 0), n0 + n1}, s_red, &tot);
    int2* vl = (a.vcap > 0) ? a.vlist : nullptr;
    if (t < S) {
        // C's key is the first slot after the (A, C) points (section 4.4.2)
        record_vertex(a.bitmap, a.vidx, vl, a.info, g.off + n0, g.cid);
        int k = ex.a, vs = ex.b;
        if (n0 > 0) {
            Seg r;
            r.ax = g.ax; r.ay = g.ay; r.bx = g.cx; r.by = g.cy;
            r.cx = s_c[t][0].x; r.cy = s_c[t][0].y;
            r.off = g.off; r.len = n0;
            gst(a.segs[nxt] + k, r);
            a.seg_cid[nxt][k] = s_c[t][0].id;
            a.vstart[nxt][k] = vs;
            ++k;
            vs += n0;
        }
        if (n1 > 0) {
            Seg r;
            r.ax = g.cx; r.ay = g.cy; r.bx = g.bx; r.by = g.by;
            r.cx = s_c[t][1].x; r.cy = s_c[t][1].y;
            r.off = g.off + g.len - n1; r.len = n1;
            gst(a.segs[nxt] + k, r);
            a.seg_cid[nxt][k] = s_c[t][1].id;
            a.vstart[nxt][k] = vs;
        }
    }
    __syncthreads();  // every thread has read the cursors
    if (t < 2 * kSPassMaxS) (&ws->pcursor[0][0])[t] = 0u;
    if (t == 0) {
        a.vstart[nxt][tot.a] = tot.b;
        a.sv[2 * nxt] = tot.a;
        a.sv[2 * nxt + 1] = tot.b;
        if (pass == 0) a.info->first_v = V;
        a.info->pass_s[pass] = S;
        a.info->pass_v[pass] = V;
        a.info->passes = pass + 1;
        a.info->spass_n = pass + 1;
        ws->state[0] = nxt;
        ws->state[1] = pass + 1;
        ws->done[3] = 0u;
        stamp_here(a, 100 + pass);
    }
}

// ---- the last passes of a large hull, in LDS ------------------------------
//
// Once at most kLPoints points are left (and few enough segments), one
// workgroup copies them into LDS and runs the remaining passes there, six
// points per thread: each point is classified against A->C and C->B of its
// segment (section 4.4.3) and takes its rank in its child from an LDS
// counter; the farthest point of each child (section 4.4.1) is found among
// the points whose area interval reaches the largest lower bound in the
// child, by exact comparison with a leader (the leader steps down when a
// candidate beats it, until none does); a block scan places the children
// (section 4.4.4) and the points move to their child in place (each thread
// holds its points in registers across the move). Slot ranges and vertex
// keys follow the global passes exactly (child (A, C) keeps the front of the
// parent's slots, (C, B) the back, C's key is off + |(A, C)|); inside a child
// the points keep no order.
constexpr int kLPoints = 6144;            // at most this many points ...
constexpr int kLSegs = 1024;              // ... and table entries
constexpr int kLPer = kLPoints / kBlock;  // points per thread
static_assert(kSPassMinV == kLPoints, "the streaming passes stop where the LDS passes can start");
static_assert(kLPoints % kBlock == 0 && kLPoints <= 8192 && kLSegs <= kBlock, "packing and one thread per segment");

struct LSeg {
    float ax, ay, bx, by, cx, cy;  // A, B and the farthest point C
    int off, len, cid, vs;         // slot range, C's index, first point in LDS
};
struct LTail {
    float x[kLPoints], y[kLPoints];
    int id[kLPoints];
    LSeg seg[kLSegs + 1];         // + the sentinel: seg[S].vs = V
    int cnt[2 * kLSegs];          // per (segment, child): its points; bit 31: the leader was beaten
    unsigned key[2 * kLSegs];     // ... the largest lower bound (ordered bits); then the child's first point
    int lead[2 * kLSegs];         // ... the leading candidate (a position)
    float la[2 * kLSegs], lw[2 * kLSegs];  // ... the leader's area interval a +- w
    int any;                      // some leader was beaten in this round
};

// A workgroup barrier that orders LDS accesses only: global stores still in
// flight (counters, vertex records) need not complete first.
__device__ __forceinline__ void lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// block_excl_scan with barriers that order LDS only: a pass of the LDS tail
// does not wait here for its vertex records and counters to reach memory.
__device__ __forceinline__ Pair lds_excl_scan(Pair v, Pair* red, Pair* tot)
{
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    const Pair inc = {wave_incl_sum(v.a), wave_incl_sum(v.b)};
    lds_sync();
    if (lane == 63) red[w] = inc;
    lds_sync();
    Pair off = {0, 0}, all = {0, 0};
#pragma unroll
    for (int u = 0; u < kWaves; ++u) {
        if (u < w) { off.a += red[u].a; off.b += red[u].b; }
        all.a += red[u].a; all.b += red[u].b;
    }
    *tot = all;
    return Pair{off.a + inc.a - v.a, off.b + inc.b - v.b};
}

// float -> unsigned with the same order
__device__ __forceinline__ unsigned okey(float f)
{
    const unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ int lseg_of(const LTail& L, int S, int i)
{
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.seg[mid].vs <= i) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Runs passes `pass`, pass + 1, ... of table `cur` in LDS. Returns false
// when the table outgrew the LDS first: it is then written back (points at
// their slots in buffer `cur`, the table, the pass) for the passes kernel.
__device__ __forceinline__ bool lds_passes(const HullArgs& a, int cur, int pass, LTail& L, Pair* red,
                                           Counters& ctr)
{
    const int t = (int)threadIdx.x;
    const bool f64 = a.fp64 != 0;
    int2* vl = (a.vcap > 0 && a.G == 1) ? a.vlist : nullptr;
    int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
    // the vertex list's length and the stamp count are this workgroup's
    // alone from here: kept locally, so that a pass waits on no global read
    int vcount = ld_flag(&a.info->vcount);
    int nst = ld_flag(&a.info->nstamps);
    for (int u = t; u < S; u += kBlock) {
        const Seg g = gld(a.segs[cur] + u);
        LSeg q;
        q.ax = g.ax; q.ay = g.ay; q.bx = g.bx; q.by = g.by; q.cx = g.cx; q.cy = g.cy;
        q.off = g.off; q.len = g.len;
        q.cid = gld(a.seg_cid[cur] + u);
        q.vs = gld(a.vstart[cur] + u);
        L.seg[u] = q;
    }
    if (t == 0) L.seg[S].vs = V;
    lds_sync();
    for (int i = t; i < V; i += kBlock) {
        const LSeg& q = L.seg[lseg_of(L, S, i)];
        const int p = q.off + (i - q.vs);
        L.x[i] = gld(a.X[cur] + p);
        L.y[i] = gld(a.Y[cur] + p);
        L.id[i] = gld(a.I[cur] + p);
    }
    lds_sync();
    for (;; ++pass) {
        note_pass(a, pass, S, V);
        if (S <= 0) break;
        if (pass >= kMaxInfoPasses || (S > kLSegs / 2 && V > kLSegs)) {
            // hand the table back to the passes kernel
            for (int i = t; i < V; i += kBlock) {
                const LSeg& q = L.seg[lseg_of(L, S, i)];
                const int p = q.off + (i - q.vs);
                gst(a.X[cur] + p, L.x[i]);
                gst(a.Y[cur] + p, L.y[i]);
                gst(a.I[cur] + p, L.id[i]);
            }
            for (int u = t; u < S; u += kBlock) {
                const LSeg q = L.seg[u];
                Seg g;
                g.ax = q.ax; g.ay = q.ay; g.bx = q.bx; g.by = q.by; g.cx = q.cx; g.cy = q.cy;
                g.off = q.off; g.len = q.len;
                gst(a.segs[cur] + u, g);
                a.seg_cid[cur][u] = q.cid;
                a.vstart[cur][u] = q.vs;
            }
            if (t == 0) {
                a.vstart[cur][S] = V;
                a.sv[2 * cur] = S;
                a.sv[2 * cur + 1] = V;
                auto* ws = static_cast<StreamWs*>(a.sws);
                ws->state[0] = cur;
                ws->state[1] = pass;
            }
            return false;
        }
        for (int u = t; u < 2 * S; u += kBlock) {
            L.cnt[u] = 0;
            L.key[u] = 0u;
            L.lead[u] = 0x7fffffff;
        }
        if (t == 0) L.any = 0;
        lds_sync();
        // 1. each point: its child, its rank there, its area interval
        float pa[kLPer], pw[kLPer];
        int pk[kLPer];  // segment << 14 | child << 13 | rank, or -1
#pragma unroll
        for (int r = 0; r < kLPer; ++r) {
            const int i = t + kBlock * r;
            pk[r] = -1;
            pa[r] = 0.0f; pw[r] = 0.0f;
            if (i < V) {
                const int sg = lseg_of(L, S, i);
                const LSeg& q = L.seg[sg];
                const float x = L.x[i], y = L.y[i];
                const Edge e0 = make_edge(q.ax, q.ay, q.cx, q.cy), e1 = make_edge(q.cx, q.cy, q.bx, q.by);
                const Orient32 o1 = orient32(e0, x, y), o2 = orient32(e1, x, y);
                int s1 = fast_sign(o1, f64), s2 = fast_sign(o2, f64);
                settle(s1, s1 == 0, e0, x, y, ctr.orient_exact);
                settle(s2, s1 >= 0 && s2 == 0, e1, x, y, ctr.orient_exact);
                ctr.orient += 2;
                const int k = s1 < 0 ? 0 : (s2 < 0 ? 1 : -1);
                if (k >= 0) {
                    pa[r] = -(k == 0 ? o1.d : o2.d);
                    pw[r] = 2.0f * (k == 0 ? o1.es : o2.es);
                    const int u = 2 * sg + k;
                    const int rank = atomicAdd(&L.cnt[u], 1);
                    atomicMax(&L.key[u], okey(pa[r] - pw[r]));
                    pk[r] = (sg << 14) | (k << 13) | rank;
                }
            }
        }
        lds_sync();
        // 2. the farthest point of each child. Candidates: points whose upper
        // bound reaches the child's largest lower bound (every point in the
        // float64-only mode); the first leader is the lowest position
        // holding that lower bound.
        bool cand[kLPer];
#pragma unroll
        for (int r = 0; r < kLPer; ++r) {
            cand[r] = false;
            if (pk[r] >= 0) {
                const int u = pk[r] >> 13;
                const unsigned kmax = L.key[u];
                const unsigned lo = okey(pa[r] - pw[r]);
                cand[r] = f64 || okey(pa[r] + pw[r]) >= kmax;
                if (lo == kmax) atomicMin(&L.lead[u], t + kBlock * r);
            }
        }
        lds_sync();
#pragma unroll
        for (int r = 0; r < kLPer; ++r) {
            if (cand[r] && L.lead[pk[r] >> 13] == t + kBlock * r) {
                L.la[pk[r] >> 13] = pa[r];
                L.lw[pk[r] >> 13] = pw[r];
            }
        }
        lds_sync();
        for (;;) {
            // every other candidate against the leader
#pragma unroll
            for (int r = 0; r < kLPer; ++r) {
                if (!cand[r]) continue;
                const int u = pk[r] >> 13, i = t + kBlock * r;
                const int l = L.lead[u];
                if (l == i) continue;
                const LSeg& q = L.seg[pk[r] >> 14];
                const Edge E = (u & 1) ? make_edge(q.cx, q.cy, q.bx, q.by) : make_edge(q.ax, q.ay, q.cx, q.cy);
                Cand P, Q;
                P.a = pa[r]; P.w = pw[r]; P.x = L.x[i]; P.y = L.y[i]; P.id = L.id[i];
                Q.a = L.la[u]; Q.w = L.lw[u]; Q.x = L.x[l]; Q.y = L.y[l]; Q.id = L.id[l];
                if (beats(E, P, Q, f64, ctr.cmp_exact)) {
                    atomicOr(&L.cnt[u], (int)0x80000000u);
                    L.any = 1;
                } else {
                    cand[r] = false;
                }
            }
            lds_sync();
            if (!L.any) break;  // (uniform)
            // a beaten leader steps down; its challengers elect the lowest position
#pragma unroll
            for (int r = 0; r < kLPer; ++r)
                if (cand[r] && L.cnt[pk[r] >> 13] < 0 && L.lead[pk[r] >> 13] == t + kBlock * r) cand[r] = false;
            lds_sync();
            for (int u = t; u < 2 * S; u += kBlock)
                if (L.cnt[u] < 0) L.lead[u] = 0x7fffffff;
            lds_sync();
#pragma unroll
            for (int r = 0; r < kLPer; ++r)
                if (cand[r] && L.cnt[pk[r] >> 13] < 0) atomicMin(&L.lead[pk[r] >> 13], t + kBlock * r);
            lds_sync();
#pragma unroll
            for (int r = 0; r < kLPer; ++r) {
                if (cand[r] && L.cnt[pk[r] >> 13] < 0 && L.lead[pk[r] >> 13] == t + kBlock * r) {
                    L.la[pk[r] >> 13] = pa[r];
                    L.lw[pk[r] >> 13] = pw[r];
                }
            }
            lds_sync();
            for (int u = t; u < 2 * S; u += kBlock) L.cnt[u] &= 0x7fffffff;
            if (t == 0) L.any = 0;
            lds_sync();
        }
        // 3. the children of segment t, C's vertex key, the next table
        LSeg mine = {};
        int n0 = 0, n1 = 0;
        LSeg ch0 = {}, ch1 = {};
        if (t < S) {
            mine = L.seg[t];
            n0 = L.cnt[2 * t];
            n1 = L.cnt[2 * t + 1];
        }
        Pair tot;
        const Pair ex = lds_excl_scan(Pair{n0 + n1, (n0 > 0) + (n1 > 0)}, red, &tot);
        if (t < S) {
            // C is a vertex: its key is the first slot after the (A, C) points
            const int key = mine.off + n0;
            atomicOr((unsigned long long*)&a.bitmap[key >> 6], 1ull << (key & 63));
            gst(a.vidx + key, mine.cid);
            if (vl && vcount + t < a.vcap) vl[vcount + t] = make_int2(key, mine.cid);
            if (n0 > 0) {
                const int l = L.lead[2 * t];
                ch0.ax = mine.ax; ch0.ay = mine.ay; ch0.bx = mine.cx; ch0.by = mine.cy;
                ch0.cx = L.x[l]; ch0.cy = L.y[l]; ch0.cid = L.id[l];
                ch0.off = mine.off; ch0.len = n0; ch0.vs = ex.a;
            }
            if (n1 > 0) {
                const int l = L.lead[2 * t + 1];
                ch1.ax = mine.cx; ch1.ay = mine.cy; ch1.bx = mine.bx; ch1.by = mine.by;
                ch1.cx = L.x[l]; ch1.cy = L.y[l]; ch1.cid = L.id[l];
                ch1.off = mine.off + mine.len - n1; ch1.len = n1; ch1.vs = ex.a + n0;
            }
        }
        lds_sync();  // every read of the table and of the leaders is done
        if (t < S) {
            int j = ex.b;
            if (n0 > 0) L.seg[j++] = ch0;
            if (n1 > 0) L.seg[j] = ch1;
            L.key[2 * t] = (unsigned)ex.a;
            L.key[2 * t + 1] = (unsigned)(ex.a + n0);
        }
        if (t == 0) L.seg[tot.b].vs = tot.a;
        lds_sync();
        // 4. every kept point to its child, in place: each thread reads its
        // points, then (after the barrier) writes them
        float px[kLPer], py[kLPer];
        int pid[kLPer], dst[kLPer];
#pragma unroll
        for (int r = 0; r < kLPer; ++r) {
            const int i = t + kBlock * r;
            dst[r] = -1;
            px[r] = 0.0f; py[r] = 0.0f; pid[r] = 0;
            if (pk[r] >= 0) {
                px[r] = L.x[i]; py[r] = L.y[i]; pid[r] = L.id[i];
                dst[r] = (int)L.key[pk[r] >> 13] + (pk[r] & 0x1fff);
            }
        }
        lds_sync();
#pragma unroll
        for (int r = 0; r < kLPer; ++r) {
            if (dst[r] < 0) continue;
            L.x[dst[r]] = px[r];
            L.y[dst[r]] = py[r];
            L.id[dst[r]] = pid[r];
        }
        lds_sync();
        vcount += S;
        if (t == 0) {
            a.info->vcount = vcount;
            if (a.timing && nst < kMaxStamps) {
                a.info->stamp[nst] = wall_clock64();
                a.info->stamp_tag[nst] = 100 + pass;
                a.info->nstamps = ++nst;
            }
        }
        S = tot.b;
        V = tot.a;
    }
    if (t == 0) {
        a.sv[2 * cur] = 0;
        a.sv[2 * cur + 1] = 0;
        auto* ws = static_cast<StreamWs*>(a.sws);
        ws->state[0] = cur;
        ws->state[1] = pass;
    }
    return true;
}

// The streaming path's last kernel (one workgroup, an ordinary launch): once
// at most kTinyPoints points are left, the remaining passes in LDS (the
// passes kernel's own tail) and the ordered emission of the vertex list.
// Leaves info->stream_done = 1 when the hull is complete; otherwise (more
// points left, or a vertex list too long for one workgroup) the passes
// kernel continues from the state left in the workspace.
__global__ __launch_bounds__(kBlock) void k_stail(HullArgs a)
{
    static_assert(sizeof(LTail) >= sizeof(int2) * kSmallHull, "the emission reuses the passes' LDS");
    __shared__ LTail lds;
    __shared__ Pair red[kWaves];
    auto* ws = static_cast<StreamWs*>(a.sws);
    Counters ctr = {0u, 0u, 0u};
    if (ld_flag(a.err)) return;
    const int cur = ld_flag(&ws->state[0]) & 1, pass = ld_flag(&ws->state[1]);
    const int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
    // left to the passes kernel: too many points, or a table that could outgrow the LDS
    if (S > 0 && (V > kLPoints || (S > kLSegs / 2 && V > kLSegs) || pass >= kMaxInfoPasses)) return;
    if (S > 0) {
        const bool done = lds_passes(a, cur, pass, lds, red, ctr);
        flush_counters(a.stats, ctr);
        if (!done) return;
    } else if (threadIdx.x == 0) {
        note_pass(a, pass, 0, 0);
    }
    __syncthreads();
    const int h = ld_flag(&a.info->vcount);
    if (!(h <= kSmallHull && h <= a.vcap)) return;  // the grid emission in the passes kernel
    emit_small(a, h, reinterpret_cast<int2*>(&lds));
    if (threadIdx.x == 0) {
        a.info->stream_done = 1;
        stamp(a, 4);
    }
}

}  // namespace sqh
