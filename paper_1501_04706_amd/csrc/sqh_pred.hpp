// Exact geometric predicates for float32 points (device code, gfx950).
//
// The paper's kernels compute point-to-line distances and side tests in
// plain float (section 4, Table 1 "float dist[n]"). Here every side test and
// every farthest-point comparison is exact, so the hull does not depend on
// rounding: a float32 evaluation with a proven error bound decides almost
// all cases and an exact float64 expansion decides the rest.
//
// Build with -ffp-contract=off: the bounds below assume that every
// operation is rounded separately and that nothing is reassociated.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sqh {

// Loads and stores through pointers that live in structs lose their address
// space and compile to FLAT instructions; these casts keep them GLOBAL.
// Structs move as 16-, 8- or 4-byte words (clang vector types have no user
// constructors, so they copy across address spaces).
#define SQH_GLOBAL __attribute__((address_space(1)))
typedef unsigned int sqh_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int sqh_u32x2 __attribute__((ext_vector_type(2)));

template <class W, class T>
__device__ __forceinline__ T gld_words(const T* p)
{
    constexpr int n = (int)(sizeof(T) / sizeof(W));
    const SQH_GLOBAL W* q = (const SQH_GLOBAL W*)p;
    W w[n];
#pragma unroll
    for (int i = 0; i < n; ++i) w[i] = q[i];
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}
template <class W, class T>
__device__ __forceinline__ void gst_words(T* p, const T& v)
{
    constexpr int n = (int)(sizeof(T) / sizeof(W));
    W w[n];
    __builtin_memcpy(w, &v, sizeof(T));
    SQH_GLOBAL W* q = (SQH_GLOBAL W*)p;
#pragma unroll
    for (int i = 0; i < n; ++i) q[i] = w[i];
}
template <class T>
__device__ __forceinline__ T gld(const T* p)
{
    if constexpr (__is_arithmetic(T)) return *(const SQH_GLOBAL T*)p;
    else if constexpr (sizeof(T) % 16 == 0) return gld_words<sqh_u32x4>(p);
    else if constexpr (sizeof(T) % 8 == 0) return gld_words<sqh_u32x2>(p);
    else return gld_words<unsigned int>(p);
}
template <class T>
__device__ __forceinline__ void gst(T* p, const T& v)
{
    if constexpr (__is_arithmetic(T)) *(SQH_GLOBAL T*)p = v;
    else if constexpr (sizeof(T) % 16 == 0) gst_words<sqh_u32x4>(p, v);
    else if constexpr (sizeof(T) % 8 == 0) gst_words<sqh_u32x2>(p, v);
    else gst_words<unsigned int>(p, v);
}

// Orientation of p against the directed edge o -> e:
//   orient = (ex - ox) * (py - oy) - (ey - oy) * (px - ox)
// > 0: p left of o->e;  < 0: p right of o->e (outside a counter-clockwise
// hull edge);  0: collinear.
struct Edge {
    float ox, oy, ex, ey;  // end points
    float dx, dy;          // fl(ex - ox), fl(ey - oy)
    int fwd;               // 1 if e is lexicographically after o
};

__device__ __forceinline__ Edge make_edge(float ox, float oy, float ex, float ey)
{
    Edge E;
    E.ox = ox; E.oy = oy; E.ex = ex; E.ey = ey;
    E.dx = ex - ox; E.dy = ey - oy;
    E.fwd = (ex > ox) || (ex == ox && ey > oy);
    return E;
}

// ---- float32 filter -------------------------------------------------------
//
// With u = 2^-24, a1 = py-oy, b1 = px-ox (each rounded once, |delta| <= u;
// a difference that lands in the subnormal range is exact), P = fl(dx*a1),
// Q = fl(dy*b1) (relative error u plus an absolute underflow term
// eta <= 2^-150 each) and d = fl(P - Q):
//   |(P - Q) - orient| <= ((1+u)^3 - 1)/(1-u)^3 * (|P| + |Q|) + 2.0001 eta
//                       <= 3.0001 u S + 2.0001 eta,       S = |P| + |Q|.
// fl(P - Q) has the sign of P - Q, and |P - Q| >= |d| / (1 + u). Hence with
//   es = fl(fl(2^-22 * fl(S)) + TAU),   TAU = 2^-140 (>> 4 eta),
// |d| > es proves sign(d) == sign(orient):  es/(1+u) >= 3.9999 u S + 0.9999
// TAU exceeds the error bound (the rounding of fl(S) and of the sum are
// inside the margin). The same es also bounds the error of d itself:
//   |d - orient| <= 4.0002 u S + 2.0001 eta <= 2 es,
// so [d - 2es, d + 2es] encloses the exact orientation; the farthest-point
// comparison uses that interval. Any overflow makes S or d non-finite and
// the comparisons below false, which routes the case to the exact path.
constexpr float kFilterScale = 0x1p-22f;
constexpr float kFilterTau = 0x1p-140f;

struct Orient32 {
    float d;   // fl(orient)
    float es;  // sign certificate bound; 2*es bounds |d - orient|
};

__device__ __forceinline__ Orient32 orient32(const Edge& E, float px, float py)
{
    float a1 = py - E.oy;
    float b1 = px - E.ox;
    float P = E.dx * a1;
    float Q = E.dy * b1;
    Orient32 r;
    r.d = P - Q;
    float S = fabsf(P) + fabsf(Q);
    r.es = S * kFilterScale + kFilterTau;
    return r;
}

// The same for the edge o -> e given by its end points (no edge record).
__device__ __forceinline__ Orient32 orient32p(float ox, float oy, float ex, float ey, float px, float py)
{
    const float dx = ex - ox, dy = ey - oy;
    float a1 = py - oy;
    float b1 = px - ox;
    float P = dx * a1;
    float Q = dy * b1;
    Orient32 r;
    r.d = P - Q;
    float S = fabsf(P) + fabsf(Q);
    r.es = S * kFilterScale + kFilterTau;
    return r;
}

// ---- exact float64 path ---------------------------------------------------
//
// The product of two float32 values is exact in float64 (24+24 significand
// bits; exponents stay inside the normal float64 range), so orient is an
// exact sum of six float64 terms. Its sign is the sign of the most
// significant nonzero component of the nonoverlapping expansion built with
// Knuth's TwoSum and Shewchuk's Grow-Expansion (J. R. Shewchuk, "Adaptive
// Precision Floating-Point Arithmetic and Fast Robust Geometric Predicates",
// 1997). Every partial sum is a multiple of 2^-298, so TwoSum never
// underflows.

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    e = (a - av) + (b - bv);
    s = x;
}

template <int K>
__device__ __forceinline__ int expansion_sign(const double (&t)[K])
{
    double e[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double q = t[i];
#pragma unroll
        for (int j = 0; j < i; ++j) {
            double s, h;
            two_sum(q, e[j], s, h);
            e[j] = h;
            q = s;
        }
        e[i] = q;
    }
    int sg = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) sg = e[j] > 0.0 ? 1 : (e[j] < 0.0 ? -1 : sg);
    return sg;
}

// float64 stage. With float32 inputs, each difference fl64(q - o) has a
// relative error of at most u = 2^-53, the products neither underflow (a
// nonzero product is >= 2^-298) nor overflow, so t1 = fl(a1 a2) and
// t2 = fl(b1 b2) are each within (3u + 4u^2)|t| of the exact product, and
// the final subtraction adds at most u(|t1| + |t2|). Hence
//   |fl(t1 - t2) - orient| <= (4u + 4u^2)(|t1| + |t2|),
// and the constant below (4u scaled by 1 + 2^-10) also covers the rounding of
// the bound's own evaluation. |D| > bound certifies sign(D), and
// [D - bound, D + bound] encloses the exact orientation.
constexpr double kD64Rel = 4.4453e-16;  // 4 * 2^-53 * (1 + 2^-10) = 4.445229e-16, rounded up

__device__ __forceinline__ double orient64(float ox, float oy, float ex, float ey, float px, float py, double& bound)
{
    const double a1 = (double)ex - (double)ox, a2 = (double)py - (double)oy;
    const double b1 = (double)ey - (double)oy, b2 = (double)px - (double)ox;
    const double t1 = a1 * a2, t2 = b1 * b2;
    bound = kD64Rel * (fabs(t1) + fabs(t2));
    return t1 - t2;
}

// sign of orient(o, e, p), exactly: float64 stage, then the 6-term expansion
//   ex*py - ex*oy - ox*py - ey*px + ey*ox + oy*px
// (the _inl form is for code that must not contain calls)
__device__ __forceinline__ int orient_exact_inl(float ox, float oy, float ex, float ey, float px, float py)
{
    double bound;
    const double d = orient64(ox, oy, ex, ey, px, py, bound);
    if (d > bound) return 1;
    if (-d > bound) return -1;
    double t[6];
    t[0] = (double)ex * (double)py;
    t[1] = -((double)ex * (double)oy);
    t[2] = -((double)ox * (double)py);
    t[3] = -((double)ey * (double)px);
    t[4] = (double)ey * (double)ox;
    t[5] = (double)oy * (double)px;
    return expansion_sign(t);
}
__device__ __noinline__ int orient_exact(float ox, float oy, float ex, float ey, float px, float py)
{
    return orient_exact_inl(ox, oy, ex, ey, px, py);
}

// sign of area(P) - area(Q) for the edge o -> e, where area(X) = -orient(o,e,X):
// float64 stage (areas with their bounds; fl(x) > fl(y) implies x > y), then
//   (ex-ox)(qy-py) - (ey-oy)(qx-px)
//   = ex*qy - ex*py - ox*qy + ox*py - ey*qx + ey*px + oy*qx - oy*px
__device__ __forceinline__ int area_cmp_exact_inl(float ox, float oy, float ex, float ey,
                                                  float px, float py, float qx, float qy)
{
    double bp, bq;
    const double ap = -orient64(ox, oy, ex, ey, px, py, bp);
    const double aq = -orient64(ox, oy, ex, ey, qx, qy, bq);
    if (ap - bp > aq + bq) return 1;
    if (aq - bq > ap + bp) return -1;
    double t[8];
    t[0] = (double)ex * (double)qy;
    t[1] = -((double)ex * (double)py);
    t[2] = -((double)ox * (double)qy);
    t[3] = (double)ox * (double)py;
    t[4] = -((double)ey * (double)qx);
    t[5] = (double)ey * (double)px;
    t[6] = (double)oy * (double)qx;
    t[7] = -((double)oy * (double)px);
    return expansion_sign(t);
}
__device__ __noinline__ int area_cmp_exact(float ox, float oy, float ex, float ey,
                                           float px, float py, float qx, float qy)
{
    return area_cmp_exact_inl(ox, oy, ex, ey, px, py, qx, qy);
}

// Filter-only sign: +-1 when certified, 0 when undecided (the exact sign may
// be 0 or not). `fp64_only` leaves every case undecided.
__device__ __forceinline__ int fast_sign(const Orient32& o, bool fp64_only)
{
    const bool ok = !fp64_only && fabsf(o.d) > o.es;
    return ok ? (o.d > 0.0f ? 1 : -1) : 0;
}

// Settles undecided signs with the exact path; the exact code runs only if
// some lane of the wave needs it.
__device__ __forceinline__ void settle(int& s, bool need, const Edge& E, float px, float py, uint32_t& n_exact)
{
    if (__ballot(need)) {
        if (need) {
            s = orient_exact(E.ox, E.oy, E.ex, E.ey, px, py);
            ++n_exact;
        }
    }
}

// settle() for the edge o -> e given by its end points
__device__ __forceinline__ void settle_p(int& s, bool need, float ox, float oy, float ex, float ey, float px,
                                         float py, uint32_t& n_exact)
{
    if (__ballot(need)) {
        if (need) {
            s = orient_exact(ox, oy, ex, ey, px, py);
            ++n_exact;
        }
    }
}

// Exact sign of orient(o, e, p), filtered. `fp64_only` skips the filter.
// Also returns the float32 estimate for the farthest-point interval.
__device__ __forceinline__ int orient_sign(const Edge& E, float px, float py, bool fp64_only,
                                           Orient32& o, uint32_t& n_exact)
{
    o = orient32(E, px, py);
    if (!fp64_only && fabsf(o.d) > o.es) return o.d > 0.0f ? 1 : -1;
    ++n_exact;
    return orient_exact(E.ox, E.oy, E.ex, E.ey, px, py);
}

// ---- farthest-point candidates ---------------------------------------------
//
// A candidate is a point strictly right of its segment's edge. `a` is the
// float32 estimate of its area -orient (positive), `w` a bound on the
// estimate's error, `id` its input index (-1: no candidate).
struct Cand {
    float a, w;
    float x, y;
    int id;
};

__device__ __forceinline__ Cand no_cand()
{
    Cand c;
    c.a = 0.0f; c.w = 0.0f; c.x = 0.0f; c.y = 0.0f; c.id = -1;
    return c;
}

// Total order "P is farther from the edge than Q" (section 4.4.1 finds the
// farthest point; the paper does not say how ties are broken). Exact area
// first; among points at equal area (they lie on one line parallel to the
// edge) the one earliest along o -> e wins -- an end point of that run and
// hence a hull vertex; coincident points: the lowest index. A total order
// makes the reduction result independent of the reduction tree.
__device__ __forceinline__ bool beats(const Edge& E, const Cand& P, const Cand& Q, bool fp64_only,
                                      uint32_t& n_exact)
{
    if (Q.id < 0) return P.id >= 0;
    if (P.id < 0) return false;
    if (!fp64_only) {
        // fl(x) > fl(y) implies x > y (rounding is monotone), so these
        // certify area(P) >= P.a - P.w > Q.a + Q.w >= area(Q).
        if (P.a - P.w > Q.a + Q.w) return true;
        if (Q.a - Q.w > P.a + P.w) return false;
    }
    ++n_exact;
    int s = area_cmp_exact(E.ox, E.oy, E.ex, E.ey, P.x, P.y, Q.x, Q.y);
    if (s != 0) return s > 0;
    if (P.x == Q.x && P.y == Q.y) return P.id < Q.id;
    bool p_first = (P.x < Q.x) || (P.x == Q.x && P.y < Q.y);
    return E.fwd ? p_first : !p_first;
}

// Farthest-point comparison without the exact path: 1 if P certainly beats
// Q, 0 if it certainly does not, -1 if undecided.
__device__ __forceinline__ int beats_fast(const Cand& P, const Cand& Q, bool fp64_only)
{
    const bool qn = Q.id < 0, pn = P.id < 0;
    const bool win = P.a - P.w > Q.a + Q.w;
    const bool lose = Q.a - Q.w > P.a + P.w;
    int r = (fp64_only || !(win || lose)) ? -1 : (win ? 1 : 0);
    r = pn ? 0 : r;
    r = qn ? (pn ? 0 : 1) : r;
    return r;
}

// Candidate for a point known to be strictly right of E (orient < 0).
__device__ __forceinline__ Cand make_cand(const Orient32& o, float x, float y, int id)
{
    Cand c;
    c.a = -o.d;
    c.w = 2.0f * o.es;
    c.x = x; c.y = y; c.id = id;
    return c;
}

}  // namespace sqh
