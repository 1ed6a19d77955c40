// Segmented tile processing with single-pass decoupled look-back (device code).
//
// Every phase of the method is a pass over a position space [0, P) that is
// cut into contiguous groups: the point sets of a batch for the seed and the
// first split, the segments for the passes (paper section 2: segments are
// contiguous partitions kept by head flags / keys). Each point is classified
// into at most one of NB buckets (the two sides of the first split, the two
// child segments of a pass); per group and bucket the pass needs
//   * the number of points (section 4.4.4's stable partition needs ranks),
//   * the farthest point (section 4.4.1's segmented reduction).
//
// A tile of kWaves * ROWS * 64 consecutive positions is processed by one
// workgroup; each wave owns ROWS rows of 64 consecutive positions. A wave
// whose range lies inside one group (the common case) counts with ballots
// and keeps a private farthest candidate per lane; a wave that crosses group
// boundaries uses head flags, ballot ranks and a segmented shuffle scan per
// row. Waves are combined in LDS, and a group that started in an earlier
// tile gets its prefix (counts and running farthest point) from the
// preceding tiles through decoupled look-back on 64-bit status words that
// carry both the flag and the value, so no memory fence is needed. The last
// tile that holds a group's end has its complete aggregate and finalises it.
//
// Forward progress: tiles are assigned statically, tile t to workgroup
// t mod gridDim, and the grid is launched cooperatively (all workgroups
// resident), so the lowest unfinished tile is always running. Every spin is
// bounded; on timeout the kernel raises an error flag and continues.
#pragma once
#include "sqh_pred.hpp"

namespace sqh {

constexpr int kWaves = 4;
constexpr int kBlock = kWaves * 64;
constexpr int kSpinLimit = 1 << 22;
constexpr int kNone = -1;

// error flags (device status word)
constexpr int kErrNonFinite = 1;
constexpr int kErrSpin = 2;
constexpr int kErrBounds = 4;

// stats slots: [kStatSlots][4]: orient evals, orient exact, cmp exact, spare
constexpr int kStatSlots = 64;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }
__device__ __forceinline__ uint64_t mask_lt(int l) { return (1ull << l) - 1ull; }
__device__ __forceinline__ uint64_t mask_le(int l) { return l >= 63 ? ~0ull : ((2ull << l) - 1ull); }
// bits [lo, hi], 0 <= lo, hi <= 63; empty if hi < lo
__device__ __forceinline__ uint64_t mask_range(int lo, int hi)
{
    return hi < lo ? 0ull : (mask_le(hi) & ~mask_lt(lo));
}

// ---- status words: bit 62 = valid, bits [31,62) = hi, bits [0,31) = lo ----
__device__ __forceinline__ uint64_t pack2(uint32_t hi, uint32_t lo)
{
    return (1ull << 62) | ((uint64_t)(hi & 0x7fffffffu) << 31) | (uint64_t)(lo & 0x7fffffffu);
}
__device__ __forceinline__ bool word_ok(uint64_t w) { return (w >> 62) == 1ull; }
__device__ __forceinline__ uint32_t word_hi(uint64_t w) { return (uint32_t)(w >> 31) & 0x7fffffffu; }
__device__ __forceinline__ uint32_t word_lo(uint64_t w) { return (uint32_t)w & 0x7fffffffu; }
__device__ __forceinline__ uint64_t ld_word(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_word(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- cross-lane moves of candidates ----
__device__ __forceinline__ Cand shfl_xor_cand(const Cand& c, int m)
{
    Cand r;
    r.a = __shfl_xor(c.a, m); r.w = __shfl_xor(c.w, m);
    r.x = __shfl_xor(c.x, m); r.y = __shfl_xor(c.y, m);
    r.id = __shfl_xor(c.id, m); r.pos = __shfl_xor(c.pos, m);
    return r;
}
__device__ __forceinline__ Cand shfl_up_cand(const Cand& c, int d)
{
    Cand r;
    r.a = __shfl_up(c.a, d); r.w = __shfl_up(c.w, d);
    r.x = __shfl_up(c.x, d); r.y = __shfl_up(c.y, d);
    r.id = __shfl_up(c.id, d); r.pos = __shfl_up(c.pos, d);
    return r;
}
__device__ __forceinline__ float rl_f(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int rl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ Cand readlane_cand(const Cand& c, int l)
{
    Cand r;
    r.a = rl_f(c.a, l); r.w = rl_f(c.w, l); r.x = rl_f(c.x, l); r.y = rl_f(c.y, l);
    r.id = rl_i(c.id, l); r.pos = rl_i(c.pos, l);
    return r;
}

// Per-thread counters, flushed once per tile.
struct Counters {
    uint32_t orient, orient_exact, cmp_exact;
};

template <int NB>
struct Agg {
    int cnt[NB];
    Cand best[NB];
};

template <int NB>
__device__ __forceinline__ void agg_clear(Agg<NB>& a)
{
#pragma unroll
    for (int k = 0; k < NB; ++k) { a.cnt[k] = 0; a.best[k] = no_cand(); }
}

template <int NB>
__device__ __forceinline__ Agg<NB> readlane_agg(const Agg<NB>& a, int l)
{
    Agg<NB> r;
#pragma unroll
    for (int k = 0; k < NB; ++k) { r.cnt[k] = rl_i(a.cnt[k], l); r.best[k] = readlane_cand(a.best[k], l); }
    return r;
}

// a <- a (+) b  for group context c
template <class Pol>
__device__ __forceinline__ void agg_add(const Pol& pol, const typename Pol::Ctx& c, Agg<Pol::NB>& a,
                                        const Agg<Pol::NB>& b, Counters& ctr)
{
#pragma unroll
    for (int k = 0; k < Pol::NB; ++k) {
        a.cnt[k] += b.cnt[k];
        if (pol.beats(c, k, b.best[k], a.best[k], ctr)) a.best[k] = b.best[k];
    }
}

// wave-wide reduction of one candidate per lane (all lanes end with the max)
template <class Pol>
__device__ __forceinline__ Cand wave_max(const Pol& pol, const typename Pol::Ctx& c, int k, Cand v, Counters& ctr)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        Cand o = shfl_xor_cand(v, m);
        // the order is total, so both lanes of a pair pick the same winner
        if (pol.beats(c, k, o, v, ctr)) v = o;
    }
    return v;
}

// number of status words for a policy
template <class Pol>
struct LB {
    static constexpr int NC = Pol::COUNTS ? (Pol::NB + 1) / 2 : 0;  // count words
    static constexpr int NP = (Pol::NB + 1) / 2;                    // position words
    static constexpr int NW = NC + NP;
};

template <class Pol>
__device__ __forceinline__ void agg_to_words(const Agg<Pol::NB>& a, uint64_t* w)
{
    constexpr int NB = Pol::NB;
    int i = 0;
    if constexpr (Pol::COUNTS) {
#pragma unroll
        for (int k = 0; k < NB; k += 2) w[i++] = pack2(a.cnt[k], k + 1 < NB ? a.cnt[k + 1] : 0);
    }
#pragma unroll
    for (int k = 0; k < NB; k += 2)
        w[i++] = pack2((uint32_t)(a.best[k].pos + 1), k + 1 < NB ? (uint32_t)(a.best[k + 1].pos + 1) : 0u);
}

template <class Pol>
__device__ __forceinline__ void words_to_agg(const Pol& pol, const typename Pol::Ctx& c, const uint64_t* w,
                                             Agg<Pol::NB>& a, Counters& ctr)
{
    constexpr int NB = Pol::NB;
    int i = 0;
    if constexpr (Pol::COUNTS) {
#pragma unroll
        for (int k = 0; k < NB; k += 2) {
            a.cnt[k] = (int)word_hi(w[i]);
            if (k + 1 < NB) a.cnt[k + 1] = (int)word_lo(w[i]);
            ++i;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NB; ++k) a.cnt[k] = 0;
    }
#pragma unroll
    for (int k = 0; k < NB; k += 2) {
        int p0 = (int)word_hi(w[i]) - 1;
        a.best[k] = p0 >= 0 ? pol.fetch_cand(c, k, p0, ctr) : no_cand();
        if (k + 1 < NB) {
            int p1 = (int)word_lo(w[i]) - 1;
            a.best[k + 1] = p1 >= 0 ? pol.fetch_cand(c, k + 1, p1, ctr) : no_cand();
        }
        ++i;
    }
}

// Decoupled look-back for tile t, executed by one whole wave. Returns the
// aggregate of group g over tiles [start tile of g, t). Status layout per
// tile: [agg words NW][inc words NW].
template <class Pol>
__device__ Agg<Pol::NB> look_back(const Pol& pol, const typename Pol::Ctx& c, const uint64_t* lb, int t,
                                  int* err, Counters& ctr)
{
    constexpr int NW = LB<Pol>::NW;
    const int lane = lane_id();
    Agg<Pol::NB> acc;
    agg_clear(acc);
    int base = t - 1;
    int spins = 0;
    while (true) {
        const int j = base - lane;
        uint64_t w[NW];
        bool inc_ok = false, agg_ok = false;
        if (j >= 0) {
            const uint64_t* s = lb + (size_t)j * (2 * NW);
            inc_ok = true;
#pragma unroll
            for (int i = 0; i < NW; ++i) { w[i] = ld_word(s + NW + i); inc_ok &= word_ok(w[i]); }
            if (!inc_ok) {
                agg_ok = true;
#pragma unroll
                for (int i = 0; i < NW; ++i) { w[i] = ld_word(s + i); agg_ok &= word_ok(w[i]); }
            }
        }
        const uint64_t incm = __ballot(inc_ok);
        const uint64_t rdym = __ballot(inc_ok || agg_ok);
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
        Agg<Pol::NB> mine;
        agg_clear(mine);
        if (lane <= first_inc && j >= 0) words_to_agg(pol, c, w, mine, ctr);
        // reduce the window's contributions
#pragma unroll
        for (int k = 0; k < Pol::NB; ++k) {
            int s = mine.cnt[k];
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m);
            acc.cnt[k] += s;
            Cand b = wave_max(pol, c, k, mine.best[k], ctr);
            if (pol.beats(c, k, b, acc.best[k], ctr)) acc.best[k] = b;
        }
        if (first_inc < 64) break;
        base -= 64;
    }
    return acc;
}

template <class Pol>
__device__ __forceinline__ void publish(uint64_t* lb, int t, bool inclusive, const Agg<Pol::NB>& a)
{
    constexpr int NW = LB<Pol>::NW;
    uint64_t w[NW];
    agg_to_words<Pol>(a, w);
    uint64_t* s = lb + (size_t)t * (2 * NW) + (inclusive ? NW : 0);
#pragma unroll
    for (int i = 0; i < NW; ++i) st_word(s + i, w[i]);
}

template <class Pol>
struct TileShared {
    int gf, gl;
    int gf_before;  // gf started before this tile
    int wgf[kWaves], wgl[kWaves], wflag[kWaves];  // wflag: 0 empty, 1 crossing, 2 one group
    Agg<Pol::NB> first[kWaves], last[kWaves];
    Agg<Pol::NB> pref[kWaves];
    Agg<Pol::NB> tile_cin;
    int code[kWaves][Pol::ROWS * 64];  // per-position codes of waves that cross groups
};

// Flush per-thread counters (one atomic per wave and counter).
__device__ __forceinline__ void flush_counters(uint32_t* stats, Counters& ctr)
{
    uint32_t v[3] = {ctr.orient, ctr.orient_exact, ctr.cmp_exact};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        uint32_t s = v[i];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) s += __shfl_xor(s, m);
        if (lane_id() == 0 && s) atomicAdd(&stats[(blockIdx.x % kStatSlots) * 4 + i], s);
    }
    ctr.orient = ctr.orient_exact = ctr.cmp_exact = 0;
}

// Process one tile. Pol supplies:
//   NB, COUNTS, SCATTER, MULTI, ROWS, struct Ctx
//   int  group_of(int q, int lo, int hi)         largest g in [lo,hi] with start(g) <= q
//   int  group_start(int g), group_end(int g)
//   Ctx  ctx(int g)
//   void load(const Ctx&, int g, int q, float& x, float& y, int& id)
//   int  classify(const Ctx&, int g, int q, float x, float y, int id, Cand& c, Counters&)
//            -> bucket or kNone (MULTI: bit mask of buckets, same candidate)
//   bool beats(const Ctx&, int k, const Cand& P, const Cand& Q, Counters&)
//   Cand fetch_cand(const Ctx&, int k, int pos, Counters&)
//   int  place(const Ctx&, int g, int k, int rank)       (SCATTER)
//   void store(int dst, float x, float y, int id)        (SCATTER)
//   void finalize(const Ctx&, int g, const Agg<NB>&)
template <class Pol>
__device__ void process_tile(Pol& pol, int t, int P, int G, uint64_t* lb, int* err, TileShared<Pol>& sh,
                             Counters& ctr)
{
    constexpr int NB = Pol::NB;
    constexpr int R = Pol::ROWS;
    constexpr int WR = R * 64;
    constexpr int T = WR * kWaves;
    using Ctx = typename Pol::Ctx;

    const int lane = lane_id();
    const int w = (int)(threadIdx.x >> 6);
    const int q0 = t * T;
    const int q1 = min(q0 + T, P);

    if (threadIdx.x == 0) {
        int gf = pol.group_of(q0, 0, G - 1);
        int gl = pol.group_of(q1 - 1, gf, G - 1);
        sh.gf = gf;
        sh.gl = gl;
        sh.gf_before = pol.group_start(gf) < q0;
    }
    __syncthreads();
    const int gf = sh.gf, gl = sh.gl;

    const int wq0 = q0 + w * WR;
    const int wq1 = min(wq0 + WR, q1);
    const bool wempty = wq0 >= wq1;
    int wgf = gf, wgl = gf;
    if (!wempty) {
        wgf = pol.group_of(wq0, gf, gl);
        wgl = pol.group_of(wq1 - 1, wgf, gl);
    }
    const bool one_group = (wgf == wgl);

    float px[R], py[R];
    int pid[R], code[R];  // code: (g - wgf) << 16 | rank << 3 | bucket, or kNone
    Agg<NB> first, last;
    agg_clear(first);
    agg_clear(last);

    if (!wempty && one_group) {
        // ---------------- one group in this wave ----------------
        const Ctx c = pol.ctx(wgf);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = wq0 + r * 64 + lane;
            if (q < wq1) pol.load(c, wgf, q, px[r], py[r], pid[r]);
        }
        int run[NB];
        Cand pb[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) { run[k] = 0; pb[k] = no_cand(); }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int q = wq0 + r * 64 + lane;
            Cand cand;
            int b = kNone;
            if (q < wq1) b = pol.classify(c, wgf, q, px[r], py[r], pid[r], cand, ctr);
            code[r] = kNone;
            if constexpr (Pol::MULTI) {
#pragma unroll
                for (int k = 0; k < NB; ++k)
                    if (b != kNone && ((b >> k) & 1) && pol.beats(c, k, cand, pb[k], ctr)) pb[k] = cand;
            } else {
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const uint64_t M = __ballot(b == k);
                    if (b == k) {
                        code[r] = ((run[k] + __popcll(M & mask_lt(lane))) << 3) | k;
                        if (pol.beats(c, k, cand, pb[k], ctr)) pb[k] = cand;
                    }
                    run[k] += __popcll(M);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            first.cnt[k] = Pol::COUNTS ? run[k] : 0;
            first.best[k] = wave_max(pol, c, k, pb[k], ctr);
        }
        last = first;
    } else if (!wempty) {
        // ---------------- several groups in this wave ----------------
        int carry_g = -1;
        Agg<NB> carry;
        agg_clear(carry);
        bool have_first = false;
        int prev_g = wgf;
#pragma unroll 1
        for (int r = 0; r < R; ++r) {
            const int rowbase = wq0 + r * 64;
            if (rowbase >= wq1) { sh.code[w][r * 64 + lane] = kNone; continue; }
            const int q = rowbase + lane;
            const bool valid = q < wq1;
            const int g = valid ? pol.group_of(q, prev_g, wgl) : 0x7fffffff;
            if (valid) prev_g = g;
            const int L = min(63, wq1 - 1 - rowbase);  // last valid lane of the row
            Ctx c;
            Cand cand;
            int b = kNone;
            if (valid) {
                float x, y;
                int id;
                c = pol.ctx(g);
                pol.load(c, g, q, x, y, id);
                b = pol.classify(c, g, q, x, y, id, cand, ctr);
            }
            // the carried group ended exactly at the previous row's end
            const int g0 = rl_i(g, 0);
            if (carry_g >= 0 && g0 != carry_g) {
                if (carry_g == wgf) {
                    first = carry;
                    have_first = true;
                } else if (lane == 0) {
                    const Ctx cc = pol.ctx(carry_g);
                    pol.finalize(cc, carry_g, carry);
                }
                carry_g = -1;
                agg_clear(carry);
            }
            // runs of equal group across lanes
            const int gup = __shfl_up(g, 1);
            const bool head = (lane == 0) || (g != gup);
            const uint64_t H = __ballot(head);
            const int s = 63 - __clzll(H & mask_le(lane));
            const uint64_t above = H & ~mask_le(lane);
            const int e = above ? (__ffsll((unsigned long long)above) - 2) : 63;
            const uint64_t runm = mask_range(s, e);
            const bool cont = valid && (g == carry_g);  // lanes of the row's first run only
            Agg<NB> tot;
            int rank = 0;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                if constexpr (Pol::MULTI) {
                    tot.cnt[k] = 0;
                } else {
                    const uint64_t M = __ballot(valid && b == k);
                    const int add = cont ? carry.cnt[k] : 0;
                    if (b == k) rank = __popcll(M & runm & mask_lt(lane)) + add;
                    tot.cnt[k] = Pol::COUNTS ? __popcll(M & runm) + add : 0;
                }
                // segmented inclusive max-scan of candidates within the run
                Cand x = no_cand();
                if constexpr (Pol::MULTI) {
                    if (b != kNone && ((b >> k) & 1)) x = cand;
                } else {
                    if (b == k) x = cand;
                }
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const Cand y = shfl_up_cand(x, d);
                    if (lane - d >= s && valid && pol.beats(c, k, y, x, ctr)) x = y;
                }
                if (cont && pol.beats(c, k, carry.best[k], x, ctr)) x = carry.best[k];
                tot.best[k] = x;
            }
            int cd = kNone;
            if constexpr (!Pol::MULTI) cd = (valid && b != kNone) ? (((g - wgf) << 16) | (rank << 3) | b) : kNone;
            sh.code[w][r * 64 + lane] = cd;

            // runs that end inside the row are complete within this wave
            const bool leader = valid && lane == e;
            const bool continues = (e >= L);
            const uint64_t firstm = __ballot(leader && !continues && g == wgf);
            if (firstm) {
                first = readlane_agg(tot, __ffsll((unsigned long long)firstm) - 1);
                have_first = true;
            }
            if (leader && !continues && g != wgf) pol.finalize(c, g, tot);
            // the run holding the row's last valid lane carries on
            carry_g = rl_i(g, L);
            carry = readlane_agg(tot, L);
        }
        (void)have_first;
        last = carry;  // group wgl, started inside this wave
    }

    // ---------------- combine the waves of the tile ----------------
    if (lane == 0) {
        sh.wgf[w] = wgf;
        sh.wgl[w] = wgl;
        sh.wflag[w] = wempty ? 0 : (one_group ? 2 : 1);
        sh.first[w] = first;
        sh.last[w] = last;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // in-tile prefix of each wave's first group from the waves before it
        for (int v = 0; v < kWaves; ++v) {
            Agg<NB> cin;
            agg_clear(cin);
            if (sh.wflag[v]) {
                const int g = sh.wgf[v];
                const Ctx c = pol.ctx(g);
                for (int u = v - 1; u >= 0; --u) {
                    if (!sh.wflag[u] || sh.wgl[u] != g) break;
                    agg_add(pol, c, cin, sh.last[u], ctr);
                    if (sh.wgf[u] != g) break;
                }
            }
            sh.pref[v] = cin;
        }
    }
    __syncthreads();
    if (w == 0) {
        // aggregate of the tile's last group inside this tile
        int vl = kWaves - 1;
        while (vl > 0 && !sh.wflag[vl]) --vl;
        Agg<NB> tagg = sh.pref[vl];
        {
            const Ctx c = pol.ctx(gl);
            if (sh.wgf[vl] == gl) {
                agg_add(pol, c, tagg, sh.first[vl], ctr);  // wave vl holds gl from its start
            } else {
                agg_clear(tagg);
                tagg = sh.last[vl];
            }
        }
        const bool gl_inside = pol.group_start(gl) >= q0;
        if (gl_inside) {
            if (lane == 0) publish<Pol>(lb, t, true, tagg);
        } else if (gl == gf) {
            if (lane == 0) publish<Pol>(lb, t, false, tagg);
        }
        Agg<NB> cin;
        agg_clear(cin);
        if (sh.gf_before) {
            const Ctx c = pol.ctx(gf);
            cin = look_back(pol, c, lb, t, err, ctr);
            if (gl == gf) {
                Agg<NB> inc = cin;
                agg_add(pol, c, inc, tagg, ctr);
                if (lane == 0) publish<Pol>(lb, t, true, inc);
            }
        }
        if (lane == 0) sh.tile_cin = cin;
    }
    __syncthreads();

    // ---------------- finalise and scatter ----------------
    if (!wempty) {
        Agg<NB> pref = sh.pref[w];
        if (wgf == gf && sh.gf_before) {
            const Ctx c = pol.ctx(gf);
            agg_add(pol, c, pref, sh.tile_cin, ctr);
        }
        if (lane == 0) {
            if (one_group) {
                if (pol.group_end(wgf) <= wq1) {
                    const Ctx c = pol.ctx(wgf);
                    Agg<NB> tot = pref;
                    agg_add(pol, c, tot, first, ctr);
                    pol.finalize(c, wgf, tot);
                }
            } else {
                {
                    const Ctx c = pol.ctx(wgf);
                    Agg<NB> tot = pref;
                    agg_add(pol, c, tot, first, ctr);
                    pol.finalize(c, wgf, tot);
                }
                if (pol.group_end(wgl) <= wq1) {
                    const Ctx c = pol.ctx(wgl);
                    pol.finalize(c, wgl, last);
                }
            }
        }
        if constexpr (Pol::SCATTER) {
            if (one_group) {
                const Ctx c = pol.ctx(wgf);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if (code[r] != kNone) {
                        const int k = code[r] & 7;
                        const int rank = ((code[r] >> 3) & 0x1fff) + pref.cnt[k];
                        pol.store(pol.place(c, wgf, k, rank), px[r], py[r], pid[r]);
                    }
                }
            } else {
#pragma unroll 1
                for (int r = 0; r < R; ++r) {
                    const int cd = sh.code[w][r * 64 + lane];
                    if (cd != kNone) {
                        const int k = cd & 7;
                        const int goff = cd >> 16;
                        const int g = wgf + goff;
                        int rank = (cd >> 3) & 0x1fff;
                        if (goff == 0) rank += pref.cnt[k];
                        const Ctx c = pol.ctx(g);
                        float x, y;
                        int id;
                        pol.load(c, g, wq0 + r * 64 + lane, x, y, id);
                        pol.store(pol.place(c, g, k, rank), x, y, id);
                    }
                }
            }
        }
    }
    __syncthreads();
}

}  // namespace sqh
