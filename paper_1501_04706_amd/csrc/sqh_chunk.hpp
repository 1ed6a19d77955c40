// Segmented chunk processing for the persistent hull kernel (device code).
//
// Every phase of the method is a pass over a position space [0, P) cut into
// contiguous groups: the point sets of a batch for the seed and the first
// split, the segments for the passes (paper section 2: segments are
// contiguous partitions kept by head flags / keys). Each point falls into at
// most one of NB buckets (the sides of the first split, the two child
// segments of a pass); per group and bucket a pass needs
//   * the number of points and each point's rank (section 4.4.4's stable
//     partition), and
//   * the farthest point (section 4.4.1's segmented reduction).
//
// The persistent grid gives workgroup b one contiguous chunk of positions,
// and each of its waves one contiguous part of the chunk. A phase runs in up
// to three steps separated by grid barriers (reduce-then-scan):
//   A  every wave streams its part 64 positions (one row) at a time, ROWS
//      rows per batch while the batch stays inside one group; it keeps the
//      running counts of the current group and one private farthest
//      candidate per lane, and reduces them across the wave only when the
//      group ends. Groups that start and end inside the part are finalised
//      on the spot. One thread then chains the four parts of the chunk, and
//      the aggregate of the group running past the chunk's end is published;
//   B  the workgroup adds up the published aggregates of the chunks before
//      it that belong to its first group (the count prefix), and the
//      workgroup holding a group's end finalises it;
//   C  every wave streams its part again from its count prefix and writes
//      each point to its rank in its child segment.
// A row that crosses a group boundary uses head flags, ballot ranks and a
// segmented shuffle scan of the candidates.
#pragma once
#include "sqh_pred.hpp"

namespace sqh {

constexpr int kWaves = 16;  // one 1024-thread workgroup per compute unit
constexpr int kBlock = kWaves * 64;
constexpr int kSpinLimit = 1 << 22;
constexpr int kNone = -1;

// error flags (device status word)
constexpr int kErrNonFinite = 1;
constexpr int kErrSpin = 2;
constexpr int kErrBounds = 4;

// stats slots: [kStatSlots][4]: orient evals, orient exact, cmp exact, spare
constexpr int kStatSlots = 64;

enum { kModeAgg = 0, kModeScatter = 1 };

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

// Wave-wide inclusive prefix sum with DPP moves (every lane active): adds
// within each 16-lane row from 1, 2, 4 and 8 lanes back (lanes with no
// source add 0), then row 0's total into row 1 and row 2's into row 3
// (row_bcast:15), then the total of rows 0-1 into rows 2 and 3
// (row_bcast:31). Lane 63 ends with the wave's total.
__device__ __forceinline__ int wave_incl_sum(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}
// The wave's total, in every lane (scalar).
__device__ __forceinline__ int wave_total(int v) { return __builtin_amdgcn_readlane(wave_incl_sum(v), 63); }
__device__ __forceinline__ uint64_t mask_lt(int l) { return (1ull << l) - 1ull; }
__device__ __forceinline__ uint64_t mask_le(int l) { return l >= 63 ? ~0ull : ((2ull << l) - 1ull); }
// bits [lo, hi], 0 <= lo, hi <= 63; empty if hi < lo
__device__ __forceinline__ uint64_t mask_range(int lo, int hi)
{
    return hi < lo ? 0ull : (mask_le(hi) & ~mask_lt(lo));
}

// ---- cross-lane moves of candidates ----
__device__ __forceinline__ Cand shfl_xor_cand(const Cand& c, int m)
{
    Cand r;
    r.a = __shfl_xor(c.a, m); r.w = __shfl_xor(c.w, m);
    r.x = __shfl_xor(c.x, m); r.y = __shfl_xor(c.y, m);
    r.id = __shfl_xor(c.id, m);
    return r;
}
__device__ __forceinline__ Cand shfl_up_cand(const Cand& c, int d)
{
    Cand r;
    r.a = __shfl_up(c.a, d); r.w = __shfl_up(c.w, d);
    r.x = __shfl_up(c.x, d); r.y = __shfl_up(c.y, d);
    r.id = __shfl_up(c.id, d);
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
    r.id = rl_i(c.id, l);
    return r;
}

// Per-thread counters, flushed once at the end of the kernel.
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

// a <- a (+) b for group context c; with WITH_BEST false only counts add
template <class Pol, bool WITH_BEST>
__device__ __forceinline__ void agg_add(const Pol& pol, const typename Pol::Ctx& c, Agg<Pol::NB>& a,
                                        const Agg<Pol::NB>& b, Counters& ctr)
{
#pragma unroll
    for (int k = 0; k < Pol::NB; ++k) {
        a.cnt[k] += b.cnt[k];
        if constexpr (WITH_BEST) {
            if (pol.beats(c, k, b.best[k], a.best[k], ctr)) a.best[k] = b.best[k];
        }
    }
}

// wave-wide reduction of one candidate per lane (all lanes end with the max)
template <class Pol>
__device__ __forceinline__ Cand wave_max(const Pol& pol, const typename Pol::Ctx& c, int k, Cand v, Counters& ctr)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const Cand o = shfl_xor_cand(v, m);
        // the order is total, so both lanes of a pair pick the same winner
        if (pol.beats(c, k, o, v, ctr)) v = o;
    }
    return v;
}

// Published per chunk after step A.
template <int NB>
struct ChunkSlot {
    int last_g;        // group running past the chunk's end (-1: none)
    int first_g;       // group holding the chunk's first position
    int first_before;  // ... which started before the chunk
    int first_done;    // ... and ended inside it
    int tab_a, tab_b;  // active child segments / their points, of groups finalised in step A
    int pad[2];
    Agg<NB> last;      // aggregate of last_g inside the chunk
    Agg<NB> first;     // first_done: aggregate of first_g inside the chunk
};

template <class Pol>
struct ChunkShared {
    // per-wave results of step A (kept until step C)
    int wfirst_g[kWaves], wfirst_before[kWaves], wfirst_done[kWaves], wlast_g[kWaves], wempty[kWaves];
    Agg<Pol::NB> wfirst_total[kWaves], wlast[kWaves];
    int wpref[kWaves][Pol::NB];  // count prefix of each wave's first group from earlier waves
    // chunk level
    int first_done;            // the chunk's first group started before it and ended inside
    Agg<Pol::NB> first_total;  // ... its aggregate inside the chunk
    int carry_g;               // A: group running past the chunk end; B: first group's count prefix
    Agg<Pol::NB> carry;
    Agg<Pol::NB> red[kWaves];  // block reductions
};

__device__ __forceinline__ void flush_counters(uint32_t* stats, Counters& ctr)
{
    const uint32_t v[3] = {ctr.orient, ctr.orient_exact, ctr.cmp_exact};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const uint32_t s = (uint32_t)wave_total((int)v[i]);
        if (lane_id() == 0 && s) atomicAdd(&stats[(blockIdx.x % kStatSlots) * 4 + i], s);
    }
    ctr.orient = ctr.orient_exact = ctr.cmp_exact = 0;
}

// Pol supplies:
//   NB, COUNTS, SCATTER, MULTI, ROWS, struct Ctx
//   int  num_groups()
//   int  group_of(int q, int lo, int hi)   largest g in [lo,hi] with start(g) <= q
//   int  group_start(int g), group_end(int g)
//   Ctx  ctx(int g)
//   void load(const Ctx&, int g, int q, float& x, float& y, int& id)
//   int  classify(const Ctx&, int g, int q, float x, float y, int id, Cand& c, Counters&)
//            -> bucket or kNone (MULTI: bit mask of buckets, same candidate)
//   bool beats(const Ctx&, int k, const Cand& P, const Cand& Q, Counters&)
//   int  place(const Ctx&, int g, int k, int rank)       (SCATTER)
//   void store(int dst, float x, float y, int id)        (SCATTER)
//   void finalize(const Ctx&, int g, const Agg<NB>&)

// Points of one row inside one group: ballot counts / ranks, private
// candidates (MODE kModeAgg) or scatter (kModeScatter).
template <class Pol, int MODE>
__device__ __forceinline__ void row_one_group(const Pol& pol, const typename Pol::Ctx& c, int g, int q, bool valid,
                                              float x, float y, int id, int (&cnt)[Pol::NB], Cand (&pb)[Pol::NB],
                                              Counters& ctr)
{
    constexpr int NB = Pol::NB;
    const int lane = lane_id();
    Cand cand;
    int b = kNone;
    if (valid) b = pol.classify(c, g, q, x, y, id, cand, ctr);
    if constexpr (Pol::MULTI) {
        if constexpr (MODE == kModeAgg) {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                const bool mine = b != kNone && ((b >> k) & 1);
                if (mine && pol.beats_fast(c, k, cand, pb[k]) > 0) pb[k] = cand;
            }
        }
    } else {
        int rank = 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const uint64_t M = __ballot(b == k);
            rank = b == k ? cnt[k] + __popcll(M & mask_lt(lane)) : rank;
            if constexpr (MODE == kModeAgg) {
                // the exact comparison runs only if some lane cannot decide
                int r = b == k ? pol.beats_fast(c, k, cand, pb[k]) : 0;
                if (__ballot(r < 0)) {
                    if (r < 0) r = pol.beats(c, k, cand, pb[k], ctr) ? 1 : 0;
                }
                if (r > 0) pb[k] = cand;
            }
            cnt[k] += __popcll(M);
        }
        if constexpr (MODE == kModeScatter && Pol::SCATTER) {
            if (b != kNone) pol.store(pol.place(c, g, b, rank), x, y, id);
        }
    }
}

// Groups g, g+1, ... that start at or after qs and end at or before re,
// inside the row [q, re) of one wave (qs > q, and g ends before re): every
// lane takes its own group's context; ranks come from the ballot of its
// bucket masked to its group's lanes, and the farthest point of each group
// and bucket from a segmented inclusive shuffle scan, whose last lane
// finalises the group. Needs non-empty groups (at most 63 then start inside
// a row, so the starts of g .. g+63 give every end). On return qs is the end
// of the last such group and g, ge, c describe the group holding it, or
// open is false if the wave's part ends there.
template <class Pol, int MODE>
__device__ __forceinline__ void middle_groups(const Pol& pol, int q, int& qs, int re, int we, int& g, int& ge,
                                              typename Pol::Ctx& c, bool& open, Counters& ctr)
{
    constexpr int NB = Pol::NB;
    using Ctx = typename Pol::Ctx;
    const int lane = lane_id();
    const int G = pol.num_groups();
    // starts of groups g + lane; group_start(G) is the end of the last group
    const int stl = (g + lane <= G) ? pol.group_start(g + lane) : 0x7fffffff;
    const int m = __popcll(__ballot(lane >= 1 && stl <= re));  // groups ending at or before re
    const int emid = rl_i(stl, m);
    const int pos = q + lane;
    const bool in_mid = pos >= qs && pos < emid;
    // this lane's group: the largest j < m with start(g + j) <= pos
    int j = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const int t = j + step;
        const int st = __shfl(stl, t & 63);
        if (t < m && st <= pos) j = t;
    }
    const int gs_l = __shfl(stl, j), ge_l = __shfl(stl, j + 1);
    const int gl = g + j;
    const Ctx cl = pol.ctx(gl);
    float x = 0.0f, y = 0.0f;
    int id = 0;
    Cand cand;
    int bk = kNone;
    if (in_mid) {
        pol.load(cl, gl, pos, x, y, id);
        bk = pol.classify(cl, gl, pos, x, y, id, cand, ctr);
    }
    const int lo = gs_l - q;  // first lane of this lane's group
    const uint64_t gm = mask_range(lo, ge_l - q - 1);
    Agg<NB> tot;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const uint64_t M = __ballot(bk == k);
        tot.cnt[k] = __popcll(M & gm);
        if constexpr (MODE == kModeScatter && Pol::SCATTER) {
            if (bk == k) pol.store(pol.place(cl, gl, k, __popcll(M & gm & mask_lt(lane))), x, y, id);
        }
        if constexpr (MODE == kModeAgg) {
            Cand v = bk == k ? cand : no_cand();
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const Cand o = shfl_up_cand(v, d);
                if (lane - d >= lo && pol.beats(cl, k, o, v, ctr)) v = o;
            }
            tot.best[k] = v;
        }
    }
    if constexpr (MODE == kModeAgg) {
        if (in_mid && pos == ge_l - 1) pol.finalize(cl, gl, tot);
    }
    qs = emid;
    g += m;
    if (emid >= we) {
        open = false;
    } else {
        ge = pol.group_end(g);
        c = pol.ctx(g);
    }
}

// One wave streams [wb, we), a part of chunk [cb, ..) whose groups are
// glo..ghi. kModeAgg: finalises groups that start and end inside the part,
// records the part's first group if it started before wb and ends inside
// (wfirst_*) and the aggregate of the group running past we (wlast_*;
// wlast_g = -1 if a group ends exactly at we). kModeScatter: writes every
// point to its rank, starting from the count prefix init_cnt of the part's
// first group.
//
// A row that crosses group boundaries is processed run by run: the lanes of
// one group at a time, with that group's (wave-uniform) context.
template <class Pol, int MODE>
__device__ __forceinline__ void process_wave(const Pol& pol, int wb, int we, int glo, int ghi, const int* init_cnt,
                             ChunkShared<Pol>& sh, Counters& ctr)
{
    constexpr int NB = Pol::NB;
    constexpr int R = Pol::ROWS;
    constexpr bool AGG = (MODE == kModeAgg);
    using Ctx = typename Pol::Ctx;
    const int lane = lane_id();
    const int w = (int)(threadIdx.x >> 6);

    int g = pol.group_of(wb, glo, ghi);
    int ge = pol.group_end(g);
    bool first_open = pol.group_start(g) < wb;
    bool open = true;
    if constexpr (AGG) {
        if (lane == 0) {
            sh.wfirst_g[w] = g;
            sh.wfirst_before[w] = first_open ? 1 : 0;
        }
    }
    Ctx c = pol.ctx(g);
    int cnt[NB];
    Cand pb[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) { cnt[k] = init_cnt ? init_cnt[k] : 0; pb[k] = no_cand(); }

    // group g ended at ge: finalise it, or hand it to the block if it started
    // before this part; then move to the next group (if inside the part)
    auto end_group = [&](void) {
        // the next group holding position ge: with non-empty groups its loads
        // are issued before this group's reduction and finalisation
        const bool more = ge < we;
        int g2 = g, ge2 = ge;
        Ctx c2 = c;
        if constexpr (Pol::MIDDLE) {
            if (more) {
                g2 = g + 1;
                ge2 = pol.group_end(g2);
                c2 = pol.ctx(g2);
            }
        }
        if constexpr (AGG) {
            Agg<NB> tot;
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                tot.cnt[k] = Pol::COUNTS ? cnt[k] : 0;
                tot.best[k] = wave_max(pol, c, k, pb[k], ctr);
            }
            if (lane == 0) {
                if (first_open) {
                    sh.wfirst_total[w] = tot;
                    sh.wfirst_done[w] = 1;
                } else {
                    pol.finalize(c, g, tot);
                }
            }
        }
        if constexpr (!Pol::MIDDLE) {
            if (more) {
                // skipping empty groups
                const int q0 = ge;
                g2 = g + 1;
                ge2 = pol.group_end(g2);
                while (ge2 <= q0) ge2 = pol.group_end(++g2);
                c2 = pol.ctx(g2);
            }
        }
        if (more) {
            g = g2;
            ge = ge2;
            c = c2;
        } else {
            open = false;
        }
        first_open = false;
#pragma unroll
        for (int k = 0; k < NB; ++k) { cnt[k] = 0; pb[k] = no_cand(); }
    };

    int q = wb;
    while (q < we) {
        if (q + 64 * R <= min(ge, we)) {
            // R full rows inside group g: issue all loads first
            float px[R], py[R];
            int pid[R];
#pragma unroll
            for (int r = 0; r < R; ++r) pol.load(c, g, q + 64 * r + lane, px[r], py[r], pid[r]);
#pragma unroll
            for (int r = 0; r < R; ++r)
                row_one_group<Pol, MODE>(pol, c, g, q + 64 * r + lane, true, px[r], py[r], pid[r], cnt, pb, ctr);
            q += 64 * R;
            if (q == ge) end_group();
            continue;
        }
        // one row [q, re), run by run
        const int re = min(q + 64, we);
        const int pos = q + lane;
        int qs = q;  // start of the current run
        while (true) {
            const int run_end = min(ge, re);
            const bool in_run = pos >= qs && pos < run_end;
            float x = 0.0f, y = 0.0f;
            int id = 0;
            if (in_run) pol.load(c, g, pos, x, y, id);
            row_one_group<Pol, MODE>(pol, c, g, pos, in_run, x, y, id, cnt, pb, ctr);
            if (ge > re) break;  // g goes on past this row
            qs = ge;
            end_group();
            if (!open || qs >= re) break;
            if constexpr (Pol::MIDDLE) {
                if (ge < re) middle_groups<Pol, MODE>(pol, q, qs, re, we, g, ge, c, open, ctr);
                if (!open || qs >= re) break;
            }
        }
        q = re;
    }
    if constexpr (AGG) {
        Agg<NB> last;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            last.cnt[k] = Pol::COUNTS ? cnt[k] : 0;
            last.best[k] = open ? wave_max(pol, c, k, pb[k], ctr) : no_cand();
        }
        if (lane == 0) {
            sh.wlast_g[w] = open ? g : -1;
            sh.wlast[w] = last;
        }
    }
}

// The waves of a workgroup split chunk [cb, ce) into contiguous parts.
__device__ __forceinline__ void wave_part(int cb, int ce, int w, int& wb, int& we)
{
    const int rows = (ce - cb + 63) / 64;
    const int per = (rows + kWaves - 1) / kWaves;
    wb = min(cb + w * per * 64, ce);
    we = min(wb + per * 64, ce);
}

// Walk chunk [cb, ce) (groups glo..ghi). kModeAgg: counts and farthest
// points; groups that start and end inside the chunk are finalised; the
// aggregate of the group running past ce is left in sh.carry(_g), and the
// chunk's first group, if it started before cb and ends inside, in
// sh.first_total. kModeScatter: ranks and scatter, starting from the count
// prefix in sh.carry (set by chunk_step_b).
template <class Pol, int MODE>
__device__ __forceinline__ void process_chunk(const Pol& pol, int cb, int ce, int glo, int ghi, ChunkShared<Pol>& sh,
                              Counters& ctr)
{
    constexpr int NB = Pol::NB;
    using Ctx = typename Pol::Ctx;
    const int lane = lane_id();
    const int w = (int)(threadIdx.x >> 6);
    int wb, we;
    wave_part(cb, ce, w, wb, we);
    if constexpr (MODE == kModeAgg) {
        if (lane == 0) {
            sh.wfirst_done[w] = 0;
            sh.wempty[w] = wb >= we;
        }
        if (wb < we) process_wave<Pol, MODE>(pol, wb, we, glo, ghi, nullptr, sh, ctr);
        __syncthreads();
        if (w == 0) {
            // Chain the parts, one lane per wave (active waves are a prefix).
            // R[v], the aggregate of the group running out of part v, is a
            // segmented inclusive scan: R[v] = R[v-1] (+) wlast[v] when part v
            // lies inside the group running into it, else wlast[v]. The count
            // prefix of part v's first group is R[v-1].
            const int v = lane;
            const bool act = v < kWaves && !sh.wempty[v];
            int g0 = -1, lg = -1;
            bool fb = false, fd = false;
            if (act) {
                g0 = sh.wfirst_g[v];
                fb = sh.wfirst_before[v] != 0;
                fd = sh.wfirst_done[v] != 0;
                lg = sh.wlast_g[v];
            }
            const bool cont = act && v > 0 && fb && !fd && lg == g0;
            const bool use_pre = act && fb && v > 0;
            const int last_act = 63 - __clzll(__ballot(act));
            {
                const Ctx cs = pol.ctx(act && lg >= 0 ? lg : glo);
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    int cnt = 0;
                    Cand best = no_cand();
                    if (act && lg >= 0) {
                        cnt = Pol::COUNTS ? sh.wlast[v].cnt[k] : 0;
                        best = sh.wlast[v].best[k];
                    }
                    bool flag = !cont;
#pragma unroll
                    for (int d = 1; d < kWaves; d <<= 1) {
                        const int oc = __shfl_up(cnt, d);
                        const Cand ob = shfl_up_cand(best, d);
                        const int of = __shfl_up(flag ? 1 : 0, d);
                        if (v >= d && !flag) {
                            cnt += oc;
                            if (pol.beats(cs, k, ob, best, ctr)) best = ob;
                            flag = of != 0;
                        }
                    }
                    const int pc = __shfl_up(cnt, 1);
                    const Cand pb_ = shfl_up_cand(best, 1);
                    if (act) {
                        sh.wpref[v][k] = use_pre ? pc : 0;
                        sh.red[v].cnt[k] = use_pre ? pc : 0;
                        sh.red[v].best[k] = use_pre ? pb_ : no_cand();
                    }
                    if (v == last_act) {
                        sh.carry.cnt[k] = lg >= 0 ? cnt : 0;
                        sh.carry.best[k] = lg >= 0 ? best : no_cand();
                    }
                }
            }
            if (v == last_act) sh.carry_g = lg;
            if (fd) {
                // part v closes its first group: prefix (+) its own aggregate
                const Ctx cf = pol.ctx(g0);
                Agg<NB> tot;
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    tot.cnt[k] = sh.red[v].cnt[k] + sh.wfirst_total[v].cnt[k];
                    tot.best[k] = sh.wfirst_total[v].best[k];
                    if (pol.beats(cf, k, sh.red[v].best[k], tot.best[k], ctr)) tot.best[k] = sh.red[v].best[k];
                }
                if (pol.group_start(g0) >= cb) {
                    pol.finalize(cf, g0, tot);
                } else {
                    sh.first_total = tot;
                    sh.first_done = 1;
                }
            }
        }
        __syncthreads();
    } else {
        if (wb < we) {
            int init[NB];
            const bool chain = sh.carry_g >= 0 && sh.carry_g == pol.group_of(wb, glo, ghi);
#pragma unroll
            for (int k = 0; k < NB; ++k) init[k] = sh.wpref[w][k] + (chain ? sh.carry.cnt[k] : 0);
            process_wave<Pol, MODE>(pol, wb, we, glo, ghi, init, sh, ctr);
        }
    }
}

// Block-wide sum of an int over all threads (result on every thread).
__device__ __forceinline__ int block_sum(int v, int* red)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
    const int w = (int)(threadIdx.x >> 6);
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int u = 0; u < kWaves; ++u) s += red[u];
    __syncthreads();
    return s;
}

// Step B: the chunk's first group g, if it started before the chunk, gets
// its count prefix from the chunks before (`prefix`, or, if null, summed here
// over the chunks it spans); if g also ends inside this chunk, its farthest
// points are reduced over those chunks and it is finalised here. The count
// prefix is left in sh.carry (carry_g = g).
template <class Pol>
__device__ __forceinline__ void chunk_first_group(const Pol& pol, int b, int cb, int CH,
                                                  const ChunkSlot<Pol::NB>* slots, const int* prefix,
                                                  ChunkShared<Pol>& sh, Counters& ctr)
{
    constexpr int NB = Pol::NB;
    using Ctx = typename Pol::Ctx;
    const int g = pol.group_of(cb, 0, pol.num_groups() - 1);
    const int gs = pol.group_start(g);
    const bool finalizing = gs < cb && sh.first_done;
    if (threadIdx.x == 0) {
        sh.carry_g = gs < cb ? g : -1;
        agg_clear(sh.carry);
        if (gs < cb && prefix) {
#pragma unroll
            for (int k = 0; k < NB; ++k) sh.carry.cnt[k] = prefix[k];
        }
    }
    __syncthreads();
    if (!finalizing) return;  // uniform
    // g ends inside this chunk: reduce over chunks c0 .. b-1, plus ours
    const int c0 = gs / CH;
    const Ctx c = pol.ctx(g);
    Cand best[NB];
    int cnt[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) { best[k] = no_cand(); cnt[k] = 0; }
    for (int j = c0 + (int)threadIdx.x; j < b; j += kBlock) {
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            const Cand o = gld(&slots[j].last.best[k]);
            if (pol.beats(c, k, o, best[k], ctr)) best[k] = o;
            cnt[k] += gld(&slots[j].last.cnt[k]);
        }
    }
    const int w = (int)(threadIdx.x >> 6);
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        best[k] = wave_max(pol, c, k, best[k], ctr);
        int v = cnt[k];
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) v += __shfl_xor(v, m);
        cnt[k] = v;
    }
    if (lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < NB; ++k) { sh.red[w].best[k] = best[k]; sh.red[w].cnt[k] = cnt[k]; }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Agg<NB> all;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            all.cnt[k] = sh.first_total.cnt[k];
            all.best[k] = sh.first_total.best[k];
        }
        for (int u = 0; u < kWaves; ++u) {
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                all.cnt[k] += sh.red[u].cnt[k];
                if (pol.beats(c, k, sh.red[u].best[k], all.best[k], ctr)) all.best[k] = sh.red[u].best[k];
            }
        }
        pol.finalize(c, g, all);
    }
    __syncthreads();
}

}  // namespace sqh
