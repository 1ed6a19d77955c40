// Serving engine kernels (device code): one step of continuous batching.
//
// The engine keeps many requests resident in one slot space. A request owns
// a 64-aligned range of slots for its whole life: its surviving points, its
// vertex keys and, once finished, its hull. A step
//   1. runs the seed, the first split and the first compaction (sections
//      4.3, 4.4) over the requests admitted since the last step, whose
//      points were staged back to back; their first segments are appended to
//      the resident segment table;
//   2. runs up to max_passes segmented passes (section 4.4) over every
//      resident segment of every request at once;
//   3. finds the requests left without segments and writes their hulls in
//      ring order into their own slots.
// Requests therefore join and leave the segment table between pass groups,
// and the passes of old and new requests share every launch.
// Included by the host driver after sqh_kernels.hip (one translation unit).

namespace sqh {

// Workgroup-wide ordered emission of one set: the set bits of the vertex
// bitmap over the set's slots, in key order, give the ring; writes the
// vertex indices to hout[base ..] and returns the count (every thread).
__device__ __forceinline__ int emit_set(const HullArgs& a, int base, int n, Pair* red)
{
    const int w0 = base >> 6, w1 = (base + n + 63) >> 6;
    int done = 0;
    for (int wb = w0; wb < w1; wb += kBlock) {
        const int w = wb + (int)threadIdx.x;
        uint64_t bits = w < w1 ? gld(a.bitmap + w) : 0ull;
        Pair tot;
        const Pair ex = block_excl_scan(Pair{(int)__popcll(bits), 0}, red, &tot);
        int r = base + done + ex.a;
        while (bits) {
            const int t = __ffsll((unsigned long long)bits) - 1;
            bits &= bits - 1;
            gst(a.hout + r, gld(a.vidx + (w << 6) + t));
            ++r;
        }
        done += tot.a;
    }
    return done;
}

__global__ __launch_bounds__(kBlock) void k_engine_step(HullArgs a)
{
    __shared__ ChunkShared<PolFirst> sh_first;
    __shared__ Pair red[kWaves];
    auto& shF = sh_first;
    auto& shS = *reinterpret_cast<ChunkShared<PolSeed>*>(&sh_first);
    auto& shP = *reinterpret_cast<ChunkShared<PolSplit>*>(&sh_first);
    auto& shQ = *reinterpret_cast<ChunkShared<PolPass>*>(&sh_first);
    Counters ctr = {0u, 0u, 0u};
    const int b = (int)blockIdx.x, nb = (int)gridDim.x;
    int cur = a.cur0;
    // the resident table, read before the first compaction appends to it
    const Pair res = {ld_flag(a.sv + 2 * cur), ld_flag(a.sv + 2 * cur + 1)};

    stamp(a, 0);
    if (a.G > 0) {
        {
            PolSeed pol{a.xy, a.gstart, a.sets, a.err, nullptr, a.bad, a.G};
            phase_reduce(a, pol, a.N, shS, red, ctr);
        }
        stamp(a, 1);
        {
            PolSplit pol{a.xy, a.gstart, a.sbase, a.bad, nullptr, a.sets, a.bitmap, a.vidx, nullptr, a.info, a.fp64,
                         a.G};
            phase_reduce(a, pol, a.N, shP, red, ctr);
        }
        stamp(a, 2);
        {
            PolFirst pol{a.xy,   a.gstart,  a.sbase,  a.bad,  nullptr, a.sets, a.X[cur], a.Y[cur], a.I[cur],
                         a.recs, a.rec_cid, a.bitmap, a.vidx, nullptr, a.info, a.fp64,   a.G};
            phase_compact<PolFirst, false>(a, pol, a.N, 4, a.segs[cur], a.seg_cid[cur], a.vstart[cur],
                                           a.sv + 2 * cur, res, shF, red, ctr);
        }
        stamp(a, 3);
    }
    // ---- a group of passes over all resident segments
    for (int pass = 0;; ++pass) {
        const int S = ld_flag(a.sv + 2 * cur), V = ld_flag(a.sv + 2 * cur + 1);
        if (b == 0) note_pass(a, pass, S, V);
        if (S <= 0 || pass >= a.max_passes) break;
        if (V <= a.tail_points && S <= kTailSegs) {
            if (b == 0) {
                for (int p = pass;; ++p) {
                    const int S2 = ld_flag(a.sv + 2 * cur), V2 = ld_flag(a.sv + 2 * cur + 1);
                    note_pass(a, p, S2, V2);
                    if (S2 <= 0 || p >= a.max_passes) break;
                    run_pass<PolPass, true>(a, cur, S2, V2, shQ, red, ctr);
                    stamp(a, 100 + p);
                    cur ^= 1;
                }
            }
            break;
        }
        run_pass<PolPass, false>(a, cur, S, V, shQ, red, ctr);
        stamp(a, 100 + pass);
        cur ^= 1;
    }
    if (b == 0 && threadIdx.x == 0) a.info->cur_out = cur;
    grid_sync(a.bar, a.err);  // workgroup 0 may still have run tail passes
    cur = ld_flag(&a.info->cur_out);
    // ---- census: which resident sets still own a segment
    {
        const int S = ld_flag(a.sv + 2 * cur);
        const Seg* segs = a.segs[cur];
        for (int i = b * kBlock + (int)threadIdx.x; i < S; i += nb * kBlock) {
            const int off = gld(&segs[i].off);
            int lo = 0, hi = a.nres - 1;  // largest r with res_base[r] <= off
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (gld(a.res_base + mid) <= off) lo = mid;
                else hi = mid - 1;
            }
            a.res_alive[lo] = 1;
        }
    }
    grid_sync(a.bar, a.err);
    // ---- ordered emission of the sets that finished
    for (int r = b; r < a.nres; r += nb) {
        if (ld_flag(a.res_alive + r)) continue;  // same value on every thread
        const int h = emit_set(a, gld(a.res_base + r), gld(a.res_n + r), red);
        if (threadIdx.x == 0) a.res_h[r] = h;
        __syncthreads();
    }
    stamp(a, 4);
    flush_counters(a.stats, ctr);
}

// Per-step initialisation: barrier, status, counters, the new sets' child
// records, bad flags and vertex-bitmap words (their slot ranges are
// 64-aligned, so whole words belong to one set), and the census flags.
__global__ void k_engine_reset(HullArgs a)
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
        a.info->vcap = 0;
        a.info->cur_out = a.cur0;
    }
    if (gtid < kBarSub) a.bar->sub[gtid][0] = 0;
    for (int i = gtid; i < 4 * kStatSlots; i += gstride) a.stats[i] = 0;
    for (int i = gtid; i < 4 * a.G; i += gstride) {
        a.recs[i].len = 0;
        a.rec_cid[i] = -1;
    }
    for (int i = gtid; i < a.G; i += gstride) a.bad[i] = 0;
    for (int i = gtid; i < a.nres; i += gstride) {
        a.res_alive[i] = 0;
        a.res_h[i] = 0;
    }
    for (int g = (int)blockIdx.x; g < a.G; g += (int)gridDim.x) {
        const int base = a.sbase[g], n = a.gstart[g + 1] - a.gstart[g];
        for (int w = (base >> 6) + (int)threadIdx.x; w < ((base + n + 63) >> 6); w += (int)blockDim.x)
            a.bitmap[w] = 0ull;
    }
}

}  // namespace sqh
