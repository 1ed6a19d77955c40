// Test hooks: the device predicates, the farthest-point order and the
// workgroup scan run on caller-given cases, so that tests can compare the
// device's decisions with exact arithmetic case by case (the hull path
// only shows them through its output). Not used by any hull call.
#pragma once

namespace sqh {

// Per case (ox, oy, ex, ey, px, py): the orientation sign the kernels use
// (semi-static float32 filter, then the exact path), and the two filters'
// raw figures: d, es of the semi-static filter, t, m of the static line
// filter (bounds Mx, My from the case's own coordinates; m = -1 where the
// line filter does not apply). flags bit 0: the semi-static filter decided.
__global__ __launch_bounds__(256) void k_diag_orient(const float* tri, int n, int fp64, int32_t* sign, float* vals,
                                                     int32_t* flags)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const float ox = tri[6 * i], oy = tri[6 * i + 1], ex = tri[6 * i + 2], ey = tri[6 * i + 3];
    const float px = tri[6 * i + 4], py = tri[6 * i + 5];
    const Edge E = make_edge(ox, oy, ex, ey);
    const Orient32 o = orient32(E, px, py);
    int s = fast_sign(o, fp64 != 0);
    const int decided = s != 0;
    if (!decided) s = orient_exact(ox, oy, ex, ey, px, py);
    const float Mx = fmaxf(fabsf(ox), fmaxf(fabsf(ex), fabsf(px)));
    const float My = fmaxf(fabsf(oy), fmaxf(fabsf(ey), fabsf(py)));
    float t = 0.0f, m = -1.0f;
    if (fmaxf(Mx, My) <= kLineCoordMax) {
        const LineF L = make_line(ox, oy, ex, ey, Mx, My);
        t = line_eval(L, px, py);
        m = L.m;
    }
    sign[i] = s;
    flags[i] = decided;
    vals[4 * i] = o.d;
    vals[4 * i + 1] = o.es;
    vals[4 * i + 2] = t;
    vals[4 * i + 3] = m;
}

// Per case (ox, oy, ex, ey, px, py, qx, qy) with indices (pid, qid): 1 when
// P comes before Q in the farthest-point order for the edge o -> e (larger
// area right of the edge; equal areas: earlier along the edge; the same
// position: lower index), with both points' float32 intervals as the
// kernels form them; bit 1 holds the reverse comparison.
__global__ __launch_bounds__(256) void k_diag_compare(const float* cs, const int32_t* ids, int n, int fp64,
                                                      int32_t* out)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const float* c = cs + 8 * i;
    const Edge E = make_edge(c[0], c[1], c[2], c[3]);
    const Cand P = make_cand(orient32(E, c[4], c[5]), c[4], c[5], ids[2 * i]);
    const Cand Q = make_cand(orient32(E, c[6], c[7]), c[6], c[7], ids[2 * i + 1]);
    uint32_t nx = 0;
    const bool pq = beats(E, P, Q, fp64 != 0, nx), qp = beats(E, Q, P, fp64 != 0, nx);
    out[i] = (pq ? 1 : 0) | (qp ? 2 : 0);
}

// Exclusive scans of (v, 1) over each run of kBlock values by the
// workgroup scan every kernel uses; the run totals go to tot.
__global__ __launch_bounds__(kBlock) void k_diag_scan(const int32_t* in, int n, int32_t* ex_a, int32_t* ex_b,
                                                      int32_t* tot)
{
    __shared__ Pair red[kWaves];
    const int i = (int)(blockIdx.x * kBlock + threadIdx.x);
    const Pair v = {i < n ? in[i] : 0, i < n ? 1 : 0};
    Pair all;
    const Pair e = block_excl_scan(v, red, &all);
    if (i < n) {
        ex_a[i] = e.a;
        ex_b[i] = e.b;
    }
    if (threadIdx.x == 0) {
        tot[2 * blockIdx.x] = all.a;
        tot[2 * blockIdx.x + 1] = all.b;
    }
}

}  // namespace sqh
