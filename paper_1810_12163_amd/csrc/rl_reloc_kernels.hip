// rl_reloc_kernels.hip -- per-frame relocalisation kernels (gfx950, wave64).
//
// Pipeline per frame (Sec. 3.2.3 of Cavallari et al., TPAMI 2019):
//   k_prep          clear per-frame state
//   k_traverse      features + routing of every pixel through every tree (Eq. 1-3)
//   k_eligible      raster-order list of pixels with depth and >= 1 mode,
//                   with per-pixel records (colour-check bits of M(u))
//   k_hyp_search    hypothesis generation: all (slot, iteration chunk)
//                   pairs in parallel, first iteration passing checks 1-3
//                   by atomicMin
//   k_hyp_finalize  rebuild each slot's triplet, Kabsch pose (continuing
//                   the scan past a degenerate fit)
//   k_ransac_init   survivors = valid slots in slot order
//   k_score/k_select  one preemptive-RANSAC round each (Eq. 5, halving)
//   k_finalize      winner, optional refit over inliers, result record
#include <hip/hip_runtime.h>
#include <limits.h>

#include <algorithm>

#include "rl_internal.hpp"

namespace rl {

__device__ __forceinline__ int wave_lane() { return threadIdx.x & 63; }

// exclusive prefix of a predicate within a block of 256 threads (4 waves);
// returns the prefix, writes the block total to *total.
__device__ __forceinline__ int block_prefix256(bool pred, int* s_wave, int* total)
{
    const unsigned long long b = __ballot(pred);
    const int lane = wave_lane(), wv = threadIdx.x >> 6;
    const int below_lane = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[wv] = __popcll(b);
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < wv) base += s_wave[i];
        tot += s_wave[i];
    }
    __syncthreads();
    *total = tot;
    return base + below_lane;
}

// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prep(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s < J.N) J.hyp_best[s] = INT_MAX;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        J.st->n_elig = 0;
        J.st->n_valid = 0;
        J.st->n_surv = 0;
        J.st->rounds_run = 0;
        J.st->done = 1;
    }
}

// ------------------------------------------------------------------------
// Frame ingest: the probe image (a plane of depth bits, a plane of R, G, B
// bytes) that routing reads, one pass over the caller's buffers (any row pitch, RGB or
// RGBA, every pixel or every second one); every later read of the frame is a
// read of this image.
__global__ __launch_bounds__(256) void k_pack(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    const int P = J.w * J.h;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int x = p % J.w, y = p / J.w;
    const uint8_t* c = J.src.c(x, y);
    const uint32_t r = ldg(c), g = ldg(c + 1), b = ldg(c + 2);
    J.probe[p] = __float_as_uint(J.src.d(x, y));
    J.probe[P + p] = r | (g << 8) | (b << 16);
}

// ------------------------------------------------------------------------
// Workgroup (x, y) of a (tiles, jobs) grid runs on XCD (x + y gridDim.x) mod
// 8.  With gridDim.x a multiple of 8, XCD e takes the e-th eighth of each
// frame's tiles (a band of rows), so its L2 holds the part of the frame that
// its probes read rather than the whole frame.  -1: no tile.
__device__ __forceinline__ int band_tile(int bx, int gx, int ntiles)
{
    if (gx & 7) return bx < ntiles ? bx : -1;
    const int per = (ntiles + 7) >> 3, k = bx >> 3;
    const int t = (bx & 7) * per + k;
    return (k < per && t < ntiles) ? t : -1;
}

// One thread per pixel, all trees in lockstep.  Writes leaves (16 B/pixel),
// per-tree mode counts (8 B/pixel), |M(u)| and the tile's eligible count.
template <int T, int TOP>
__global__ __launch_bounds__(256) void k_traverse(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    const int w = J.w, h = J.h, P = w * h;
    const int tile = band_tile((int)blockIdx.x, (int)gridDim.x, (P + 255) / 256);
    if (tile < 0) return;
    __shared__ int s_wave[4];
    // the top levels of every tree, shared by the block's pixels
    __shared__ float4 s_top[T * ((1 << TOP) - 1)];
    const int ktop = min(J.D, TOP), ntop = (1 << ktop) - 1;
    for (int i = threadIdx.x; i < T * ntop; i += 256) {
        const int t = i / ntop;
        s_top[i] = ldg(J.nodes + t * ((1 << J.D) - 1) + (i - t * ntop));
    }
    __syncthreads();
    const int p = tile * 256 + threadIdx.x;
    bool elig = false;
    if (p < P) {
        const int x = p % w, y = p / w;
        const float d = __uint_as_float(ldg(J.probe + p));
        uint16_t lf[8];
        uint8_t nmt[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            lf[t] = (uint16_t)kLeafNone;
            nmt[t] = 0;
        }
        int total = 0;
        if (depth_ok(d)) {
            const int NT = (1 << J.D) - 1;
            int leaf[T];
            const PackedProbe pr{J.probe, (uint32_t)w, (uint32_t)P};
            if (J.s == 1.0f) route<T, true>(J.nodes, NT, J.D, pr, w, h, x, y, d, J.s, leaf, s_top, ktop);
            else route<T, false>(J.nodes, NT, J.D, pr, w, h, x, y, d, J.s, leaf, s_top, ktop);
#pragma unroll
            for (int t = 0; t < T; ++t) {
                lf[t] = (uint16_t)leaf[t];
                const int c = ldg(J.nmodes + ((size_t)t << J.D) + leaf[t]);
                nmt[t] = (uint8_t)c;
                total += c;
            }
        }
        uint4 lw;
        lw.x = (uint32_t)lf[0] | ((uint32_t)lf[1] << 16);
        lw.y = (uint32_t)lf[2] | ((uint32_t)lf[3] << 16);
        lw.z = (uint32_t)lf[4] | ((uint32_t)lf[5] << 16);
        lw.w = (uint32_t)lf[6] | ((uint32_t)lf[7] << 16);
        reinterpret_cast<uint4*>(J.leaves)[p] = lw;
        uint2 nw;
        nw.x = (uint32_t)nmt[0] | ((uint32_t)nmt[1] << 8) | ((uint32_t)nmt[2] << 16) | ((uint32_t)nmt[3] << 24);
        nw.y = (uint32_t)nmt[4] | ((uint32_t)nmt[5] << 8) | ((uint32_t)nmt[6] << 16) | ((uint32_t)nmt[7] << 24);
        reinterpret_cast<uint2*>(J.nmt)[p] = nw;
        J.nm[p] = (uint8_t)min(total, 255);
        elig = total > 0;
    }
    int tot;
    (void)block_prefix256(elig, s_wave, &tot);
    if (threadIdx.x == 0) J.tile_count[tile] = tot;
}

// A walk over M(u) in tree-major order (the order mode_row numbers it): the
// row index of the current mode, advanced one mode at a time; the leaf's
// base row is recomputed only when the walk moves on to another tree.
// Rows fit 32 bits (T * 2^D * M <= 8 * 32768 * 64).
struct ModeWalk {
    uint4 lw;
    uint2 nw;
    int T, D, M, t, j, c;
    uint32_t base;
    __device__ __forceinline__ ModeWalk(const Job& J, uint4 lw_, uint2 nw_)
        : lw(lw_), nw(nw_), T(J.T), D(J.D), M(J.M), t(0), j(0)
    {
        c = (int)count_of(nw, 0);
        while (t < T - 1 && c == 0) c = (int)count_of(nw, ++t);
        base = (((uint32_t)t << D) + leaf_of(lw, t)) * (uint32_t)M;
    }
    // positioned at mode m of M(u) (m below |M(u)|)
    __device__ __forceinline__ ModeWalk(const Job& J, uint4 lw_, uint2 nw_, int m)
        : lw(lw_), nw(nw_), T(J.T), D(J.D), M(J.M), t(0), j(m)
    {
        c = (int)count_of(nw, 0);
        while (j >= c) {
            j -= c;
            c = (int)count_of(nw, ++t);
        }
        base = (((uint32_t)t << D) + leaf_of(lw, t)) * (uint32_t)M;
    }
    __device__ __forceinline__ uint32_t row() const { return base + (uint32_t)j; }
    // called only while another mode of M(u) follows
    __device__ __forceinline__ void next()
    {
        if (++j < c) return;
        j = 0;
        do c = (int)count_of(nw, ++t);
        while (c == 0);
        base = (((uint32_t)t << D) + leaf_of(lw, t)) * (uint32_t)M;
    }
};

// Record of eligible pixel p at list position e: |M(u)| and the colour-check
// bit of every mode of M(u), in M(u) order, from the modes' colour boxes.
// The boxes are walked tree by tree, eight loaded ahead of their checks.
__device__ __forceinline__ void write_erec(const Job& J, int e, uint4 lw, uint2 nw, uint32_t rgb)
{
    uint64_t* rec = J.erec + (size_t)e * J.ew;
    const uint32_t x = box_colour(rgb);
    const int total = modes_total(nw, J.T);
    uint64_t w0 = 0, cur = 0;
    ModeWalk mw(J, lw, nw);
    for (int m0 = 0; m0 < total; m0 += 8) {
        uint2 bx[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bx[u] = ldg(J.cbox + mw.row());
            if (m0 + u + 1 < total) mw.next();
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t m = (uint32_t)(m0 + u);
            if ((int)m >= total) break;
            const uint64_t b = box_pass(bx[u], x) ? 1u : 0u;
            if (m < 56) {
                w0 |= b << (8 + m);
            } else {
                const uint32_t k = m - 56;
                cur |= b << (k & 63);
                if ((k & 63) == 63) {
                    rec[1 + (k >> 6)] = cur;
                    cur = 0;
                }
            }
        }
    }
    if (total > 56 && ((total - 56) & 63)) rec[1 + ((total - 56) >> 6)] = cur;
    rec[0] = w0 | (uint64_t)total;
}

// Exclusive scan of the traversal's per-tile eligible counts (in place) and
// the list length; one block per job.
__global__ __launch_bounds__(1024) void k_tile_scan(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.x];
    const int P = J.w * J.h;
    const int ntiles = (P + 255) / 256;
    __shared__ int s_sum[1024];
    const int per = (ntiles + 1023) / 1024;
    const int t0 = (int)threadIdx.x * per, t1 = min(t0 + per, ntiles);
    int sum = 0;
    for (int i = t0; i < t1; ++i) sum += J.tile_count[i];
    s_sum[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {          // inclusive scan of the thread sums
        const int v = (int)threadIdx.x >= off ? s_sum[threadIdx.x - off] : 0;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        __syncthreads();
    }
    int run = s_sum[threadIdx.x] - sum;
    for (int i = t0; i < t1; ++i) {
        const int c = J.tile_count[i];
        J.tile_count[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) J.st->n_elig = s_sum[1023];
}

// The record when every pixel's bits fit word 0 (the room, or the batch,
// has at most 56 modes per pixel): M(u) is walked tree by tree, a tree's rows
// contiguous from its leaf's base row, eight loaded ahead of their tests.
// A wave runs each tree's loop to its largest count, but no lane leaves a
// loop for another tree mid-way, which in the single walk above made every
// step pay for some lane's tree switch.  Same order, same bits.
template <int T>
__device__ __forceinline__ void write_erec_w0(const Job& J, int e, uint4 lw, uint2 nw, uint32_t rgb)
{
    const uint32_t x = box_colour(rgb);
    uint64_t w0 = 0;
    int m0 = 0;   // modes of M(u) in the trees before t
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int c = (int)count_of(nw, t);
        const uint2* rows = J.cbox + (size_t)((((uint32_t)t << J.D) + leaf_of(lw, t)) * (uint32_t)J.M);
        for (int j0 = 0; j0 < c; j0 += 8) {
            uint2 bx[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u < c) bx[u] = ldg(rows + j0 + u);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j0 + u < c && box_pass(bx[u], x)) w0 |= 1ull << (8 + m0 + j0 + u);
        }
        m0 += c;
    }
    J.erec[(size_t)e * J.ew] = w0 | (uint64_t)m0;
}

// Raster-order compaction of eligible pixels over the traversal's tiles, and
// their records.
template <int T>
__global__ __launch_bounds__(256) void k_eligible(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    const int P = J.w * J.h;
    const int ntiles = (P + 255) / 256;
    if ((int)blockIdx.x >= ntiles) return;
    __shared__ int s_wave[4];
    const int base = J.tile_count[blockIdx.x];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool e = p < P && ldg(J.nm + p) > 0;
    int tot;
    const int pre = block_prefix256(e, s_wave, &tot);
    if (e) {
        const int k = base + pre;
        J.eligible[k] = p;
        const uint4 lw = ldg(reinterpret_cast<const uint4*>(J.leaves) + p);
        const uint2 nw = ldg(reinterpret_cast<const uint2*>(J.nmt) + p);
        const uint32_t pd = ldg(J.probe + p), pc = ldg(J.probe + P + p);
        J.ecold[2 * k] = make_uint4((uint32_t)p, pd, nw.x, nw.y);
        J.ecold[2 * k + 1] = lw;
        if (J.ew == 1) write_erec_w0<T>(J, k, lw, nw, pc);
        else write_erec(J, k, lw, nw, pc);
    }
}

// ------------------------------------------------------------------------
// Hypothesis generation (Sec. 3.2.3).  Iteration it of slot s draws two
// Philox blocks, counters (HYP|blk, s, it, 0).  Block 0 serves the pair the
// colour check looks at: a.x picks that pair k* in {0,1,2}, a.y its pixel
// (eligible list), a.z its mode (M(u)); block 1 serves the other two pairs in
// increasing order (b.x, b.y pixels; b.z, b.w modes).  Checks: (1) colour of
// pair k* (L-infinity, float32), (2) pairwise world distances^2 >= min, (3)
// rigidity, then Kabsch non-degenerate.  Check quantities are evaluated
// exactly as written (no contraction).
//
// The search is split in two stages so that the cheap, selective colour
// check (about 1 in 9 passes) runs dense over many iterations and only its
// survivors, compacted into an LDS queue, pay for the other two pixels, the
// back-projections and the rigidity test: lanes stay busy instead of idling
// behind divergent branches.  The colour check itself is a bit test in the
// eligible-pixel record (its outcome per (pixel, mode) is fixed per frame).

__device__ __forceinline__ uint32_t mode_row_index(const Job& J, uint4 lw, uint2 nw, int m)
{
    int t = 0;
    for (; t < J.T - 1; ++t) {
        const int c = (int)count_of(nw, t);
        if (m < c) break;
        m -= c;
    }
    return ((((uint32_t)t << J.D) + leaf_of(lw, t)) * (uint32_t)J.M + (uint32_t)m);
}

// One (pixel, mode) pair of a triplet, from list entry e and mode index m of
// M(u): the entry's 32-byte record holds the pixel, its depth and its leaf
// record, so the pair costs two dependent gathers (record, mode row).
struct Pair {
    int p, m;
    float d;
    uint32_t row;
    double xw[3], xc[3];
};

// the pair from list-entry record (c0, c1) and mode index m of M(u)
__device__ __forceinline__ void pair_from(const Job& J, uint4 c0, uint4 c1, int m, Pair& q)
{
    q.p = (int)c0.x;
    q.d = __uint_as_float(c0.y);
    q.m = m;
    q.row = mode_row_index(J, c1, make_uint2(c0.z, c0.w), m);
    const float4 w = ldg(J.modes + (size_t)q.row * 4);
    q.xw[0] = w.x;
    q.xw[1] = w.y;
    q.xw[2] = w.z;
}

// the pair drawn by (rp, rm): entry from rp, mode from rm over |M(u)|; both
// halves of the entry's record are loaded together (one cache line), so the
// pair costs two dependent gathers
__device__ __forceinline__ void draw_pair(const Job& J, int n_elig, uint32_t rp, uint32_t rm, Pair& q)
{
    const uint32_t e = below(rp, (uint32_t)n_elig);
    const uint4 c0 = ldg(J.ecold + 2 * e), c1 = ldg(J.ecold + 2 * e + 1);
    const uint2 nw = make_uint2(c0.z, c0.w);
    pair_from(J, c0, c1, (int)below(rm, (uint32_t)modes_total(nw, J.T)), q);
}

__device__ __forceinline__ void pair_backproject(const Job& J, Pair& q)
{
    backproject(q.d, q.p % J.w, q.p / J.w, J.fx, J.fy, J.cx, J.cy, q.xc);
}

// checks 2 and 3 on one pair of pairs: world distance^2 >= min, and the
// camera and world distances agree within the rigidity tolerance
__device__ __forceinline__ bool world_far(const Job& J, const Pair& a, const Pair& b, double& dw2)
{
#pragma clang fp contract(off)
    const double dx = a.xw[0] - b.xw[0], dy = a.xw[1] - b.xw[1], dz = a.xw[2] - b.xw[2];
    dw2 = dx * dx + dy * dy + dz * dz;
    return !(dw2 < J.min_sq_dist);
}

__device__ __forceinline__ bool rigid_pair(const Job& J, const Pair& a, const Pair& b, double dw2)
{
#pragma clang fp contract(off)
    const double dx = a.xc[0] - b.xc[0], dy = a.xc[1] - b.xc[1], dz = a.xc[2] - b.xc[2];
    const double dc2 = dx * dx + dy * dy + dz * dz;
    return !(fabs(sqrt(dc2) - sqrt(dw2)) > J.theta_rig);
}

// stage A: the colour check of pair k* (list entry ec, mode mc of M(u))
__device__ __forceinline__ bool hyp_stage_a(const Job& J, int n_elig, int slot, int it, int& kc, int& ec,
                                            int& mc)
{
    const uint4 a = philox(make_uint4((kTagHyp << 28) | 0u, (uint32_t)slot, (uint32_t)it, 0u), J.key0, J.key1);
    kc = (int)below(a.x, 3u);
    ec = (int)below(a.y, (uint32_t)n_elig);
    const uint64_t* rec = J.erec + (uint32_t)ec * (uint32_t)J.ew;
    const uint64_t h = ldg(rec);
    const uint32_t m = below(a.z, erec_total(h));
    mc = (int)m;
    return erec_bit(rec, h, m);
}

// Degeneracy test of the Kabsch fit without an eigen-solver: for a triplet A
// has rank <= 2, so the eigenvalues l1 >= l2 of A^T A follow from
// e1 = l1 + l2 = |A|_F^2 and e2 = l1 l2 = sum of squared 2x2 minors of A.
// The search rejects a triplet only when l2 < 1e-8 l1 holds with a relative
// margin of 1e-6, far beyond the rounding of either computation, so it never
// rejects a triplet the exact test (rigid_from_cov) accepts.
__device__ __forceinline__ bool clearly_degenerate(const double A[9])
{
    double e1 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) e1 += A[i] * A[i];
    double e2 = 0.0;
#pragma unroll
    for (int r1 = 0; r1 < 2; ++r1)
#pragma unroll
        for (int r2 = r1 + 1; r2 < 3; ++r2)
#pragma unroll
            for (int c1 = 0; c1 < 2; ++c1)
#pragma unroll
                for (int c2 = c1 + 1; c2 < 3; ++c2) {
                    const double mnr = A[r1 * 3 + c1] * A[r2 * 3 + c2] - A[r1 * 3 + c2] * A[r2 * 3 + c1];
                    e2 += mnr * mnr;
                }
    if (!(e1 > 0.0)) return true;
    const double l1 = 0.5 * (e1 + sqrt(fmax(e1 * e1 - 4.0 * e2, 0.0)));
    const double l2 = e2 / l1;
    return l2 < 1e-8 * (1.0 - 1e-6) * l1;
}

// stage B: the other two pairs, checks 2 and 3; with KABSCH the Kabsch fit
// (rejecting degenerate triplets) and the hypothesis record.  The search runs
// without KABSCH and rejects only clearly degenerate triplets: the FP64
// eigen-solver would otherwise set the search kernel's register budget.
// The checks are a conjunction over the three unordered pairs of pairs, so
// they are evaluated pair by pair and the third pair is only gathered when
// the first two agree; each quantity is computed as in the canonical order
// (a squared difference does not depend on its sign).
template <bool KABSCH>
__device__ __forceinline__ bool hyp_stage_b(const Job& J, int n_elig, int slot, int it, int kc, int ec, int mc,
                                            Hyp* out)
{
#pragma clang fp contract(off)
    // pair k*'s record is known before the second block is drawn
    const uint4 k0 = ldg(J.ecold + 2 * (uint32_t)ec), k1 = ldg(J.ecold + 2 * (uint32_t)ec + 1);
    const uint4 b = philox(make_uint4((kTagHyp << 28) | 1u, (uint32_t)slot, (uint32_t)it, 0u), J.key0, J.key1);
    Pair pk, pa, pb;
    pair_from(J, k0, k1, mc, pk);
    draw_pair(J, n_elig, b.x, b.z, pa);
    double dka, dkb, dab;
    if (!world_far(J, pk, pa, dka)) return false;
    pair_backproject(J, pk);
    pair_backproject(J, pa);
    if (!rigid_pair(J, pk, pa, dka)) return false;
    draw_pair(J, n_elig, b.y, b.w, pb);
    if (!world_far(J, pk, pb, dkb) || !world_far(J, pa, pb, dab)) return false;
    pair_backproject(J, pb);
    if (!rigid_pair(J, pk, pb, dkb) || !rigid_pair(J, pa, pb, dab)) return false;
    // canonical order: pair k* at position kc, the other two in draw order
    const Pair& q0 = kc == 0 ? pk : pa;
    const Pair& q1 = kc == 1 ? pk : (kc == 0 ? pa : pb);
    const Pair& q2 = kc == 2 ? pk : pb;
    const double* xc[3] = {q0.xc, q1.xc, q2.xc};
    const double* xw[3] = {q0.xw, q1.xw, q2.xw};
    double cc[3], cw[3], A[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cc[i] = (xc[0][i] + xc[1][i] + xc[2][i]) / 3.0;
        cw[i] = (xw[0][i] + xw[1][i] + xw[2][i]) / 3.0;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            A[i * 3 + j] = (xc[0][i] - cc[i]) * (xw[0][j] - cw[j]) + (xc[1][i] - cc[i]) * (xw[1][j] - cw[j])
                         + (xc[2][i] - cc[i]) * (xw[2][j] - cw[j]);
    if (!KABSCH) return !(J.screen && clearly_degenerate(A));
    double R[9], t[3];
    if (!rigid_from_cov(A, cc, cw, R, t)) return false;
    for (int i = 0; i < 9; ++i) out->R[i] = (float)R[i];
    for (int i = 0; i < 3; ++i) out->t[i] = (float)t[i];
    out->pix[0] = q0.p;
    out->pix[1] = q1.p;
    out->pix[2] = q2.p;
    out->mode[0] = q0.m;
    out->mode[1] = q1.m;
    out->mode[2] = q2.m;
    return true;
}

// Tuning of the search kernel: an optional minimum of resident waves per
// SIMD (caps registers; 0 = none) and the early exit; the iterations per
// thread are chosen at run time (rl_batch_set_schedule).
#ifndef RL_HYP_WAVES
#define RL_HYP_WAVES 0
#endif
#ifndef RL_HYP_EARLY_EXIT
#define RL_HYP_EARLY_EXIT 1
#endif
#if RL_HYP_WAVES > 0
#define RL_HYP_BOUNDS __launch_bounds__(256, RL_HYP_WAVES)
#else
#define RL_HYP_BOUNDS __launch_bounds__(256)
#endif

// XCD-aware placement of a one-dimensional grid over (job, x < X): workgroup
// w is dispatched to XCD w % 8.  Jobs are dealt round-robin to groups of s
// XCDs (s = 8 for one job, 1 for eight or more), so that each XCD's L2 holds
// the tables of the few jobs it works on instead of every XCD caching all.
// Returns false for the grid's padding.
__device__ __forceinline__ bool xcd_place(int w, int X, int njobs, int s, int& job, int& x)
{
    const int e = w & 7, groups = 8 / s;
    const int q = (w >> 3) * s + e % s;
    const int js = q / X;
    x = q - js * X;
    job = e / s + groups * js;
    return job < njobs;
}

// Per job, x = chunk * Nmax + slot (chunk-major); a block covers 256 * IPT
// consecutive iterations of one slot, each of its waves 64 * IPT of them on
// its own: stage A, a queue in the wave's part of LDS (positions from a
// ballot), stage B, with no block barrier, so a wave never waits for
// another.  A wave whose iterations start after an already-found passing
// iteration leaves at once; the minimum stays exact because every lower
// iteration is always evaluated, and a passing iteration lowers the slot's
// minimum directly (rare, so the atomics are few).
template <int IPT>
__global__ RL_HYP_BOUNDS void k_hyp_search(const Job* __restrict__ jobs, int Nmax, int njobs, int X, int s)
{
    int job, x;
    if (!xcd_place((int)blockIdx.x, X, njobs, s, job, x)) return;
    const Job& J = jobs[job];
    const int slot = x % Nmax, chunk = x / Nmax;
    if (slot >= J.N) return;
    const int wv = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int it0 = chunk * 256 * IPT + wv * 64 * IPT;
    if (it0 >= J.I_max) return;
    const int n_elig = J.st->n_elig;
    if (n_elig <= 0) return;
    __shared__ uint32_t q_it[4][64 * IPT];   // iteration | k* << 30
    __shared__ uint32_t q_em[4][64 * IPT];   // list entry | mode << 24
#if RL_HYP_EARLY_EXIT
    // the exit is decided on one value for the whole wave (other blocks
    // lower it concurrently), so its lanes leave together
    const int best = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&J.hyp_best[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (best < it0) return;
#endif
    // stage A in two passes: all IPT draws and record loads are issued before
    // any of them is consumed, so the gathers overlap
    uint32_t ka[IPT], ea[IPT], za[IPT];
    uint64_t ha[IPT];
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const uint32_t it = (uint32_t)(it0 + k * 64 + lane);
        const uint4 a = philox(make_uint4((kTagHyp << 28) | 0u, (uint32_t)slot, it, 0u), J.key0, J.key1);
        ka[k] = below(a.x, 3u);
        ea[k] = below(a.y, (uint32_t)n_elig);
        za[k] = a.z;
        ha[k] = ldg(J.erec + ea[k] * (uint32_t)J.ew);
    }
    int n = 0;
#pragma unroll
    for (int k = 0; k < IPT; ++k) {
        const int it = it0 + k * 64 + lane;
        const uint32_t m = below(za[k], erec_total(ha[k]));
        const bool pass = it < J.I_max && erec_bit(J.erec + ea[k] * (uint32_t)J.ew, ha[k], m);
        const uint64_t mask = __ballot(pass);
        if (pass) {
            const int q = n + (int)__popcll(mask & ((1ull << lane) - 1ull));
            q_it[wv][q] = (uint32_t)it | (ka[k] << 30);
            q_em[wv][q] = ea[k] | (m << 24);
        }
        n += (int)__popcll(mask);
    }
    // the wave reads back only its own queue: its LDS writes precede its reads
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < n; j += 64) {
        const int it = (int)(q_it[wv][j] & 0x3FFFFFFFu), kc = (int)(q_it[wv][j] >> 30);
        const int ec = (int)(q_em[wv][j] & 0xFFFFFFu), mc = (int)(q_em[wv][j] >> 24);
        if (hyp_stage_b<false>(J, n_elig, slot, it, kc, ec, mc, nullptr)) atomicMin(&J.hyp_best[slot], it);
    }
}

__global__ __launch_bounds__(256) void k_hyp_finalize(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    const int slot = blockIdx.x * 256 + threadIdx.x;
    if (slot >= J.N) return;
    Hyp hy;
    for (int i = 0; i < 9; ++i) hy.R[i] = 0.0f;
    for (int i = 0; i < 3; ++i) {
        hy.t[i] = 0.0f;
        hy.pix[i] = -1;
        hy.mode[i] = -1;
    }
    hy.iter = -1;
    hy.valid = 0;
    // hyp_best = first iteration passing checks 1-3.  If its Kabsch fit is
    // degenerate the answer is the first later iteration passing everything,
    // found by continuing the scan here (triplets that pass the distance and
    // rigidity checks and are still collinear are practically absent).
    const int n_elig = J.st->n_elig;
    if (n_elig > 0) {
        for (int it = max(J.hyp_best[slot], 0); it < J.I_max; ++it) {
            int kc, ec, mc;
            if (hyp_stage_a(J, n_elig, slot, it, kc, ec, mc) && hyp_stage_b<true>(J, n_elig, slot, it, kc, ec, mc, &hy)) {
                hy.iter = it;
                hy.valid = 1;
                atomicAdd(&J.st->n_valid, 1);
                break;
            }
        }
    }
    J.hyps[slot] = hy;
}

// Survivors = valid slots in ascending slot order; energies cleared.
__global__ __launch_bounds__(256) void k_ransac_init(const Job* __restrict__ jobs)
{
    const Job& J = jobs[blockIdx.y];
    __shared__ int s_wave[4];
    int base = 0;
    for (int s0 = 0; s0 < J.N; s0 += 256) {
        const int s = s0 + threadIdx.x;
        const bool v = s < J.N && J.hyps[s].valid;
        if (s < J.N) J.E[s] = 0.0;
        int tot;
        const int pre = block_prefix256(v, s_wave, &tot);
        if (v) J.surv[base + pre] = s;
        base += tot;
    }
    if (threadIdx.x == 0) {
        J.st->n_surv = base;
        J.st->rounds_run = 0;
        J.st->done = (base == 0 || J.st->n_elig <= 0) ? 1 : 0;
    }
}

// ------------------------------------------------------------------------
// Eq. 5 distance q = d^T A d for d = y - mu (A = the row's Sigma^-1, or I)
// from a mode row already loaded (mean in a.xyz; Sigma^-1 upper triangle in
// b.xyzw, c.xy)
template <bool COV>
__device__ __forceinline__ double row_q(const float4& a, const float4& b, const float4& c, double y0, double y1,
                                        double y2)
{
#pragma clang fp contract(off)
    const double d0 = y0 - (double)a.x, d1 = y1 - (double)a.y, d2 = y2 - (double)a.z;
    if (!COV) return d0 * d0 + d1 * d1 + d2 * d2;
    const double m3 = b.x, m4 = b.y, m5 = b.z, m6 = b.w, m7 = c.x, m8 = c.y;
    return d0 * (m3 * d0 + m4 * d1 + m5 * d2) + d1 * (m4 * d0 + m6 * d1 + m7 * d2)
         + d2 * (m5 * d0 + m7 * d1 + m8 * d2);
}

// Eq. 5 terms of one hypothesis (R, t) over the pixels k0 .. k0 + tp - 1 of
// round `round`, summed in pixel order in FP64.  Every lane of a wave walks
// the same pixels and the same mode rows of M(u) (one broadcast request per
// row for the wave).  Lane 0 of a wave with write_I records the pixels in I.
// The rows of M(u) (tree-major, as mode_row orders them) are visited
// kScoreRows at a time, all loaded before their comparisons; the minimum is taken
// in M(u) order.  The tile's list entries and records are loaded before its
// first pixel is scored.
#ifndef RL_SCORE_ROWS
#define RL_SCORE_ROWS 2
#endif
constexpr int kScoreRows = RL_SCORE_ROWS;

template <bool COV>
__device__ __forceinline__ double nearest_q(const Job& J, uint4 lw, uint2 nw, double y0, double y1, double y2)
{
    const int total = modes_total(nw, J.T);
    double best = INFINITY;
    ModeWalk mw(J, lw, nw);
    for (int m0 = 0; m0 < total; m0 += kScoreRows) {
        float4 ra[kScoreRows], rb[kScoreRows], rc[kScoreRows];
#pragma unroll
        for (int u = 0; u < kScoreRows; ++u) {
            const float4* row = J.modes + (size_t)mw.row() * 4;
            ra[u] = ldg(row);
            if (COV) {
                rb[u] = ldg(row + 1);
                rc[u] = ldg(row + 2);
            } else {
                rb[u] = rc[u] = ra[u];
            }
            if (m0 + u + 1 < total) mw.next();
        }
#pragma unroll
        for (int u = 0; u < kScoreRows; ++u)
            if (m0 + u < total) best = fmin(best, row_q<COV>(ra[u], rb[u], rc[u], y0, y1, y2));
    }
    return best;
}

__device__ __forceinline__ double score_pixels(const Job& J, int round, int k0, int tp, bool write_I,
                                               const double R[9], const double t[3])
{
#pragma clang fp contract(off)
    const bool cov = J.use_cov != 0;
    const uint32_t n_elig = (uint32_t)J.st->n_elig;
    const uint32_t blk0 = (uint32_t)k0 >> 2;
    const uint4 rb0 = philox(make_uint4(kTagScore << 28, (uint32_t)round, blk0, 0u), J.key0, J.key1);
    uint4 c0[kScoreTile], lw[kScoreTile];
#pragma unroll
    for (int i = 0; i < kScoreTile; ++i) {
        const int k = k0 + min(i, tp - 1);
        const uint4 rb = ((uint32_t)k >> 2) == blk0
                             ? rb0
                             : philox(make_uint4(kTagScore << 28, (uint32_t)round, (uint32_t)(k >> 2), 0u), J.key0,
                                      J.key1);
        const uint32_t rv = (k & 3) == 0 ? rb.x : (k & 3) == 1 ? rb.y : (k & 3) == 2 ? rb.z : rb.w;
        const uint32_t e = below(rv, n_elig);
        c0[i] = ldg(J.ecold + 2 * e);
        lw[i] = ldg(J.ecold + 2 * e + 1);
    }
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < kScoreTile; ++i) {
        if (i >= tp) break;
        const int k = k0 + i;
        const int p = (int)c0[i].x;
        if (write_I) J.I[round * J.eta + k] = p;
        double x[3];
        backproject(__uint_as_float(c0[i].y), p % J.w, p / J.w, J.fx, J.fy, J.cx, J.cy, x);
        const double y0 = R[0] * x[0] + R[1] * x[1] + R[2] * x[2] + t[0];
        const double y1 = R[3] * x[0] + R[4] * x[1] + R[5] * x[2] + t[1];
        const double y2 = R[6] * x[0] + R[7] * x[1] + R[8] * x[2] + t[2];
        const uint2 nw = make_uint2(c0[i].z, c0[i].w);
        const double best = cov ? nearest_q<true>(J, lw[i], nw, y0, y1, y2) : nearest_q<false>(J, lw[i], nw, y0, y1, y2);
        acc += sqrt(fmax(best, 0.0));
    }
    return acc;
}

__device__ __forceinline__ void hyp_pose(const Hyp& hy, double R[9], double t[3])
{
    for (int i = 0; i < 9; ++i) R[i] = hy.R[i];
    for (int i = 0; i < 3; ++i) t[i] = hy.t[i];
}

// sum of n values p[0], p[stride], ... in index order; loads are issued W at
// a time (the last group padded) ahead of the additions
template <int W = 16>
__device__ __forceinline__ double sum_in_order(const double* p, size_t stride, int n)
{
    double acc = 0.0;
    for (int i = 0; i < n; i += W) {
        const int m = min(W, n - i);
        double v[W];
#pragma unroll
        for (int k = 0; k < W; ++k) v[k] = k < m ? ldg(p + (size_t)(i + k) * stride) : 0.0;
#pragma unroll
        for (int k = 0; k < W; ++k)
            if (k < m) acc += v[k];
    }
    return acc;
}

// One scoring round (while a job has more than fast_max survivors): grid.x =
// ptiles * htiles, one wave per block; the wave takes TP of this round's
// pixels and 64 survivors, one per lane.
__global__ __launch_bounds__(64) void k_score(const Job* __restrict__ jobs, int round, int nptiles)
{
    const Job& J = jobs[blockIdx.y];
    const int n = J.st->n_surv;
    // jobs with LM refinement: this kernel scores their first round only
    if (J.st->done || (J.lm ? round > 0 : n <= J.fast_max)) return;
    const int ptile = blockIdx.x % nptiles, htile = blockIdx.x / nptiles;
    const int TP = J.TP;
    const int k0 = ptile * TP;
    if (k0 >= J.eta || htile * 64 >= n) return;
    const int tp = min(TP, J.eta - k0);
    const int pos = htile * 64 + (int)threadIdx.x;
    const bool active = pos < n;
    double R[9], t[3];
    hyp_pose(J.hyps[active ? J.surv[pos] : J.surv[0]], R, t);
    const double acc = score_pixels(J, round, k0, tp, htile == 0 && threadIdx.x == 0, R, t);
    if (active) J.partial[(size_t)ptile * J.N + pos] = acc;
}

// Rounds of a job with n valid hypotheses (initial cull, then halving to
// n_out; at least one round).
__device__ __forceinline__ int rounds_of(int n, int n_cull, int n_out, int r = 0)
{
    bool first = r == 0;
    while (first || n > n_out) {
        n = (first && n_cull < n) ? n_cull : (n > n_out ? (n + 1) / 2 : n);
        ++r;
        first = false;
    }
    return r;
}

// The remaining rounds at once, once a job's survivors fit fast_max lanes
// (from its first round when it has at most fast_max valid hypotheses, else
// after the per-round kernels have halved it that far): which pixels a round
// adds does not depend on the survivors, so each (round, pixel tile, 64
// hypotheses) wave scores every current survivor, whether or not it lives to
// that round; the selection below uses only the survivors' values.
// The rounds can also be taken a window at a time (the first wr rounds, a
// selection, then the rest): the later rounds then score only the survivors
// of the window, with the same per-round sums.  A wave serves 64 lanes: with
// at most 32 survivors it takes G = 64 / H pixel tiles, H lanes (the power of
// two at or above the survivor count) per tile, so the waves a round needs
// shrink with its survivors; every (survivor, tile) sum is the same.
// grid.x = wr * ptiles * fw: rounds r0 .. r0 + wr - 1 of each job, r0 = the
// rounds it has run; fw = fast_max / 64.
__global__ __launch_bounds__(64) void k_score_all(const Job* __restrict__ jobs, int nptiles, int fw)
{
    const Job& J = jobs[blockIdx.y];
    if (J.st->done || J.lm) return;
    const int n = J.st->n_surv, r0 = J.st->rounds_run;
    const int htile = blockIdx.x % fw, rt = blockIdx.x / fw;
    const int round = r0 + rt / nptiles, pt = rt % nptiles;
    if (htile * 64 >= n || round >= rounds_of(n, J.n_cull, J.n_out, r0)) return;
    int H = 64;
    while (H > 1 && (H >> 1) >= n) H >>= 1;
    const int G = 64 / H, lane = (int)threadIdx.x;
    if (pt * G * J.TP >= J.eta) return;
    const int ptile = pt * G + lane / H;
    const int k0 = ptile * J.TP;
    if (k0 >= J.eta) return;
    const int tp = min(J.TP, J.eta - k0);
    const int pos = htile * 64 + (lane & (H - 1));
    double R[9], t[3];
    hyp_pose(J.hyps[ldg(J.surv + (pos < n ? pos : 0))], R, t);
    const double acc = score_pixels(J, round, k0, tp, htile == 0 && (lane & (H - 1)) == 0, R, t);
    if (pos < n) J.partial_all[((size_t)round * nptiles + ptile) * kFastStride + pos] = acc;
}

// Those rounds' selections, one block per job, thread = position in the
// survivor list: same accumulation (tile order, rounds in order, onto the
// energies of earlier rounds), ranking by (energy, slot), initial cull and
// halving as k_select.  A round's tile sum does not depend on the ranking,
// so the whole block first forms every (round, position) sum at once, in
// LDS (up to kSelSums of them; any beyond are summed in the ranking loop, to
// the same value).
constexpr int kSelSums = 4096;

// At most wr rounds are run; the job is done once its survivors are down to
// n_out.
__global__ __launch_bounds__(kFastStride) void k_select_all(const Job* __restrict__ jobs, int nptiles, int wr)
{
    const Job& J = jobs[blockIdx.x];
    if (J.st->done || J.lm) return;
    __shared__ double sE[kFastStride];
    __shared__ int sS[kFastStride], sA[kFastStride];
    __shared__ double sSum[kSelSums];
    const int n0 = J.st->n_surv, r0 = J.st->rounds_run;
    const int lane = (int)threadIdx.x;
    const int ptiles = min(nptiles, (J.eta + J.TP - 1) / J.TP);
    const int r_end = min(rounds_of(n0, J.n_cull, J.n_out, r0), r0 + wr);
    const int nsum = min((r_end - r0) * n0, kSelSums);
    for (int i = lane; i < nsum; i += kFastStride) {
        const int rr = i / n0, pos = i - rr * n0;
        sSum[i] = sum_in_order<32>(J.partial_all + (size_t)(r0 + rr) * nptiles * kFastStride + pos, kFastStride,
                                   ptiles);
    }
    __syncthreads();
    const bool valid = lane < n0;
    const int slot = valid ? ldg(J.surv + lane) : INT_MAX;
    double E = valid ? J.E[slot] : 0.0;
    bool alive = valid;
    int n = n0, round = r0, rank = 0;
    bool first = round == 0;
    while ((first || n > J.n_out) && round < r_end) {
        if (alive) {
            const int i = (round - r0) * n0 + lane;
            E = E + (i < nsum ? sSum[i]
                              : sum_in_order(J.partial_all + (size_t)round * nptiles * kFastStride + lane,
                                             kFastStride, ptiles));
        }
        const double key = isnan(E) ? INFINITY : E;
        sE[lane] = key;
        sS[lane] = slot;
        sA[lane] = alive ? 1 : 0;
        __syncthreads();
        const int keep = (first && J.n_cull < n) ? J.n_cull : (n > J.n_out ? (n + 1) / 2 : n);
        rank = 0;
        if (alive)
            for (int q = 0; q < n0; ++q)
                rank += (sA[q] && (sE[q] < key || (sE[q] == key && sS[q] < slot))) ? 1 : 0;
        if (alive && rank < keep) {
            if (J.trace) {
                J.trace_slots[(size_t)round * J.N + rank] = slot;
                J.trace_E[(size_t)round * J.N + rank] = key;
            }
        } else {
            alive = false;
        }
        __syncthreads();
        n = keep;
        ++round;
        first = false;
    }
    if (alive) {
        J.surv[rank] = slot;
        J.E[slot] = E;
    }
    if (lane == 0) {
        J.st->n_surv = n;
        J.st->rounds_run = round;
        J.st->done = (first || n > J.n_out) ? 0 : 1;
    }
}

// ------------------------------------------------------------------------
// Levenberg-Marquardt refinement in se(3) (Sec. 3.2.3, step (ii) of every
// preemptive-RANSAC iteration after the first): each survivor's E of Eq. 5
// over the whole cumulative I is minimised from its pose so far.  Each
// iteration linearises at the current pose: per pixel the nearest mode
// (ties to the lower index in M(u)), residual r = H x - mu, e = |r|_A
// (A = Sigma^-1, or I without the covariance), the Jacobian J = [-[y]x | I]
// of exp(xi^) y at xi = 0 and the weight 1 / max(e, 1e-6), whose normal
// equations N d = -g share E's gradient.  The step solves
// (N + lambda diag N) d = -g by Cholesky (a non-positive pivot rejects it);
// exp(d^) H is accepted iff its energy is lower (lambda / 10), else
// lambda * 10; lambda starts at 1e-3.  The survivor's energy becomes E at
// the final pose.
//
// The work is spread over the grid: a pass evaluates (E, g, N) for every
// survivor of every job at once, one wave per (survivor, one or two
// kLmTile-pixel tiles) writing each tile's partial sums; a step kernel (one wave per survivor)
// adds the tiles in order, takes the accept/reject decision and the next
// damped step.  Both stride over the round's plan of the running jobs'
// items and survivors, so their grids do not scale with the batch's
// survivor bound.  Per round: k_lm_draw, k_lm_init, k_lm_plan, then
// (iterations + 1) x (k_lm_pass, k_lm_step).

// per-slot state (doubles): current pose, candidate pose, N (upper), g, E,
// lambda, go (the candidate awaits evaluation)
enum { kLmCur = 0, kLmCand = 12, kLmN = 24, kLmG = 45, kLmE = 51, kLmLambda = 52, kLmGo = 53 };

// list entries of the cumulative I: all of rounds 0 and 1 in round 1, the
// round's own afterwards (the pixels are those the scoring draws)
__global__ __launch_bounds__(256) void k_lm_draw(const Job* __restrict__ jobs, int round)
{
    const Job& J = jobs[blockIdx.y];
    if (!J.lm || J.st->done || J.st->n_elig <= 0) return;
    const int k = (round == 1 ? 0 : round * J.eta) + (int)(blockIdx.x * 256 + threadIdx.x);
    if (k >= (round + 1) * J.eta) return;
    const int rk = k / J.eta, kk = k - rk * J.eta;
    const uint4 rb = philox(make_uint4(kTagScore << 28, (uint32_t)rk, (uint32_t)(kk >> 2), 0u), J.key0, J.key1);
    const uint32_t rv = (kk & 3) == 0 ? rb.x : (kk & 3) == 1 ? rb.y : (kk & 3) == 2 ? rb.z : rb.w;
    const uint32_t e = below(rv, (uint32_t)J.st->n_elig);
    const uint4 c0 = ldg(J.ecold + 2 * e);
    const int p = (int)c0.x;
    J.Ie[k] = (int)e;
    J.I[k] = p;
    // the pixel's camera point and |M(u)|; k_lm_rows stages its rows
    double x[3];
    backproject(__uint_as_float(c0.y), p % J.w, p / J.w, J.fx, J.fy, J.cx, J.cy, x);
    J.lm_px[k] = make_double4(x[0], x[1], x[2], (double)modes_total(make_uint2(c0.z, c0.w), J.T));
}

// The rows of M(u) (mean, Sigma^-1: the first 48 bytes of each mode row) of
// the pixels k_lm_draw added, flattened tree-major into an array indexed
// [row][16-byte part][pixel of I] (lm_split: each 16-byte load of a pass
// reads consecutive addresses across a wave's pixels; faster for one frame)
// or [row][pixel of I][16-byte part] (a row's three loads share cache lines;
// faster for many frames).  The results do not depend on it.  Thread
// (k, g) copies rows 4g .. 4g + 3 of pixel k (grid: pixels / 64, row
// groups, jobs), so a pixel's rows are copied in parallel and the stores of
// one row index are contiguous across a wave.
constexpr int kLmRowsPerThread = 4;
__global__ __launch_bounds__(64) void k_lm_rows(const Job* __restrict__ jobs, int round)
{
    const Job& J = jobs[blockIdx.z];
    if (!J.lm || J.st->done || J.st->n_elig <= 0) return;
    const int k = (round == 1 ? 0 : round * J.eta) + (int)(blockIdx.x * 64 + threadIdx.x);
    if (k >= (round + 1) * J.eta) return;
    const int e = J.Ie[k];
    const uint4 c0 = ldg(J.ecold + 2 * e), lw = ldg(J.ecold + 2 * e + 1);
    const uint2 nw = make_uint2(c0.z, c0.w);
    const int m0 = (int)blockIdx.y * kLmRowsPerThread, total = modes_total(nw, J.T);
    if (m0 >= total) return;
    const int n = min(kLmRowsPerThread, total - m0);
    const int ks = J.lm_split ? 1 : 3, ps = J.lm_split ? J.lm_icap : 1;
    ModeWalk mw(J, lw, nw, m0);
    float4 r[kLmRowsPerThread][3];
#pragma unroll
    for (int u = 0; u < kLmRowsPerThread; ++u) {
        if (u < n) {
            const float4* row = J.modes + (size_t)mw.row() * 4;
            r[u][0] = ldg(row);
            r[u][1] = ldg(row + 1);
            r[u][2] = ldg(row + 2);
            if (u + 1 < n) mw.next();
        }
    }
#pragma unroll
    for (int u = 0; u < kLmRowsPerThread; ++u) {
        if (u < n) {
            float4* dst = J.lm_rows + (size_t)(m0 + u) * 3 * J.lm_icap + (size_t)k * ks;
            dst[0] = r[u][0];
            dst[ps] = r[u][1];
            dst[2 * ps] = r[u][2];
        }
    }
}

__global__ __launch_bounds__(256) void k_lm_init(const Job* __restrict__ jobs, int round)
{
    const Job& J = jobs[blockIdx.y];
    const int pos = blockIdx.x * 256 + threadIdx.x;
    if (!J.lm || J.st->done || pos >= J.st->n_surv) return;
    const int slot = J.surv[pos];
    double* S = J.lm_state + (size_t)slot * kLmStateDoubles;
    for (int i = 0; i < 12; ++i) {
        const double v = round == 1 ? (double)(i < 9 ? J.hyps[slot].R[i] : J.hyps[slot].t[i - 9])
                                    : J.pose64[12 * (size_t)slot + i];
        S[kLmCur + i] = v;
        S[kLmCand + i] = v;
    }
    S[kLmLambda] = 1e-3;
    S[kLmGo] = 1.0;
}

template <bool COV, int PAIR, bool SPLIT>
__device__ __forceinline__ void lm_pass_item(const Job& J, int pos, int tile, int tiles, int nI);

// Work plan of a round (one block), over the jobs with LM still running:
// plan[j] = first (survivor, tile) item of job j and plan[njobs] = their
// total; splan = plan + kMaxBatchFrames + 1 likewise numbers the survivors.
__global__ __launch_bounds__(1024) void k_lm_plan(const Job* __restrict__ jobs, int njobs, int round, int tpw)
{
    __shared__ int s_x[1024], s_y[1024];
    int* plan = jobs[0].lm_plan;
    int* splan = plan + kMaxBatchFrames + 1;
    int carry = 0, scarry = 0;
    for (int base = 0; base < njobs; base += 1024) {
        const int j = base + (int)threadIdx.x;
        int items = 0, surv = 0;
        if (j < njobs) {
            const Job& J = jobs[j];
            if (J.lm && !J.st->done) {
                surv = J.st->n_surv;
                items = surv * ((((round + 1) * J.eta + kLmTile - 1) / kLmTile + tpw - 1) / tpw);
            }
        }
        s_x[threadIdx.x] = items;
        s_y[threadIdx.x] = surv;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {           // inclusive scans
            const int ax = (int)threadIdx.x >= o ? s_x[threadIdx.x - o] : 0;
            const int ay = (int)threadIdx.x >= o ? s_y[threadIdx.x - o] : 0;
            __syncthreads();
            s_x[threadIdx.x] += ax;
            s_y[threadIdx.x] += ay;
            __syncthreads();
        }
        if (j < njobs) {
            plan[j] = carry + s_x[threadIdx.x] - items;
            splan[j] = scarry + s_y[threadIdx.x] - surv;
        }
        carry += s_x[1023];
        scarry += s_y[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        plan[njobs] = carry;
        splan[njobs] = scarry;
    }
}

// index of the last job whose first plan entry is <= g (plan ascending)
__device__ __forceinline__ int plan_job(const int* plan, int njobs, int g)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (plan[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// 1-D grid of waves striding over the plan's items of all jobs, so that a
// job with many survivors gets as many waves as its items need.  An item is
// tpw (1 or 2) consecutive tiles of one survivor, whose partials do not
// depend on tpw (lm_pass_item).  The pass
// waits on its row loads, so it is held to 128 VGPRs (four waves per SIMD;
// a few values spill) with two rows in flight: faster than two waves per SIMD
// with four rows in flight (190 VGPRs), or than three waves (142).
template <int PAIR, bool SPLIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_lm_pass(
    const Job* __restrict__ jobs, int njobs, int round)
{
#pragma clang fp contract(off)
    constexpr int tpw = PAIR ? 2 : 1;
    const int* plan = jobs[0].lm_plan;
    const int total = plan[njobs];
    // workgroup w runs on XCD w % 8 (gridDim.x is a multiple of 8): XCD e
    // takes the e-th eighth of the items in order, so the mode rows of the
    // few frames it works on stay in its L2 while their survivors read them
    const int e = (int)blockIdx.x & 7, per = (int)gridDim.x >> 3;
    const int chunk = (total + 7) >> 3, g1 = min(total, (e + 1) * chunk);
    for (int gi = e * chunk + ((int)blockIdx.x >> 3); gi < g1; gi += per) {
        const int lo = plan_job(plan, njobs, gi);
        const Job& J = jobs[lo];
        const int nI = (round + 1) * J.eta;
        const int tiles = (nI + kLmTile - 1) / kLmTile, groups = (tiles + tpw - 1) / tpw;
        const int item = gi - plan[lo];
        const int pos = item / groups, t0 = (item % groups) * tpw;
        if (J.use_cov) lm_pass_item<true, PAIR, SPLIT>(J, pos, t0, tiles, nI);
        else lm_pass_item<false, PAIR, SPLIT>(J, pos, t0, tiles, nI);
    }
}

// The partial of a tile is the sum over its 64 pixels of the per-pixel
// terms, pixel l and l + 32 added first, then halves, quarters, ... (the
// lane xor tree, lane_tree_sums).  With pair = 0 a wave takes one tile, a pixel per lane;
// with pair = 1 it takes tiles tile and tile + 1, lanes 0-31 and 32-63, each
// lane adding pixel l and then pixel l + 32 of its tile, which is the tree's
// first level, so both forms give the same partials bit for bit.
// One level of a lane tree over H pairs of values: a lane whose bit O is
// clear keeps values 0..H-1 and hands H..2H-1 to lane ^ O, which keeps
// those; each kept value becomes its own copy plus the partner's.
template <int H, int O>
__device__ __forceinline__ void tree_level(double* w, int lane)
{
    const bool hi = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = hi ? w[i] : w[H + i];
        const double keep = hi ? w[H + i] : w[i];
        w[i] = keep + __shfl_xor(send, O);
    }
}

// Sums of v[0..27] over the lane xor tree o = O0, O0 / 2, ..., 1 (O0 = 16:
// each lane half on its own; 32: the whole wave).  Every sum adds the same
// two operands at every level as a butterfly that adds all values at every
// level, so the sums are the same bits; a level here halves the values a
// lane carries.  Lane l ends with sum (l & 31) (O0 = 16) or ((l >> 1) & 31)
// (O0 = 32; lanes l and l ^ 1 alike); sums 28..31 are padding.
template <int O0>
__device__ __forceinline__ double lane_tree_sums(const double* v, int lane)
{
    double w[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) w[i] = i < kLmVals ? v[i] : 0.0;
    tree_level<16, O0>(w, lane);
    tree_level<8, O0 / 2>(w, lane);
    tree_level<4, O0 / 4>(w, lane);
    tree_level<2, O0 / 8>(w, lane);
    tree_level<1, O0 / 16>(w, lane);
    return O0 == 32 ? w[0] + __shfl_xor(w[0], 1) : w[0];
}

template <bool COV, int PAIR, bool SPLIT>
__device__ __forceinline__ void lm_pass_item(const Job& J, int pos, int tile, int tiles, int nI)
{
#pragma clang fp contract(off)
    const int slot = J.surv[pos];
    const double* S = J.lm_state + (size_t)slot * kLmStateDoubles;
    if (S[kLmGo] == 0.0) return;
    double P[12];
    for (int i = 0; i < 12; ++i) P[i] = S[kLmCand + i];
    double v[kLmVals];
    for (int i = 0; i < kLmVals; ++i) v[i] = 0.0;
    const int lane = (int)threadIdx.x;
    const int my_tile = PAIR ? tile + (lane >> 5) : tile;
    const int ks = SPLIT ? 1 : 3, ps = SPLIT ? J.lm_icap : 1;   // lm_rows strides (SPLIT = J.lm_split)
#pragma unroll
    for (int j = 0; j < (PAIR ? 2 : 1); ++j) {
        const int k = PAIR ? my_tile * 64 + (lane & 31) + 32 * j : tile * 64 + lane;
        if (my_tile >= tiles || k >= nI) break;
        const double4 px = ldg(J.lm_px + k);
        const double x[3] = {px.x, px.y, px.z};
        const int nm = (int)px.w;
        const double y0 = P[0] * x[0] + P[1] * x[1] + P[2] * x[2] + P[9];
        const double y1 = P[3] * x[0] + P[4] * x[1] + P[5] * x[2] + P[10];
        const double y2 = P[6] * x[0] + P[7] * x[1] + P[8] * x[2] + P[11];
        // nearest mode (ties to the lower index) over the staged rows, two at
        // a time.  With two tiles per wave (many waves in flight) the best
        // row is kept in registers; with one (few waves, whose added load
        // latency costs less than the copies) it is loaded again after the scan.
        double best = INFINITY;
        int bj = -1;
        float4 ba = make_float4(0.f, 0.f, 0.f, 0.f), bb = ba, bc = ba;
        for (int j0 = 0; j0 < nm; j0 += 2) {
            float4 ra[2], rb[2], rc[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int j = min(j0 + u, nm - 1);
                const float4* row = J.lm_rows + (size_t)j * 3 * J.lm_icap + (size_t)k * ks;
                ra[u] = ldg(row);
                if (COV) {
                    rb[u] = ldg(row + ps);
                    rc[u] = ldg(row + 2 * ps);
                } else {
                    rb[u] = rc[u] = ra[u];
                }
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                if (j0 + u >= nm) break;
                double qq = row_q<COV>(ra[u], rb[u], rc[u], y0, y1, y2);
                qq = qq < 0.0 ? 0.0 : qq;
                if (qq < best) {
                    best = qq;
                    bj = j0 + u;
                    if (PAIR) {
                        ba = ra[u];
                        bb = rb[u];
                        bc = rc[u];
                    }
                }
            }
        }
        const double en = sqrt(best);
        v[0] += en;
        if (bj < 0) continue;
        if (!PAIR) {
            const float4* brow = J.lm_rows + (size_t)bj * 3 * J.lm_icap + (size_t)k * ks;
            ba = ldg(brow);
            bb = COV ? ldg(brow + ps) : ba;
            bc = COV ? ldg(brow + 2 * ps) : ba;
        }
        const double r0 = y0 - (double)ba.x, r1 = y1 - (double)ba.y, r2 = y2 - (double)ba.z;
        double A[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
        if (COV) {
            A[0] = bb.x; A[1] = bb.y; A[2] = bb.z;
            A[3] = bb.y; A[4] = bb.w; A[5] = bc.x;
            A[6] = bb.z; A[7] = bc.x; A[8] = bc.y;
        }
        const double Jm[18] = {0.0, y2, -y1, 1.0, 0.0, 0.0,
                               -y2, 0.0, y0, 0.0, 1.0, 0.0,
                               y1, -y0, 0.0, 0.0, 0.0, 1.0};
        double AJ[18], Ar[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Ar[q] = A[3 * q] * r0 + A[3 * q + 1] * r1 + A[3 * q + 2] * r2;
#pragma unroll
            for (int jj = 0; jj < 6; ++jj)
                AJ[6 * q + jj] = A[3 * q] * Jm[jj] + A[3 * q + 1] * Jm[6 + jj] + A[3 * q + 2] * Jm[12 + jj];
        }
        const double wgt = 1.0 / (en > 1e-6 ? en : 1e-6);
        int o = 7;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            v[1 + i] += wgt * (Jm[i] * Ar[0] + Jm[6 + i] * Ar[1] + Jm[12 + i] * Ar[2]);
#pragma unroll
            for (int jj = i; jj < 6; ++jj)
                v[o++] += wgt * (Jm[i] * AJ[jj] + Jm[6 + i] * AJ[6 + jj] + Jm[12 + i] * AJ[12 + jj]);
        }
    }
    const double sum = lane_tree_sums<PAIR ? 16 : 32>(v, lane);
    const int idx = PAIR ? (lane & 31) : ((lane >> 1) & 31);
    if (idx < kLmVals && (PAIR || (lane & 1) == 0) && my_tile < tiles)
        J.lm_part[((size_t)pos * tiles + my_tile) * kLmVals + idx] = sum;
}

// M d = b for a symmetric positive definite 6x6 M; false on a pivot that is
// not positive and finite
__device__ bool chol6_solve(const double M[36], const double b[6], double d[6])
{
    double L[36];
    for (int i = 0; i < 36; ++i) L[i] = 0.0;
    for (int j = 0; j < 6; ++j) {
        double s = M[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0) || !isfinite(s)) return false;
        L[6 * j + j] = sqrt(s);
        for (int i = j + 1; i < 6; ++i) {
            double u = M[6 * i + j];
            for (int k = 0; k < j; ++k) u -= L[6 * i + k] * L[6 * j + k];
            L[6 * i + j] = u / L[6 * j + j];
        }
    }
    double z[6];
    for (int i = 0; i < 6; ++i) {
        double u = b[i];
        for (int k = 0; k < i; ++k) u -= L[6 * i + k] * z[k];
        z[i] = u / L[6 * i + i];
    }
    for (int i = 5; i >= 0; --i) {
        double u = z[i];
        for (int k = i + 1; k < 6; ++k) u -= L[6 * k + i] * d[k];
        d[i] = u / L[6 * i + i];
    }
    return true;
}

// exp of xi = (omega, v): R = I + A W + B W^2, t = (I + B W + C W^2) v, with
// A = sin(th)/th, B = (1 - cos th)/th^2, C = (th - sin th)/th^3 (Taylor
// series to th^4 below th = 1e-2)
__device__ void se3_exp(const double xi[6], double Rd[9], double td[3])
{
#pragma clang fp contract(off)
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double th2 = wx * wx + wy * wy + wz * wz;
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-2) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (1.0 - A) / th2;
    }
    const double W[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double W2[9], V[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
    for (int i = 0; i < 9; ++i) {
        const double id = (i % 4 == 0) ? 1.0 : 0.0;
        Rd[i] = id + A * W[i] + B * W2[i];
        V[i] = id + B * W[i] + C * W2[i];
    }
    for (int i = 0; i < 3; ++i) td[i] = V[3 * i] * xi[3] + V[3 * i + 1] * xi[4] + V[3 * i + 2] * xi[5];
}

// lane 0 of a survivor's step: accept or reject the evaluated candidate,
// then the next damped step (or, after the last iteration, the outputs)
__device__ __forceinline__ void lm_decide(const Job& J, int slot, double* S, bool go, int it, const double* s_v)
{
#pragma clang fp contract(off)
    double lambda = S[kLmLambda];
    if (go) {
        double v[kLmVals];
        for (int i = 0; i < kLmVals; ++i) v[i] = s_v[i];
        if (it < 0 || v[0] < S[kLmE]) {
            S[kLmE] = v[0];
            for (int i = 0; i < 21; ++i) S[kLmN + i] = v[7 + i];
            for (int i = 0; i < 6; ++i) S[kLmG + i] = v[1 + i];
            for (int i = 0; i < 12; ++i) S[kLmCur + i] = S[kLmCand + i];
            if (it >= 0) lambda /= 10.0;
        } else {
            lambda *= 10.0;
        }
    }
    if (it == J.lm_iters - 1) {
        for (int i = 0; i < 12; ++i) J.pose64[12 * (size_t)slot + i] = S[kLmCur + i];
        for (int i = 0; i < 9; ++i) J.hyps[slot].R[i] = (float)S[kLmCur + i];
        for (int i = 0; i < 3; ++i) J.hyps[slot].t[i] = (float)S[kLmCur + 9 + i];
        J.E[slot] = S[kLmE];
        S[kLmGo] = 0.0;
        S[kLmLambda] = lambda;
        return;
    }
    // the next damped step from the current pose
    double N[36], M[36], b[6], d[6];
    int o = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) N[6 * i + j] = N[6 * j + i] = S[kLmN + o++];
    for (int i = 0; i < 36; ++i) M[i] = N[i];
    for (int i = 0; i < 6; ++i) {
        M[6 * i + i] = N[6 * i + i] + lambda * N[6 * i + i];
        b[i] = -S[kLmG + i];
    }
    if (chol6_solve(M, b, d)) {
        double Rd[9], td[3];
        se3_exp(d, Rd, td);
        const double* C = S + kLmCur;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j)
                S[kLmCand + 3 * i + j] = Rd[3 * i] * C[j] + Rd[3 * i + 1] * C[3 + j] + Rd[3 * i + 2] * C[6 + j];
            S[kLmCand + 9 + i] = Rd[3 * i] * C[9] + Rd[3 * i + 1] * C[10] + Rd[3 * i + 2] * C[11] + td[i];
        }
        S[kLmGo] = 1.0;
    } else {
        lambda *= 10.0;
        S[kLmGo] = 0.0;
    }
    S[kLmLambda] = lambda;
}

// One survivor's step: lanes 0..27 add one value each over the tiles in
// order, lane 0 decides.  it = -1 follows the pass at the starting pose;
// it >= 0 follows iteration it's candidate pass.  The last iteration writes
// the refined pose (FP64, and rounded into the hypothesis table) and the
// energy.
__device__ __forceinline__ void lm_step_one(const Job& J, int pos, int round, int it, double* s_v)
{
#pragma clang fp contract(off)
    const int slot = J.surv[pos];
    double* S = J.lm_state + (size_t)slot * kLmStateDoubles;
    const bool go = S[kLmGo] != 0.0;
    if (go && threadIdx.x < kLmVals) {
        const int tiles = ((round + 1) * J.eta + kLmTile - 1) / kLmTile;
        s_v[threadIdx.x] = sum_in_order(J.lm_part + (size_t)pos * tiles * kLmVals + threadIdx.x, kLmVals, tiles);
    }
    __syncthreads();
    if (threadIdx.x == 0) lm_decide(J, slot, S, go, it, s_v);
    __syncthreads();
}

// 1-D grid of waves striding over the survivors of every job with LM (the
// round's survivor plan).
__global__ __launch_bounds__(64) void k_lm_step(const Job* __restrict__ jobs, int njobs, int round, int it)
{
    __shared__ double s_v[kLmVals];
    const int* splan = jobs[0].lm_plan + kMaxBatchFrames + 1;
    const int total = splan[njobs];
    for (int gi = blockIdx.x; gi < total; gi += gridDim.x) {
        const int lo = plan_job(splan, njobs, gi);
        const Job& J = jobs[lo];
        if (it >= J.lm_iters) continue;
        lm_step_one(J, gi - splan[lo], round, it, s_v);
    }
}

// Adds the round's partial sums (tile order), ranks survivors by
// (energy, slot) and keeps the initial cull or the better half.
__global__ __launch_bounds__(1024) void k_select(const Job* __restrict__ jobs, int round, int nptiles)
{
    const Job& J = jobs[blockIdx.y];
    if (J.st->done || (!J.lm && J.st->n_surv <= J.fast_max)) return;
    // after an LM round the energies are already over the whole cumulative I
    const bool add = !(J.lm && round > 0);
    extern __shared__ unsigned char s_raw[];
    const int n = J.st->n_surv;
    double* sE = reinterpret_cast<double*>(s_raw);
    int* sS = reinterpret_cast<int*>(s_raw + sizeof(double) * (size_t)J.N);
    const int ptiles = min(nptiles, (J.eta + J.TP - 1) / J.TP);
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const int s = J.surv[p];
        const double e = add ? J.E[s] + sum_in_order(J.partial + p, (size_t)J.N, ptiles) : J.E[s];
        J.E[s] = e;
        sE[p] = isnan(e) ? INFINITY : e;
        sS[p] = s;
    }
    __syncthreads();
    int keep;
    if (round == 0 && J.n_cull < n) keep = J.n_cull;
    else if (n > J.n_out) keep = (n + 1) / 2;
    else keep = n;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        const double e = sE[p];
        const int s = sS[p];
        int rank = 0;
        for (int q = 0; q < n; ++q) {
            const double eq = sE[q];
            rank += (eq < e || (eq == e && sS[q] < s)) ? 1 : 0;
        }
        if (rank < keep) {
            J.surv[rank] = s;
            if (J.trace) {
                J.trace_slots[(size_t)round * J.N + rank] = s;
                J.trace_E[(size_t)round * J.N + rank] = e;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        J.st->n_surv = keep;
        J.st->rounds_run = round + 1;
        J.st->done = keep <= J.n_out ? 1 : 0;
    }
}

// ------------------------------------------------------------------------
// Refit, part 1 (one thread per pixel of the final set I): the mode of M(u)
// minimising the Eq. 5 distance under the winner's pose (ties -> lower m),
// then the Euclidean inlier test.  J.inl[k] = that mode's row, or -1.  The
// modes are walked tree by tree in M(u) order, four rows loaded ahead of
// their comparisons.
__global__ __launch_bounds__(256) void k_refit_assign(const Job* __restrict__ jobs)
{
#pragma clang fp contract(off)
    const Job& J = jobs[blockIdx.y];
    if (!J.final_refine) return;
    const int n = J.st->n_surv, rounds = J.st->rounds_run;
    const int nI = rounds * J.eta;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (n <= 0 || k >= nI) return;
    const Hyp& hy = J.hyps[J.surv[0]];
    double R[9], t[3];
    for (int i = 0; i < 9; ++i) R[i] = hy.R[i];
    for (int i = 0; i < 3; ++i) t[i] = hy.t[i];
    const int p = J.I[k];
    double x[3];
    backproject(__uint_as_float(J.probe[p]), p % J.w, p / J.w, J.fx, J.fy, J.cx, J.cy, x);
    const double y0 = R[0] * x[0] + R[1] * x[1] + R[2] * x[2] + t[0];
    const double y1 = R[3] * x[0] + R[4] * x[1] + R[5] * x[2] + t[1];
    const double y2 = R[6] * x[0] + R[7] * x[1] + R[8] * x[2] + t[2];
    const uint4 lw = reinterpret_cast<const uint4*>(J.leaves)[p];
    const uint2 nw = reinterpret_cast<const uint2*>(J.nmt)[p];
    const bool cov = J.use_cov != 0;
    double best = INFINITY;
    int bri = -1;
    for (int tr = 0; tr < J.T; ++tr) {
        const int c = (int)count_of(nw, tr);
        const uint32_t base = (((uint32_t)tr << J.D) + leaf_of(lw, tr)) * (uint32_t)J.M;
        for (int j0 = 0; j0 < c; j0 += 4) {
            float4 ra[4], rb[4], rc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const float4* row = J.modes + (size_t)(base + (uint32_t)min(j0 + u, c - 1)) * 4;
                ra[u] = ldg(row);
                if (cov) {
                    rb[u] = ldg(row + 1);
                    rc[u] = ldg(row + 2);
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (j0 + u >= c) break;
                const float4 a = ra[u];
                const double d0 = y0 - a.x, d1 = y1 - a.y, d2 = y2 - a.z;
                double q;
                if (cov) {
                    const float4 b = rb[u], cc = rc[u];
                    q = d0 * (b.x * d0 + b.y * d1 + b.z * d2) + d1 * (b.y * d0 + b.w * d1 + cc.x * d2)
                      + d2 * (b.z * d0 + cc.x * d1 + cc.y * d2);
                } else {
                    q = d0 * d0 + d1 * d1 + d2 * d2;
                }
                q = fmax(q, 0.0);
                if (q < best) {
                    best = q;
                    bri = (int)(base + (uint32_t)(j0 + u));
                }
            }
        }
    }
    int flag = -1;
    if (bri >= 0) {
        const float4 a = J.modes[(size_t)bri * 4];
        const double d0 = y0 - a.x, d1 = y1 - a.y, d2 = y2 - a.z;
        if (sqrt(d0 * d0 + d1 * d1 + d2 * d2) <= J.theta_in) flag = bri;
    }
    J.inl[k] = flag;
}

// Sums of NV values over a block of kFinThreads threads in a fixed order:
// within each wave by an xor tree, then the waves' sums in wave order.
constexpr int kFinThreads = 1024;

template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* s_red)
{
    constexpr int W = kFinThreads / 64;
    const int lane = (int)threadIdx.x & 63, wave = (int)threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lane == 0) s_red[i * W + wave] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < NV) {
        double x = 0.0;
        for (int w = 0; w < W; ++w) x += s_red[threadIdx.x * W + w];
        s_red[NV * W + threadIdx.x] = x;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = s_red[NV * W + i];
    __syncthreads();
}

// The inlier pairs (x^C, mode mean) of kFinChunk consecutive positions of a
// thread (k, k + kFinThreads, ...): every gather of the chunk is issued
// before the pairs are used.  ok[u] = position k + kFinThreads u is an inlier.
constexpr int kFinChunk = 4;

__device__ __forceinline__ void inlier_chunk(const Job& J, int k, int nI, bool ok[kFinChunk],
                                             double x[kFinChunk][3], float4 a[kFinChunk])
{
    int ri[kFinChunk], p[kFinChunk];
#pragma unroll
    for (int u = 0; u < kFinChunk; ++u) ri[u] = k + kFinThreads * u < nI ? J.inl[k + kFinThreads * u] : -1;
#pragma unroll
    for (int u = 0; u < kFinChunk; ++u) p[u] = ri[u] >= 0 ? J.I[k + kFinThreads * u] : 0;
    float d[kFinChunk];
#pragma unroll
    for (int u = 0; u < kFinChunk; ++u) {
        ok[u] = ri[u] >= 0;
        d[u] = ok[u] ? __uint_as_float(J.probe[p[u]]) : 0.0f;
        a[u] = ok[u] ? J.modes[(size_t)ri[u] * 4] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < kFinChunk; ++u) backproject(d[u], p[u] % J.w, p[u] / J.w, J.fx, J.fy, J.cx, J.cy, x[u]);
}

// Refit, part 2 and the result record: centroids and cross-covariance of the
// inlier pairs (x^C, mode mean), Kabsch over all of them (>= 3 inliers).
// Each thread accumulates its positions in increasing order.
__global__ __launch_bounds__(kFinThreads) void k_finalize(const Job* __restrict__ jobs)
{
#pragma clang fp contract(off)
    const Job& J = jobs[blockIdx.y];
    __shared__ double s_red[9 * (kFinThreads / 64 + 1)];
    __shared__ double s_pose[12];
    __shared__ int s_refit;
    rl_result* res = J.result;
    const int n = J.st->n_surv;
    const int rounds = J.st->rounds_run;
    if (n <= 0 || rounds <= 0) {
        if (threadIdx.x < 16) res->cam_to_world[threadIdx.x] = (threadIdx.x % 5 == 0) ? 1.0f : 0.0f;
        if (threadIdx.x == 0) {
            res->energy = INFINITY;
            res->mean_energy = INFINITY;
            res->status = RL_NO_POSE;
            res->n_valid = J.st->n_valid;
            res->n_inliers = 0;
            res->winner = -1;
            res->refitted = 0;
            res->n_eligible = J.st->n_elig;
            res->rounds = rounds;
            res->n_out = 0;
            res->mode_version = J.mode_version;
        }
        return;
    }
    const int win = J.surv[0];
    const Hyp& hy = J.hyps[win];
    if (threadIdx.x < 9) s_pose[threadIdx.x] = hy.R[threadIdx.x];
    if (threadIdx.x < 3) s_pose[9 + threadIdx.x] = hy.t[threadIdx.x];
    if (threadIdx.x == 0) s_refit = 0;
    __syncthreads();
    const int nI = rounds * J.eta;
    int n_inl = 0;
    if (J.final_refine) {
        // count, sum of x^C, sum of the mode means
        double c7[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int k = threadIdx.x; k < nI; k += kFinThreads * kFinChunk) {
            bool ok[kFinChunk];
            double x[kFinChunk][3];
            float4 a[kFinChunk];
            inlier_chunk(J, k, nI, ok, x, a);
#pragma unroll
            for (int u = 0; u < kFinChunk; ++u) {
                if (!ok[u]) continue;
                c7[0] += 1.0;
                c7[1] += x[u][0]; c7[2] += x[u][1]; c7[3] += x[u][2];
                c7[4] += a[u].x; c7[5] += a[u].y; c7[6] += a[u].z;
            }
        }
        block_sums<7>(c7, s_red);
        const double tc = c7[0];
        double cc[3] = {c7[1], c7[2], c7[3]}, cw[3] = {c7[4], c7[5], c7[6]};
        n_inl = (int)tc;
        if (n_inl >= 3) {
            for (int i = 0; i < 3; ++i) {
                cc[i] /= tc;
                cw[i] /= tc;
            }
            double A[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            for (int k = threadIdx.x; k < nI; k += kFinThreads * kFinChunk) {
                bool ok[kFinChunk];
                double x[kFinChunk][3];
                float4 a[kFinChunk];
                inlier_chunk(J, k, nI, ok, x, a);
#pragma unroll
                for (int u = 0; u < kFinChunk; ++u) {
                    if (!ok[u]) continue;
                    const double wv[3] = {(double)a[u].x - cw[0], (double)a[u].y - cw[1], (double)a[u].z - cw[2]};
                    for (int i = 0; i < 3; ++i)
                        for (int j = 0; j < 3; ++j) A[i * 3 + j] += (x[u][i] - cc[i]) * wv[j];
                }
            }
            block_sums<9>(A, s_red);
            if (threadIdx.x == 0) {
                double R2[9], t2[3];
                if (rigid_from_cov(A, cc, cw, R2, t2)) {
                    for (int i = 0; i < 9; ++i) s_pose[i] = R2[i];
                    for (int i = 0; i < 3; ++i) s_pose[9 + i] = t2[i];
                    s_refit = 1;
                }
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        float* H = res->cam_to_world;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) H[4 * i + j] = (float)s_pose[3 * i + j];
            H[4 * i + 3] = (float)s_pose[9 + i];
        }
        H[12] = H[13] = H[14] = 0.0f;
        H[15] = 1.0f;
        const double e = J.E[win];
        res->energy = (float)e;
        res->mean_energy = (float)(e / (double)nI);
        res->status = RL_OK;
        res->n_valid = J.st->n_valid;
        res->n_inliers = n_inl;
        res->winner = win;
        res->refitted = s_refit;
        res->n_eligible = J.st->n_elig;
        res->rounds = rounds;
        res->n_out = min(n, J.n_out);
        res->mode_version = J.mode_version;
    }
}

// ------------------------------------------------------------------------
// Model-based pose score on an analytic scene (surfaces of 16 floats: p0, n,
// e1, e2, half-extents; half_a <= 0 = infinite plane): per (tile of 1024
// pixels, pose) the sum of nearest-surface distances of H x^C(u) over valid
// pixels, reduced in a fixed order; then the per-pose means.
__global__ __launch_bounds__(256) void k_plane_partial(FrameView src, int w, int h, float fx,
                                                       float fy, float cx, float cy,
                                                       const float* __restrict__ surfaces, int n_surf,
                                                       const float* __restrict__ poses,
                                                       double* __restrict__ partial, int* __restrict__ cnt)
{
    __shared__ float s_surf[64 * 16];
    __shared__ double s_red[256];
    __shared__ int s_cnt[256];
    const int tile = blockIdx.x, pose = blockIdx.y;
    for (int i = threadIdx.x; i < n_surf * 16; i += 256) s_surf[i] = surfaces[i];
    double R[9], t[3];
    for (int i = 0; i < 9; ++i) R[i] = poses[12 * pose + i];
    for (int i = 0; i < 3; ++i) t[i] = poses[12 * pose + 9 + i];
    __syncthreads();
    const int P = w * h;
    double acc = 0.0;
    int c = 0;
    for (int k = 0; k < 4; ++k) {
        const int p = tile * 1024 + k * 256 + threadIdx.x;
        if (p >= P) break;
        const float d = src.d(p % w, p / w);
        if (!depth_ok(d)) continue;
        double x[3];
        backproject(d, p % w, p / w, fx, fy, cx, cy, x);
        const double y0 = R[0] * x[0] + R[1] * x[1] + R[2] * x[2] + t[0];
        const double y1 = R[3] * x[0] + R[4] * x[1] + R[5] * x[2] + t[1];
        const double y2 = R[6] * x[0] + R[7] * x[1] + R[8] * x[2] + t[2];
        double best = INFINITY;
        for (int s = 0; s < n_surf; ++s) {
            const float* S = s_surf + 16 * s;
            const double r0 = y0 - S[0], r1 = y1 - S[1], r2 = y2 - S[2];
            const double cc = r0 * S[3] + r1 * S[4] + r2 * S[5];
            double dist;
            if (S[12] <= 0.0f) {
                dist = fabs(cc);
            } else {
                const double a = r0 * S[6] + r1 * S[7] + r2 * S[8];
                const double b = r0 * S[9] + r1 * S[10] + r2 * S[11];
                const double da = fmax(fabs(a) - (double)S[12], 0.0), db = fmax(fabs(b) - (double)S[13], 0.0);
                dist = sqrt(cc * cc + da * da + db * db);
            }
            best = fmin(best, dist);
        }
        acc += best;
        ++c;
    }
    s_red[threadIdx.x] = acc;
    s_cnt[threadIdx.x] = c;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
            s_red[threadIdx.x] += s_red[threadIdx.x + stride];
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + stride];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(size_t)tile * 64 + pose] = s_red[0];
        if (pose == 0) cnt[tile] = s_cnt[0];
    }
}

// one block per pose: thread i adds tiles i, i + 256, ... in order, then a
// fixed tree over the threads
__global__ __launch_bounds__(256) void k_plane_final(const double* __restrict__ partial,
                                                     const int* __restrict__ cnt, int ntiles,
                                                     double* __restrict__ scores)
{
    __shared__ double s_acc[256];
    __shared__ long long s_c[256];
    const int pose = blockIdx.x, i = threadIdx.x;
    double acc = 0.0;
    long long c = 0;
    for (int t = i; t < ntiles; t += 256) {
        acc += partial[(size_t)t * 64 + pose];
        c += cnt[t];
    }
    s_acc[i] = acc;
    s_c[i] = c;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (i < stride) {
            s_acc[i] += s_acc[i + stride];
            s_c[i] += s_c[i + stride];
        }
        __syncthreads();
    }
    if (i == 0) scores[pose] = s_c[0] > 0 ? s_acc[0] / (double)s_c[0] : INFINITY;
}

// ------------------------------------------------------------------------
// host-side launchers (called by the runtime)
#define RL_CHECK_LAUNCH() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_prep(const Job* jobs, int njobs, int maxN, hipStream_t st)
{
    k_prep<<<dim3((maxN + 255) / 256, njobs), dim3(256), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

template <int TOP>
static hipError_t launch_traverse_top(const Job* jobs, dim3 gp, dim3 blk, int T, hipStream_t st)
{
    switch (T) {
        case 1: k_traverse<1, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 2: k_traverse<2, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 3: k_traverse<3, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 4: k_traverse<4, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 5: k_traverse<5, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 6: k_traverse<6, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 7: k_traverse<7, TOP><<<gp, blk, 0, st>>>(jobs); break;
        case 8: k_traverse<8, TOP><<<gp, blk, 0, st>>>(jobs); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// top: tree levels read from LDS (6 or 8; a launch schedule, same leaves)
hipError_t launch_traverse(const Job* jobs, int njobs, int maxP, int T, int top, hipStream_t st)
{
    const dim3 blk(256), gp((maxP + 255) / 256, njobs);
    k_pack<<<gp, blk, 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    if (top == kTopLevelsMax) return launch_traverse_top<kTopLevelsMax>(jobs, gp, blk, T, st);
    if (top == kTopLevelsMin) return launch_traverse_top<kTopLevelsMin>(jobs, gp, blk, T, st);
    return hipErrorInvalidValue;
}

hipError_t launch_eligible(const Job* jobs, int njobs, int maxP, int T, hipStream_t st)
{
    k_tile_scan<<<dim3(njobs), dim3(1024), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    const dim3 g((maxP + 255) / 256, njobs), b(256);
    switch (T) {
        case 1: k_eligible<1><<<g, b, 0, st>>>(jobs); break;
        case 2: k_eligible<2><<<g, b, 0, st>>>(jobs); break;
        case 3: k_eligible<3><<<g, b, 0, st>>>(jobs); break;
        case 4: k_eligible<4><<<g, b, 0, st>>>(jobs); break;
        case 5: k_eligible<5><<<g, b, 0, st>>>(jobs); break;
        case 6: k_eligible<6><<<g, b, 0, st>>>(jobs); break;
        case 7: k_eligible<7><<<g, b, 0, st>>>(jobs); break;
        case 8: k_eligible<8><<<g, b, 0, st>>>(jobs); break;
        default: return hipErrorInvalidValue;
    }
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_hyp_search(const Job* jobs, int njobs, int maxN, int maxIters, int ipt, hipStream_t st)
{
    const long long chunks = (maxIters + 256LL * ipt - 1) / (256LL * ipt);
    const long long X = chunks * (long long)maxN;
    const int s = njobs >= 8 ? 1 : njobs >= 4 ? 2 : njobs >= 2 ? 4 : 8;
    const long long per_group = X * ((njobs + 8 / s - 1) / (8 / s));
    const long long grid = 8 * ((per_group + s - 1) / s);
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 g((unsigned)grid), b(256);
    switch (ipt) {
        case 2: k_hyp_search<2><<<g, b, 0, st>>>(jobs, maxN, njobs, (int)X, s); break;
        case 4: k_hyp_search<4><<<g, b, 0, st>>>(jobs, maxN, njobs, (int)X, s); break;
        case 8: k_hyp_search<8><<<g, b, 0, st>>>(jobs, maxN, njobs, (int)X, s); break;
        default: return hipErrorInvalidValue;
    }
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_hyp_finalize(const Job* jobs, int njobs, int maxN, hipStream_t st)
{
    k_hyp_finalize<<<dim3((maxN + 255) / 256, njobs), dim3(256), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_ransac_init<<<dim3(1, njobs), dim3(256), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_score(const Job* jobs, int njobs, int round, int nptiles, int maxSurv, hipStream_t st)
{
    const int htiles = (maxSurv + 63) / 64;
    k_score<<<dim3(nptiles * htiles, njobs), dim3(64), 0, st>>>(jobs, round, nptiles);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_lm(const Job* jobs, int njobs, int round, int maxSurv, int maxEta, int maxRows, int maxIters,
                     bool split, hipStream_t st)
{
    if (maxSurv < 1) return hipSuccess;
    const dim3 thr((maxSurv + 255) / 256, njobs);
    k_lm_draw<<<dim3((2 * maxEta + 255) / 256, njobs), dim3(256), 0, st>>>(jobs, round);
    RL_CHECK_LAUNCH();
    k_lm_rows<<<dim3((2 * maxEta + 63) / 64, (maxRows + kLmRowsPerThread - 1) / kLmRowsPerThread, njobs), dim3(64),
                0, st>>>(jobs, round);
    RL_CHECK_LAUNCH();
    k_lm_init<<<thr, dim3(256), 0, st>>>(jobs, round);
    RL_CHECK_LAUNCH();
    // tiles per pass item: one while the round has few (survivor, tile) pairs
    // (one frame: waves are scarce, and shorter ones finish sooner), two for
    // many frames (fewer per-item overheads); the results are the same
    const long long tiles = ((round + 1) * (long long)maxEta + kLmTile - 1) / kLmTile;
    const int tpw = (long long)maxSurv * tiles * njobs > 4096 ? 2 : 1;
    k_lm_plan<<<dim3(1), dim3(1024), 0, st>>>(jobs, njobs, round, tpw);
    RL_CHECK_LAUNCH();
    const long long items = (long long)maxSurv * ((tiles + tpw - 1) / tpw) * njobs;
    const int waves = (int)(std::min<long long>(items, 8192) + 7) / 8 * 8;
    const int step_waves = (int)std::min<long long>((long long)maxSurv * njobs, 1024);
    for (int it = -1; it < maxIters; ++it) {
        if (split) {
            if (tpw == 2) k_lm_pass<1, true><<<dim3(waves), dim3(64), 0, st>>>(jobs, njobs, round);
            else k_lm_pass<0, true><<<dim3(waves), dim3(64), 0, st>>>(jobs, njobs, round);
        } else {
            if (tpw == 2) k_lm_pass<1, false><<<dim3(waves), dim3(64), 0, st>>>(jobs, njobs, round);
            else k_lm_pass<0, false><<<dim3(waves), dim3(64), 0, st>>>(jobs, njobs, round);
        }
        RL_CHECK_LAUNCH();
        k_lm_step<<<dim3(step_waves), dim3(64), 0, st>>>(jobs, njobs, round, it);
        RL_CHECK_LAUNCH();
    }
    return hipSuccess;
}

// window = 0: every remaining round in one pass; else the first `window`
// rounds, then the rest
hipError_t launch_score_all(const Job* jobs, int njobs, int rounds, int nptiles, int fw, int window, hipStream_t st)
{
    if (fw < 1 || fw > kMaxFastWaves || window < 0) return hipErrorInvalidValue;
    const int w0 = (window > 0 && window < rounds) ? window : rounds;
    k_score_all<<<dim3(w0 * nptiles * fw, njobs), dim3(64), 0, st>>>(jobs, nptiles, fw);
    RL_CHECK_LAUNCH();
    k_select_all<<<dim3(njobs), dim3(kFastStride), 0, st>>>(jobs, nptiles, w0);
    RL_CHECK_LAUNCH();
    if (w0 < rounds) {
        k_score_all<<<dim3((rounds - w0) * nptiles * fw, njobs), dim3(64), 0, st>>>(jobs, nptiles, fw);
        RL_CHECK_LAUNCH();
        k_select_all<<<dim3(njobs), dim3(kFastStride), 0, st>>>(jobs, nptiles, rounds);
        RL_CHECK_LAUNCH();
    }
    return hipSuccess;
}

hipError_t launch_select(const Job* jobs, int njobs, int round, int nptiles, int maxN, hipStream_t st)
{
    const size_t sel_lds = (sizeof(double) + sizeof(int)) * (size_t)maxN;
    k_select<<<dim3(1, njobs), dim3(1024), sel_lds, st>>>(jobs, round, nptiles);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_plane_scores(const FrameView& src, int w, int h, float fx, float fy, float cx, float cy,
                               const float* surfaces, int n_surf, const float* poses, int n_poses,
                               double* partial, int* cnt, double* scores, hipStream_t st)
{
    if (n_poses < 1 || n_poses > 64) return hipErrorInvalidValue;
    const int ntiles = (w * h + 1023) / 1024;
    k_plane_partial<<<dim3(ntiles, n_poses), dim3(256), 0, st>>>(src, w, h, fx, fy, cx, cy, surfaces, n_surf,
                                                                  poses, partial, cnt);
    RL_CHECK_LAUNCH();
    k_plane_final<<<dim3(n_poses), dim3(256), 0, st>>>(partial, cnt, ntiles, scores);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_finalize(const Job* jobs, int njobs, int maxIlen, hipStream_t st)
{
    k_refit_assign<<<dim3((maxIlen + 255) / 256, njobs), dim3(256), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_finalize<<<dim3(1, njobs), dim3(kFinThreads), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace rl
