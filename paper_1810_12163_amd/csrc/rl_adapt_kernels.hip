// rl_adapt_kernels.hip -- online forest adaptation and mode finding (gfx950).
//
// Adaptation (Sec. 3.2.2): grid pixels (4i, 4j), i, j >= 1, are routed
// through every tree and their world points enter the reached leaves'
// reservoirs by Algorithm R.  Arrivals at one leaf are processed in the
// canonical order (raster order within a frame), but each arrival's decision
// depends only on its arrival number n (slot n-1 while n <= kappa, else a
// Philox draw keyed by (tree, leaf, n)).  So the kernels compute every
// arrival's n in parallel and resolve "the later arrival wins" for slots
// drawn twice in one frame, with a result independent of scheduling, in time
// linear in the arrivals (a leaf reached by every grid pixel costs no more
// than spread-out leaves):
//   k_ad_items    route, world point
//   k_ad_sort     per (chunk of 1024 grid pixels, tree): stable sort by leaf
//                 in LDS; each item's rank within its leaf's run of the
//                 chunk; each run joins its leaf's list
//   k_ad_runs     per run: the leaf's items in earlier chunks (its list has at
//                 most one run per chunk)
//   k_ad_claim    n = arrivals before the frame + earlier chunks + rank + 1;
//                 the slot; the largest n drawing each (leaf, slot), by
//                 atomicMax in an open-addressing table
//   k_ad_write    the item holding that largest n writes its point
//   k_ad_cleanup  arrival counters; leaf lists and table entries cleared
// Mode finding (Really Quick Shift, one workgroup per dirty leaf): k_rqs.
#include <hip/hip_runtime.h>

#include "rl_internal.hpp"

namespace rl {

// Each kernel body takes its frame's arguments and block index, so that one
// launch serves one frame (arguments by value) or one frame of each of
// several rooms (a job table in device memory, blockIdx.y or .z = job).
template <int T>
__device__ __forceinline__ void ad_items(const AdaptArgs& a, int bx)
{
#pragma clang fp contract(off)
    if (a.result && bx == 0) {
        // the record of a batched adaptation: done, no pose
        if (threadIdx.x < 16) a.result->cam_to_world[threadIdx.x] = (threadIdx.x % 5 == 0) ? 1.0f : 0.0f;
        if (threadIdx.x == 0) {
            rl_result* r = a.result;
            r->energy = 0.0f;
            r->mean_energy = 0.0f;
            r->status = RL_OK;
            r->n_valid = 0;
            r->n_inliers = 0;
            r->winner = -1;
            r->refitted = 0;
            r->n_eligible = 0;
            r->rounds = 0;
            r->n_out = 0;
            r->mode_version = a.mode_version;
            r->pad = 0;
        }
    }
    const int g = bx * 256 + threadIdx.x;
    if (g >= a.G) return;
    const int x = 4 * (g % a.gw + 1), y = 4 * (g / a.gw + 1);
    const float d = a.src.d(x, y);
    if (!depth_ok(d)) {
#pragma unroll
        for (int t = 0; t < T; ++t) a.item_leaf[(size_t)t * a.G + g] = (uint16_t)kLeafNone;
        return;
    }
    int leaf[T];
    const PlanarProbe pr{a.src};
    if (a.s == 1.0f) route<T, true>(a.nodes, a.L - 1, a.D, pr, a.w, a.h, x, y, d, a.s, leaf);
    else route<T, false>(a.nodes, a.L - 1, a.D, pr, a.w, a.h, x, y, d, a.s, leaf);
    double xc[3];
    backproject(d, x, y, a.fx, a.fy, a.cx, a.cy, xc);
    float xw[3];
    for (int r = 0; r < 3; ++r) {
        double v = a.H[4 * r + 0] * xc[0] + a.H[4 * r + 1] * xc[1];
        v = v + a.H[4 * r + 2] * xc[2];
        v = v + a.H[4 * r + 3];
        xw[r] = (float)v;
    }
    const uint8_t* c = a.src.c(x, y);
    const uint32_t col = (uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16);
    a.item_pt[g] = make_float4(xw[0], xw[1], xw[2], __uint_as_float(col));
#pragma unroll
    for (int t = 0; t < T; ++t) a.item_leaf[(size_t)t * a.G + g] = (uint16_t)leaf[t];
}

template <int T>
__global__ __launch_bounds__(256) void k_ad_items(AdaptArgs a) { ad_items<T>(a, blockIdx.x); }

template <int T>
__global__ __launch_bounds__(256) void k_ad_items_jobs(const AdaptArgs* __restrict__ jobs)
{
    ad_items<T>(jobs[blockIdx.y], blockIdx.x);
}

// One block per (chunk, tree): the chunk's (leaf << 10 | position) keys are
// sorted in LDS (bitonic; the position makes every key distinct, so equal
// leaves stay in raster order), runs of equal leaves are delimited, and every
// run heads a list entry of its leaf.  Positions of the sorted order index
// the run arrays: run_cnt is the run's length at its head, 0 elsewhere.
__device__ __forceinline__ void ad_sort(const AdaptArgs& a, int c, int t)
{
    __shared__ uint32_t s_v[kAdaptChunk];
    __shared__ int s_start[kAdaptChunk];
    const int i = threadIdx.x;
    const int g = c * kAdaptChunk + i;
    const uint32_t leaf0 = g < a.G ? (uint32_t)a.item_leaf[(size_t)t * a.G + g] : (uint32_t)kLeafNone;
    s_v[i] = (leaf0 << 10) | (uint32_t)i;
    __syncthreads();
    for (int k = 2; k <= kAdaptChunk; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int p = i ^ j;
            if (p > i) {
                const uint32_t x = s_v[i], y = s_v[p];
                if ((x > y) == ((i & k) == 0)) {
                    s_v[i] = y;
                    s_v[p] = x;
                }
            }
            __syncthreads();
        }
    }
    const uint32_t v = s_v[i];
    const uint32_t leaf = v >> 10;
    const bool head = i == 0 || (s_v[i - 1] >> 10) != leaf;
    const bool tail = i == kAdaptChunk - 1 || (s_v[i + 1] >> 10) != leaf;
    s_start[i] = head ? i : 0;
    __syncthreads();
    for (int off = 1; off < kAdaptChunk; off <<= 1) {          // inclusive max-scan: run start
        const int o = i >= off ? s_start[i - off] : 0;
        __syncthreads();
        s_start[i] = max(s_start[i], o);
        __syncthreads();
    }
    const int start = s_start[i];
    const uint32_t rbase = (uint32_t)t * (uint32_t)a.Gp + (uint32_t)c * kAdaptChunk;
    const bool valid = leaf != (uint32_t)kLeafNone;
    if (!head || !valid) a.run_cnt[rbase + i] = 0u;
    if (!valid) return;
    const size_t item = (size_t)t * a.G + (size_t)c * kAdaptChunk + (v & 1023u);
    a.item_run[item] = rbase + (uint32_t)start;
    a.item_lrank[item] = (uint16_t)(i - start);
    if (tail) {
        const uint32_t r = rbase + (uint32_t)start;
        const uint32_t tl = ((uint32_t)t << a.D) + leaf;
        a.run_cnt[r] = (uint32_t)(i - start + 1);
        a.run_tl[r] = tl;
        a.run_next[r] = atomicExch(&a.head[tl], r);
    }
}

__global__ __launch_bounds__(kAdaptChunk) void k_ad_sort(AdaptArgs a) { ad_sort(a, blockIdx.x, blockIdx.y); }

// grid (chunks, trees, jobs) of the largest frame; blocks past a job's own
// chunks or trees leave at once (before any barrier)
__global__ __launch_bounds__(kAdaptChunk) void k_ad_sort_jobs(const AdaptArgs* __restrict__ jobs)
{
    const AdaptArgs& a = jobs[blockIdx.z];
    if ((int)blockIdx.x * kAdaptChunk >= a.Gp || (int)blockIdx.y >= a.T) return;
    ad_sort(a, blockIdx.x, blockIdx.y);
}

// One thread per sorted position; each run adds up the runs of its leaf in
// earlier chunks.  A leaf's list holds at most one run per chunk.
__device__ __forceinline__ void ad_runs(const AdaptArgs& a, int n_chunks, int bx)
{
    const uint32_t r = bx * 256 + threadIdx.x;
    if (r >= (uint32_t)a.T * (uint32_t)a.Gp) return;
    const uint32_t cnt = a.run_cnt[r];
    if (cnt == 0u) return;
    const uint32_t tl = a.run_tl[r];
    const uint32_t chunk = (r % (uint32_t)a.Gp) / kAdaptChunk;
    uint32_t pre = 0, total = 0;
    uint32_t q = a.head[tl];
    for (int k = 0; k < n_chunks && q != kNone32; ++k) {
        const uint32_t qc = a.run_cnt[q];
        total += qc;
        if ((q % (uint32_t)a.Gp) / kAdaptChunk < chunk) pre += qc;
        q = a.run_next[q];
    }
    a.run_pre[r] = pre;
    a.run_tot[r] = pre + cnt == total ? total : 0u;
}

__global__ __launch_bounds__(256) void k_ad_runs(AdaptArgs a, int n_chunks) { ad_runs(a, n_chunks, blockIdx.x); }

__global__ __launch_bounds__(256) void k_ad_runs_jobs(const AdaptArgs* __restrict__ jobs)
{
    const AdaptArgs& a = jobs[blockIdx.y];
    ad_runs(a, a.Gp / kAdaptChunk, blockIdx.x);
}

__device__ __forceinline__ uint32_t slot_hash(uint32_t key, uint32_t mask)
{
    return (key * 0x9E3779B1u) & mask;
}

__device__ __forceinline__ void ad_claim(const AdaptArgs& a, int bx)
{
    const int i = bx * 256 + threadIdx.x;
    if (i >= a.T * a.G) return;
    const int t = i / a.G;
    const uint16_t lf = a.item_leaf[i];
    if (lf == kLeafNone) return;
    const uint32_t tl = ((uint32_t)t << a.D) + lf;
    const uint32_t n = a.seen[tl] + a.run_pre[a.item_run[i]] + (uint32_t)a.item_lrank[i] + 1u;
    int slot;
    if (n <= (uint32_t)a.kappa) {
        slot = (int)n - 1;
    } else {
        const uint4 r = philox(make_uint4(kTagRes << 28, (uint32_t)t, (uint32_t)lf, n), a.key0, a.key1);
        const uint32_t j = below(r.x, n);
        slot = j < (uint32_t)a.kappa ? (int)j : -1;
    }
    a.item_n[i] = n;
    a.item_slot[i] = slot;
    if (slot < 0) return;
    // the table holds at most T G keys in at least 2 T G entries, so a free
    // or matching entry is found within hmask + 1 probes
    const uint32_t key = (tl << 12) | (uint32_t)slot;
    uint32_t h = slot_hash(key, a.hmask);
    for (uint32_t probe = 0; probe <= a.hmask; ++probe) {
        const uint32_t prev = atomicCAS(&a.hkey[h], kNone32, key);
        if (prev == kNone32 || prev == key) {
            atomicMax(&a.hval[h], n);
            a.item_h[i] = h;
            return;
        }
        h = (h + 1u) & a.hmask;
    }
    a.item_slot[i] = -1;                // unreachable: the table is never full
}

__global__ __launch_bounds__(256) void k_ad_claim(AdaptArgs a) { ad_claim(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_ad_claim_jobs(const AdaptArgs* __restrict__ jobs)
{
    ad_claim(jobs[blockIdx.y], blockIdx.x);
}

__device__ __forceinline__ void ad_write(const AdaptArgs& a, int bx)
{
    const int i = bx * 256 + threadIdx.x;
    if (i >= a.T * a.G) return;
    const uint16_t lf = a.item_leaf[i];
    if (lf == kLeafNone) return;
    const int slot = a.item_slot[i];
    if (slot < 0) return;
    if (a.hval[a.item_h[i]] != a.item_n[i]) return;          // a later arrival of the frame took the slot
    const int t = i / a.G, g = i % a.G;
    const size_t tl = ((size_t)t << a.D) + lf;
    a.reservoir[tl * (size_t)a.kappa + (size_t)slot] = a.item_pt[g];
    if (atomicExch(&a.dirty[tl], 1u) == 0u) {
        const uint32_t k = atomicAdd(&a.counters[0], 1u);
        a.dirty_list[k] = (uint32_t)tl;
    }
}

__global__ __launch_bounds__(256) void k_ad_write(AdaptArgs a) { ad_write(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_ad_write_jobs(const AdaptArgs* __restrict__ jobs)
{
    ad_write(jobs[blockIdx.y], blockIdx.x);
}

// One thread per sorted position (covering the items too): the leaf's
// arrival counter from its last run, leaf lists and used table entries back
// to their empty state.
__device__ __forceinline__ void ad_cleanup(const AdaptArgs& a, int bx)
{
    const uint32_t x = bx * 256 + threadIdx.x;
    if (x < (uint32_t)a.T * (uint32_t)a.G && a.item_leaf[x] != kLeafNone && a.item_slot[x] >= 0) {
        const uint32_t h = a.item_h[x];
        a.hkey[h] = kNone32;
        a.hval[h] = 0u;
    }
    if (x < (uint32_t)a.T * (uint32_t)a.Gp && a.run_cnt[x] != 0u) {
        const uint32_t tl = a.run_tl[x];
        a.head[tl] = kNone32;
        const uint32_t tot = a.run_tot[x];
        if (tot) a.seen[tl] += tot;
    }
}

__global__ __launch_bounds__(256) void k_ad_cleanup(AdaptArgs a) { ad_cleanup(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_ad_cleanup_jobs(const AdaptArgs* __restrict__ jobs)
{
    ad_cleanup(jobs[blockIdx.y], blockIdx.x);
}

// ------------------------------------------------------------------------
// Really Quick Shift (Fulkerson & Soatto 2010) on one leaf reservoir per
// workgroup iteration, with the paper's post-processing (Sec. 3.2.2 step 3):
//   rho_k = sum_j exp(-|P_k - P_j|^2 / (2 sigma^2))   (FP64, j in order)
//   parent(k) = nearest j with (rho_j, j) > (rho_k, k) and |P_k - P_j| < tau
//   roots by pointer jumping; clusters of >= min_size points, at most M,
//   ordered by (size desc, root asc); mean, population covariance, mean
//   colour, inverse of (covariance + lambda I).
// Distances are evaluated exactly as written (no contraction).
__device__ __forceinline__ double dist2(float4 a, float4 b)
{
#pragma clang fp contract(off)
    const double dx = (double)a.x - (double)b.x, dy = (double)a.y - (double)b.y, dz = (double)a.z - (double)b.z;
    return dx * dx + dy * dy + dz * dz;
}

// rho_k, j in order
__device__ __forceinline__ double rqs_density(const float4* pts, int n, float4 pk, double two_s2)
{
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += exp(-dist2(pk, pts[j]) / two_s2);
    return acc;
}

// parent(k): the nearest point of higher (rho, index) within tau, or -1
__device__ __forceinline__ int rqs_link(const float4* pts, const double* rho, int n, int k, double tau2)
{
    const float4 pk = pts[k];
    const double rk = rho[k];
    int best = -1;
    double bestd = INFINITY;
    for (int j = 0; j < n; ++j) {
        const double rj = rho[j];
        const bool higher = rj > rk || (rj == rk && j > k);
        if (!higher) continue;
        const double d2 = dist2(pk, pts[j]);
        if (d2 < tau2 && d2 < bestd) {
            bestd = d2;
            best = j;
        }
    }
    return best;
}

// A round-robin step of at most kRqsSplitLeaves leaves computes its O(n^2)
// passes (density, then links) as row chunks of kRqsRows points in
// workgroups of their own, so that a full reservoir is spread over
// kappa / kRqsRows workgroups instead of holding one for all its rows; each
// row runs the same loop as in k_rqs, so the links are the same.
__host__ __device__ inline bool rqs_split(const RqsArgs& a)
{
    return a.rr_count > 0 && a.rr_count <= (uint32_t)kRqsSplitLeaves;
}

// grid (row chunks, leaves of the step[, rooms]); dynamic LDS float4[kappa]
__device__ __forceinline__ void rqs_density_rows(const RqsArgs& a, int c, uint32_t li)
{
    extern __shared__ unsigned char s_raw[];
    float4* pts = reinterpret_cast<float4*>(s_raw);
    if (!rqs_split(a) || li >= a.rr_count) return;
    const uint32_t tl = (a.rr_first + li) % a.n_leaves;
    const int n = (int)min(a.seen[tl], (uint32_t)a.kappa);
    if (c * kRqsRows >= n) return;
    const float4* src = a.reservoir + (size_t)tl * a.kappa;
    for (int k = threadIdx.x; k < n; k += kRqsRows) pts[k] = src[k];
    __syncthreads();
    const int k = c * kRqsRows + (int)threadIdx.x;
    if (k < n) a.rr_rho[(size_t)li * a.kappa + k] = rqs_density(pts, n, pts[k], 2.0 * a.sigma * a.sigma);
}

// dynamic LDS float4[kappa], then double[kappa]
__device__ __forceinline__ void rqs_link_rows(const RqsArgs& a, int c, uint32_t li)
{
    extern __shared__ unsigned char s_raw[];
    float4* pts = reinterpret_cast<float4*>(s_raw);
    double* rho = reinterpret_cast<double*>(s_raw + 16 * (size_t)a.kappa);
    if (!rqs_split(a) || li >= a.rr_count) return;
    const uint32_t tl = (a.rr_first + li) % a.n_leaves;
    const int n = (int)min(a.seen[tl], (uint32_t)a.kappa);
    if (c * kRqsRows >= n) return;
    const float4* src = a.reservoir + (size_t)tl * a.kappa;
    const double* lr = a.rr_rho + (size_t)li * a.kappa;
    for (int k = threadIdx.x; k < n; k += kRqsRows) {
        pts[k] = src[k];
        rho[k] = lr[k];
    }
    __syncthreads();
    const int k = c * kRqsRows + (int)threadIdx.x;
    if (k < n) a.rr_parent[(size_t)li * a.kappa + k] = rqs_link(pts, rho, n, k, a.tau * a.tau);
}

__global__ __launch_bounds__(kRqsRows) void k_rqs_density(RqsArgs a) { rqs_density_rows(a, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(kRqsRows) void k_rqs_links(RqsArgs a) { rqs_link_rows(a, blockIdx.x, blockIdx.y); }
__global__ __launch_bounds__(kRqsRows) void k_rqs_density_jobs(const RqsArgs* __restrict__ jobs)
{
    rqs_density_rows(jobs[blockIdx.z], blockIdx.x, blockIdx.y);
}
__global__ __launch_bounds__(kRqsRows) void k_rqs_links_jobs(const RqsArgs* __restrict__ jobs)
{
    rqs_link_rows(jobs[blockIdx.z], blockIdx.x, blockIdx.y);
}

// Sum over the first 256 threads of the block in a fixed tree order (the
// other threads only take part in the barriers), so that a moment does not
// depend on the block size.
__device__ __forceinline__ double rqs_block_sum(double v, double* s_red)
{
    if (threadIdx.x < 256) s_red[threadIdx.x] = v;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) s_red[threadIdx.x] += s_red[threadIdx.x + stride];
        __syncthreads();
    }
    const double r = s_red[0];
    __syncthreads();
    return r;
}

// dynamic LDS: float4 pts[kappa], double rho[kappa], int parent[kappa], int root[kappa], int size[kappa]
// BS threads per leaf: the per-point O(n^2) passes (density, links, ranks)
// stride over all of them; the moments use the first 256 in a fixed order,
// so every block size gives the same rows.
template <int BS>
__device__ __forceinline__ void rqs(const RqsArgs& a, uint32_t bx, uint32_t gx)
{
    extern __shared__ unsigned char s_raw[];
    float4* pts = reinterpret_cast<float4*>(s_raw);
    double* rho = reinterpret_cast<double*>(s_raw + 16 * (size_t)a.kappa);
    int* parent = reinterpret_cast<int*>(s_raw + 24 * (size_t)a.kappa);
    int* root = parent + a.kappa;
    int* size = root + a.kappa;
    __shared__ double s_red[256];
    __shared__ int s_chosen[64];
    __shared__ int s_ncand;
    const int tid = threadIdx.x;
    const uint32_t ndirty = a.rr_count ? a.rr_count : a.counters[0];
    const double two_s2 = 2.0 * a.sigma * a.sigma;
    const double tau2 = a.tau * a.tau;
    const bool split = rqs_split(a);
    for (uint32_t li = bx; li < ndirty; li += gx) {
        const uint32_t tl = a.rr_count ? (a.rr_first + li) % a.n_leaves : a.dirty_list[li];
        const int n = (int)min(a.seen[tl], (uint32_t)a.kappa);
        const float4* src = a.reservoir + (size_t)tl * a.kappa;
        for (int k = tid; k < n; k += BS) {
            pts[k] = src[k];
            size[k] = 0;
        }
        if (tid == 0) s_ncand = 0;
        __syncthreads();
        if (split) {
            // links computed by k_rqs_density / k_rqs_links
            const int* lp = a.rr_parent + (size_t)li * a.kappa;
            for (int k = tid; k < n; k += BS) {
                const int best = lp[k];
                parent[k] = best;
                root[k] = best < 0 ? k : best;
            }
        } else {
            for (int k = tid; k < n; k += BS) rho[k] = rqs_density(pts, n, pts[k], two_s2);
            __syncthreads();
            for (int k = tid; k < n; k += BS) {
                const int best = rqs_link(pts, rho, n, k, tau2);
                parent[k] = best;
                root[k] = best < 0 ? k : best;
            }
        }
        __syncthreads();
        // pointer jumping: after ceil(log2 n) + 1 passes every point holds its root
        for (int pass = 0; (1 << pass) <= 2 * n; ++pass) {
            for (int k = tid; k < n; k += BS) {
                const int r = root[k];
                root[k] = root[r];
            }
            __syncthreads();
        }
        for (int k = tid; k < n; k += BS) atomicAdd(&size[root[k]], 1);
        __syncthreads();
        // candidates ranked by (size desc, root asc); keep ranks < M
        for (int k = tid; k < n; k += BS) {
            if (parent[k] >= 0 || size[k] < a.min_size) continue;
            const int sk = size[k];
            int rank = 0;
            for (int j = 0; j < n; ++j) {
                if (parent[j] >= 0 || size[j] < a.min_size) continue;
                rank += (size[j] > sk || (size[j] == sk && j < k)) ? 1 : 0;
            }
            if (rank < a.M) s_chosen[rank] = k;
            atomicAdd(&s_ncand, 1);
        }
        __syncthreads();
        const int nm = min(s_ncand, a.M);
        float4* out = a.modes + (size_t)tl * a.M * 4;
        for (int m = 0; m < nm; ++m) {
            const int r = s_chosen[m];
            double sx = 0, sy = 0, sz = 0, cnt = 0, cr = 0, cg = 0, cb = 0;
            for (int k = tid; k < n && tid < 256; k += 256) {
                if (root[k] != r) continue;
                const float4 pk = pts[k];
                sx += pk.x; sy += pk.y; sz += pk.z; cnt += 1.0;
                const uint32_t c = __float_as_uint(pk.w);
                cr += (double)(c & 0xFFu);
                cg += (double)((c >> 8) & 0xFFu);
                cb += (double)((c >> 16) & 0xFFu);
            }
            cnt = rqs_block_sum(cnt, s_red);
            const double mx = rqs_block_sum(sx, s_red) / cnt, my = rqs_block_sum(sy, s_red) / cnt,
                         mz = rqs_block_sum(sz, s_red) / cnt;
            const double mr = rqs_block_sum(cr, s_red) / cnt, mg = rqs_block_sum(cg, s_red) / cnt,
                         mb = rqs_block_sum(cb, s_red) / cnt;
            double S[6] = {0, 0, 0, 0, 0, 0};
            for (int k = tid; k < n && tid < 256; k += 256) {
                if (root[k] != r) continue;
                const float4 pk = pts[k];
                const double dx = (double)pk.x - mx, dy = (double)pk.y - my, dz = (double)pk.z - mz;
                S[0] += dx * dx; S[1] += dx * dy; S[2] += dx * dz;
                S[3] += dy * dy; S[4] += dy * dz; S[5] += dz * dz;
            }
            for (int q = 0; q < 6; ++q) S[q] = rqs_block_sum(S[q], s_red) / cnt;
            if (tid == 0) {
                const double A_ = S[0] + a.lambda, B_ = S[1], C_ = S[2], D_ = S[3] + a.lambda, E_ = S[4],
                             F_ = S[5] + a.lambda;
                const double ca = D_ * F_ - E_ * E_, cb2 = C_ * E_ - B_ * F_, cc = B_ * E_ - C_ * D_;
                const double cd = A_ * F_ - C_ * C_, ce = B_ * C_ - A_ * E_, cf = A_ * D_ - B_ * B_;
                const double det = A_ * ca + B_ * cb2 + C_ * cc;
                float4* row = out + 4 * m;
                row[0] = make_float4((float)mx, (float)my, (float)mz, (float)cnt);
                row[1] = make_float4((float)(ca / det), (float)(cb2 / det), (float)(cc / det), (float)(cd / det));
                row[2] = make_float4((float)(ce / det), (float)(cf / det), (float)mr, (float)mg);
                row[3] = make_float4((float)mb, 0.0f, 0.0f, 0.0f);
                a.cbox[(size_t)tl * a.M + m] = colour_box((float)mr, (float)mg, (float)mb, a.theta_col);
            }
        }
        if (tid == 0) {
            a.nmodes[tl] = (uint8_t)nm;
            if (!a.rr_count) a.dirty[tl] = 0u;
        }
        __syncthreads();
    }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_rqs(RqsArgs a) { rqs<BS>(a, blockIdx.x, gridDim.x); }

// round-robin steps of several rooms at once: blockIdx.y = room
template <int BS>
__global__ __launch_bounds__(BS) void k_rqs_jobs(const RqsArgs* __restrict__ jobs)
{
    rqs<BS>(jobs[blockIdx.y], blockIdx.x, gridDim.x);
}

__global__ void k_rqs_done(RqsArgs a)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) a.counters[0] = 0u;
}

// ------------------------------------------------------------------------
#define RL_CHECK_LAUNCH() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_adapt(const AdaptArgs& a, hipStream_t st)
{
    if (a.G <= 0) return hipSuccess;
    const dim3 blk(256), g1((a.G + 255) / 256), gT((a.T * a.G + 255) / 256);
    switch (a.T) {
        case 1: k_ad_items<1><<<g1, blk, 0, st>>>(a); break;
        case 2: k_ad_items<2><<<g1, blk, 0, st>>>(a); break;
        case 3: k_ad_items<3><<<g1, blk, 0, st>>>(a); break;
        case 4: k_ad_items<4><<<g1, blk, 0, st>>>(a); break;
        case 5: k_ad_items<5><<<g1, blk, 0, st>>>(a); break;
        case 6: k_ad_items<6><<<g1, blk, 0, st>>>(a); break;
        case 7: k_ad_items<7><<<g1, blk, 0, st>>>(a); break;
        case 8: k_ad_items<8><<<g1, blk, 0, st>>>(a); break;
        default: return hipErrorInvalidValue;
    }
    RL_CHECK_LAUNCH();
    const int n_chunks = a.Gp / kAdaptChunk;
    const dim3 gR((a.T * a.Gp + 255) / 256);
    k_ad_sort<<<dim3(n_chunks, a.T), dim3(kAdaptChunk), 0, st>>>(a);
    RL_CHECK_LAUNCH();
    k_ad_runs<<<gR, blk, 0, st>>>(a, n_chunks);
    RL_CHECK_LAUNCH();
    k_ad_claim<<<gT, blk, 0, st>>>(a);
    RL_CHECK_LAUNCH();
    k_ad_write<<<gT, blk, 0, st>>>(a);
    RL_CHECK_LAUNCH();
    k_ad_cleanup<<<gR, blk, 0, st>>>(a);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

// One frame for each of njobs rooms (device job table, host copy hjobs for
// the shapes); all jobs have T trees.
hipError_t launch_adapt_jobs(const AdaptArgs* jobs, const AdaptArgs* hjobs, int njobs, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    int T = hjobs[0].T, G = 0, Gp = 0;
    for (int j = 0; j < njobs; ++j) {
        if (hjobs[j].T != T) return hipErrorInvalidValue;
        G = max(G, hjobs[j].G);
        Gp = max(Gp, hjobs[j].Gp);
    }
    if (G <= 0) return hipSuccess;
    const dim3 blk(256), g1((G + 255) / 256, njobs), gT((T * G + 255) / 256, njobs);
    switch (T) {
        case 1: k_ad_items_jobs<1><<<g1, blk, 0, st>>>(jobs); break;
        case 2: k_ad_items_jobs<2><<<g1, blk, 0, st>>>(jobs); break;
        case 3: k_ad_items_jobs<3><<<g1, blk, 0, st>>>(jobs); break;
        case 4: k_ad_items_jobs<4><<<g1, blk, 0, st>>>(jobs); break;
        case 5: k_ad_items_jobs<5><<<g1, blk, 0, st>>>(jobs); break;
        case 6: k_ad_items_jobs<6><<<g1, blk, 0, st>>>(jobs); break;
        case 7: k_ad_items_jobs<7><<<g1, blk, 0, st>>>(jobs); break;
        case 8: k_ad_items_jobs<8><<<g1, blk, 0, st>>>(jobs); break;
        default: return hipErrorInvalidValue;
    }
    RL_CHECK_LAUNCH();
    const dim3 gR((T * Gp + 255) / 256, njobs);
    k_ad_sort_jobs<<<dim3(Gp / kAdaptChunk, T, njobs), dim3(kAdaptChunk), 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_ad_runs_jobs<<<gR, blk, 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_ad_claim_jobs<<<gT, blk, 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_ad_write_jobs<<<gT, blk, 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    k_ad_cleanup_jobs<<<gR, blk, 0, st>>>(jobs);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

// Round-robin steps (rr_count > 0) of njobs rooms; LDS for the largest
// reservoir capacity.
hipError_t launch_rqs_jobs(const RqsArgs* jobs, const RqsArgs* hjobs, int njobs, int blocks, hipStream_t st)
{
    if (njobs <= 0) return hipSuccess;
    int kappa = 0;
    uint32_t cnt = 0, split_cnt = 0;
    for (int j = 0; j < njobs; ++j) {
        if (hjobs[j].rr_count == 0) return hipErrorInvalidValue;
        kappa = max(kappa, hjobs[j].kappa);
        cnt = max(cnt, hjobs[j].rr_count);
        if (rqs_split(hjobs[j])) split_cnt = max(split_cnt, hjobs[j].rr_count);
    }
    const int nb = (int)min((uint32_t)blocks, cnt);
    if (split_cnt > 0) {
        // the rooms whose steps are split (the others' blocks leave at once)
        const dim3 g((kappa + kRqsRows - 1) / kRqsRows, split_cnt, njobs);
        k_rqs_density_jobs<<<g, dim3(kRqsRows), 16 * (size_t)kappa, st>>>(jobs);
        RL_CHECK_LAUNCH();
        k_rqs_links_jobs<<<g, dim3(kRqsRows), 24 * (size_t)kappa, st>>>(jobs);
        RL_CHECK_LAUNCH();
    }
    k_rqs_jobs<1024><<<dim3(nb, njobs), dim3(1024), 36 * (size_t)kappa, st>>>(jobs);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_rqs(const RqsArgs& a, int blocks, hipStream_t st)
{
    const size_t lds = 36 * (size_t)a.kappa;
    if (a.rr_count) {
        // a round-robin step: few leaves, most of them full; 1024 threads each
        const int nb = (int)min((uint32_t)blocks, a.rr_count);
        if (rqs_split(a)) {
            const dim3 g((a.kappa + kRqsRows - 1) / kRqsRows, a.rr_count);
            k_rqs_density<<<g, dim3(kRqsRows), 16 * (size_t)a.kappa, st>>>(a);
            RL_CHECK_LAUNCH();
            k_rqs_links<<<g, dim3(kRqsRows), 24 * (size_t)a.kappa, st>>>(a);
            RL_CHECK_LAUNCH();
        }
        k_rqs<1024><<<dim3(nb), dim3(1024), lds, st>>>(a);
    } else {
        k_rqs<256><<<dim3(blocks), dim3(256), lds, st>>>(a);
    }
    RL_CHECK_LAUNCH();
    if (a.rr_count) return hipSuccess;      // the dirty list is left for an exact update
    k_rqs_done<<<dim3(1), dim3(64), 0, st>>>(a);
    RL_CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace rl
