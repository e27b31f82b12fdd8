// rl_internal.hpp -- device-side data layout and helpers of librl (gfx950).
//
// Every relocalisation kernel reads a device-resident job table: one Job per
// frame, holding the frame, the room's forest/mode arrays, the parameters
// and that frame's scratch arrays.  A single frame is a batch of one; a
// batch of frames from several rooms and resolutions is the same launch
// sequence with gridDim.y = number of jobs.  Because the launch parameters
// depend only on the batch shape, the sequence can be captured once in a HIP
// graph and replayed with new job tables.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rl.h"

namespace rl {

constexpr int kMaxTrees = 8;
constexpr long long kMaxPixels = 1LL << 24;   // pixel indices are packed in 24 bits
constexpr int kLeafNone = 0xFFFF;
constexpr uint32_t kTagRes = 1, kTagHyp = 2, kTagScore = 3;
#ifndef RL_SCORE_TILE
#define RL_SCORE_TILE 4
#endif
constexpr int kScoreTile = RL_SCORE_TILE;     // pixels per scoring wave
// All-rounds scoring (once a job's survivors fit fast_max = 64 * fast waves
// lanes) keeps its partials with this stride: up to 4 waves of hypotheses.
// analytic scene models for the model-based scores
constexpr int kMaxModelSurfaces = 64, kMaxModelPoses = 64;

// frames of one batched launch
constexpr int kMaxBatchFrames = 4096;

constexpr int kMaxFastWaves = 4;

// levels of every tree the traversal may read from LDS (T x (2^levels - 1)
// node records per block): a launch schedule, 6 or 8
constexpr int kTopLevelsMin = 6, kTopLevelsMax = 8;

// LM refinement: pixels per partial-sum tile of a pass (a wave takes one or
// two tiles), doubles per partial (E, g (6), upper triangle of N (21,
// row-major)), doubles of per-slot state
constexpr int kLmTile = 64;
constexpr int kLmVals = 28;
constexpr int kLmStateDoubles = 56;
constexpr int kFastStride = 64 * kMaxFastWaves;

struct JobState {
    int n_elig;
    int n_valid;
    int n_surv;
    int rounds_run;
    int done;
    int pad[3];
};

struct Hyp {                 // == rl_hypothesis
    float R[9];
    float t[3];
    int pix[3];
    int mode[3];
    int iter;
    int valid;
};
static_assert(sizeof(Hyp) == sizeof(rl_hypothesis), "hypothesis layout");

// Load through the global address space.  Pointers read from the job table
// are generic to the compiler; generic (flat) loads wait on both the memory
// and LDS counters and cannot be reordered around LDS stores, which
// serialises independent gathers.
template <class T>
__device__ __forceinline__ T ldg(const T* p)
{
    return *(const __attribute__((address_space(1))) T*)p;
}

// The caller's frame buffers, read in place: pixel (x, y) of the frame is
// sample (step x, step y) of the buffers (step 2: the 2x decimated frame);
// row pitches in bytes, ch bytes per colour sample (3 or 4).
struct FrameView {
    const float* depth;
    const uint8_t* rgb;
    uint32_t dpitch, rpitch, ch, step;
    __device__ __forceinline__ float d(int x, int y) const
    {
        return ldg(reinterpret_cast<const float*>(reinterpret_cast<const char*>(depth) +
                                                  (size_t)(step * (uint32_t)y) * dpitch +
                                                  (size_t)(step * (uint32_t)x) * 4u));
    }
    __device__ __forceinline__ const uint8_t* c(int x, int y) const
    {
        return rgb + (size_t)(step * (uint32_t)y) * rpitch + (size_t)(step * (uint32_t)x) * ch;
    }
};

struct Job {
    // room (persistent)
    const float4* nodes;      // [T][NT] (dx, dy, tau, kind bits)
    const float4* modes;      // [T][L][M] rows of 4 float4
    const uint8_t* nmodes;    // [T][L]
    const uint2* cbox;        // [T][L][M] colour box per mode row (see colour_box)
    int T, D, M;
    int screen;               // 1: the search rejects clearly degenerate triplets itself
    // frame
    FrameView src;            // the caller's buffers (read by the ingest only)
    uint32_t* probe;          // [2][P] probe image planes (depth bits; R, G, B bytes), built per frame
    int w, h;
    float fx, fy, cx, cy;
    float s;                  // w / ref_width (float32 division)
    // parameters
    int N, I_max, eta, n_cull, n_out, use_cov, final_refine, trace;
    float theta_col;
    int TP;                   // pixels per scoring block
    int fast_max;             // survivors scored round by round while above this (64 * fast waves)
    int lm, lm_iters;         // LM refinement of the survivors in every round after the first
    double min_sq_dist, theta_rig, theta_in;
    uint32_t key0, key1;
    // scratch
    uint16_t* leaves;         // [P][8]
    uint8_t* nmt;             // [P][8] modes per tree's leaf
    uint8_t* nm;              // [P] |M(u)|
    int* tile_count;          // [ceil(P/256)]
    int* eligible;            // [P]
    uint4* ecold;             // [P][2] per list entry: (pixel, depth bits, mode counts), leaves
    uint64_t* erec;           // [P][ew] eligible-pixel records (see erec_* below)
    int ew;                   // words per record: 1 for |M(u)| <= 56
    uint32_t mode_version;    // the room's mode updates when this job was queued (result record)
    int* hyp_best;            // [N]
    Hyp* hyps;                // [N]
    int* surv;                // [N]
    double* E;                // [N] energy per slot
    double* pose64;           // [N][12] LM-refined poses (R row-major, t), FP64
    double* lm_state;         // [N][kLmStateDoubles] LM iteration state per slot
    double* lm_part;          // [round's survivors][round's tiles][kLmVals] LM pass partial sums per (survivor position, tile)
    int* Ie;                  // [rounds_max * eta] eligible-list entries of I
    int* lm_plan;             // 2 x [kMaxBatchFrames + 1] LM item and survivor plans of the launch (shared by its jobs)
    double4* lm_px;           // [rounds_max * eta] camera point and |M(u)| of each pixel of I
    float4* lm_rows;          // [rows per pixel][3 x rounds_max * eta] staged rows of M(u) (mean, Sigma^-1), lm_split below
    int lm_icap;              // rounds_max * eta
    int lm_split;             // 1: lm_rows [row][16-byte part][pixel of I]; 0: [row][pixel of I][16-byte part]
    double* partial;          // [ptiles][N]
    double* partial_all;      // [rounds][ptiles][kFastStride] per-round partials once survivors fit fast_max
    int* I;                   // [rounds_max * eta]
    int* inl;                 // [rounds_max * eta] refit scratch
    int* trace_slots;         // [rounds_max][N]
    double* trace_E;          // [rounds_max][N]
    JobState* st;
    rl_result* result;
};

// Arguments of the adaptation kernels (one room, one frame; by value).
struct AdaptArgs {
    const float4* nodes;
    int T, D, L, kappa;
    FrameView src;
    int w, h, gw, G;
    float fx, fy, cx, cy, s;
    double H[12];             // camera->world rows (from float32)
    uint32_t key0, key1;
    float4* reservoir;        // [T][L][kappa]
    uint32_t* seen;           // [T][L]
    uint32_t* dirty;          // [T][L]
    uint32_t* dirty_list;     // [T*L]
    uint32_t* counters;       // [0] dirty count
    // scratch of one frame: items are (tree, grid pixel) arrivals; a run is
    // the items of one leaf within one chunk of kAdaptChunk grid pixels
    uint16_t* item_leaf;      // [T][G] leaf reached, kLeafNone for invalid depth
    float4* item_pt;          // [G] world point and colour bits
    uint32_t* item_run;       // [T][G] run (index into the run arrays)
    uint16_t* item_lrank;     // [T][G] rank within its run (raster order)
    uint32_t* item_n;         // [T][G] arrival number n
    int* item_slot;           // [T][G] reservoir slot drawn, or -1
    uint32_t* item_h;         // [T][G] hash-table entry of (leaf, slot)
    uint32_t* run_cnt;        // [T][Gp] items of the run headed at this sorted position (0: no run)
    uint32_t* run_tl;         // [T][Gp] leaf (t * L + leaf) of a run
    uint32_t* run_next;       // [T][Gp] next run of the same leaf
    uint32_t* run_pre;        // [T][Gp] the leaf's items in earlier chunks
    uint32_t* run_tot;        // [T][Gp] the leaf's items this frame, on its last run (else 0)
    // kept between frames in their cleared state
    uint32_t* head;           // [T][L] first run of the leaf's list, kNone32 when empty
    uint32_t* hkey;           // [hmask + 1] (leaf << 12 | slot), kNone32 when empty
    uint32_t* hval;           // [hmask + 1] largest arrival number drawing that slot, 0 when empty
    int Gp;                   // chunks * kAdaptChunk
    uint32_t hmask;           // hash-table size - 1 (size a power of two >= 2 T G)
    rl_result* result;        // batched adaptation: its result record (status RL_OK), else NULL
    uint32_t mode_version;    // ... and the room's mode version after it
};

constexpr int kAdaptChunk = 1024;
constexpr uint32_t kNone32 = 0xFFFFFFFFu;

struct RqsArgs {
    const float4* reservoir;
    const uint32_t* seen;
    uint32_t* dirty;
    const uint32_t* dirty_list;
    uint32_t* counters;
    float4* modes;
    uint8_t* nmodes;
    int kappa, M, min_size;
    double sigma, tau, lambda;
    uint2* cbox;              // [T][L][M] colour boxes of the mode rows
    float theta_col;
    // round-robin schedule: when rr_count > 0, the leaves rr_first ...
    // rr_first + rr_count - 1 (mod n_leaves) are clustered instead of the
    // dirty list, whose state is left as it is
    uint32_t rr_first, rr_count, n_leaves;
    // a step of at most kRqsSplitLeaves leaves: densities and links per
    // (leaf of the step, point), [kRqsSplitLeaves][kappa]
    double* rr_rho;
    int* rr_parent;
};

constexpr int kRqsSplitLeaves = 256;
constexpr int kRqsRows = 256;

// ---------------------------------------------------------------------------
#ifndef RL_PHILOX_WIDE
#define RL_PHILOX_WIDE 0
#endif

// Philox4x32-10 (Salmon et al., SC'11): two 32x32->64 multiplies per round
// on counter words 0 and 2, round keys bumped by the Weyl constants.
__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
#if RL_PHILOX_WIDE
        // one 32x32->64 multiply each (v_mad_u64_u32): fewer instructions,
        // more registers held across an unrolled search
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1, (uint32_t)p0);
#else
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
#endif
    }
    return c;
}

// HIP's vector structs would be copied through a generic reference: load
// them as native vectors instead.
typedef uint32_t rl_u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t rl_u32x4 __attribute__((ext_vector_type(4)));
typedef float rl_f32x4 __attribute__((ext_vector_type(4)));
template <>
__device__ __forceinline__ uint2 ldg<uint2>(const uint2* p)
{
    const rl_u32x2 v = *(const __attribute__((address_space(1))) rl_u32x2*)p;
    return make_uint2(v.x, v.y);
}
template <>
__device__ __forceinline__ uint4 ldg<uint4>(const uint4* p)
{
    const rl_u32x4 v = *(const __attribute__((address_space(1))) rl_u32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ float4 ldg<float4>(const float4* p)
{
    const rl_f32x4 v = *(const __attribute__((address_space(1))) rl_f32x4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
template <>
__device__ __forceinline__ double4 ldg<double4>(const double4* p)
{
    const uint4 a = ldg(reinterpret_cast<const uint4*>(p)), b = ldg(reinterpret_cast<const uint4*>(p) + 1);
    return make_double4(__hiloint2double((int)a.y, (int)a.x), __hiloint2double((int)a.w, (int)a.z),
                        __hiloint2double((int)b.y, (int)b.x), __hiloint2double((int)b.w, (int)b.z));
}

// integer in [0, n): floor(r * n / 2^32)
__device__ __forceinline__ uint32_t below(uint32_t r, uint32_t n) { return __umulhi(r, n); }

__device__ __forceinline__ bool depth_ok(float d) { return d > 0.0f && d <= 3.0e38f; }

// x^C = D(u) K^-1 (u, v, 1)^T in FP64, evaluated exactly as written.
__device__ __forceinline__ void backproject(float d, int x, int y, float fx, float fy, float cx,
                                            float cy, double out[3])
{
#pragma clang fp contract(off)
    out[0] = (double)d * (((double)x - (double)cx) / (double)fx);
    out[1] = (double)d * (((double)y - (double)cy) / (double)fy);
    out[2] = (double)d;
}

// Routes pixel (x, y) with valid depth d through T trees in lockstep: at
// every level all T node fetches and probe fetches are in flight together.
// Float32 definition: offset = rint(delta * s * (1/d)), probe clamped to the
// image, f = D(p) - D(q) or C(p,c) - C(q,c), right child iff f >= tau.
// Probe reads of the routing: from the caller's planar depth and RGB8, or
// from the probe image that a relocalisation builds first (two planes of
// 4-byte words: depth bits; R, G, B bytes), so that a probe is one 4-byte
// load, its plane picked by the feature kind without a branch.  Both give
// the same values.
struct PlanarProbe {
    FrameView f;
    typedef float Centre[3];
    __device__ __forceinline__ void centre(int x, int y, Centre cc) const
    {
        const uint8_t* c = f.c(x, y);
        cc[0] = (float)ldg(c);
        cc[1] = (float)ldg(c + 1);
        cc[2] = (float)ldg(c + 2);
    }
    typedef float2 Word;
    __device__ __forceinline__ Word load(int qx, int qy, uint32_t c, bool) const
    {
        return make_float2(f.d(qx, qy), (float)ldg(f.c(qx, qy) + c));
    }
    // the split feature: depth kind D(p) - D(q); colour kind C(p,c) - C(q,c)
    __device__ __forceinline__ float feature(Word v, bool is_depth, uint32_t c, float d, const Centre cc) const
    {
        const float fc = (c == 0u ? cc[0] : c == 1u ? cc[1] : cc[2]) - v.y;
        return is_depth ? d - v.x : fc;
    }
};

struct PackedProbe {
    const uint32_t* img;      // [2][P]: depth bits, then R | G << 8 | B << 16
    uint32_t w, P;
    typedef uint32_t Centre[1];
    __device__ __forceinline__ void centre(int x, int y, Centre cw) const
    {
        cw[0] = ldg(img + P + (uint32_t)y * w + (uint32_t)x);
    }
    typedef uint32_t Word;
    // 32-bit byte offset from the image base (below 2^27 bytes; w * h < 2^24)
    __device__ __forceinline__ Word load(int qx, int qy, uint32_t, bool is_depth) const
    {
        const uint32_t q = __umul24((uint32_t)qy, w) + (uint32_t)qx + (is_depth ? 0u : P);
        return ldg(reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(img) + q * 4u));
    }
    // colour bytes are subtracted as integers: the difference of two bytes
    // converts to the same float as the difference of their conversions
    __device__ __forceinline__ float feature(Word v, bool is_depth, uint32_t c, float d, const Centre cw) const
    {
        const int ci = (int)__builtin_amdgcn_ubfe(cw[0], 8u * c, 8u);
        const int qi = (int)__builtin_amdgcn_ubfe(v, 8u * c, 8u);
        const float fc = (float)(ci - qi);
        const float fd = d - __uint_as_float(v);
        // both features are computed; a bit select picks one without a branch
        const uint32_t m = is_depth ? 0xFFFFFFFFu : 0u;
        return __uint_as_float((__float_as_uint(fd) & m) | (__float_as_uint(fc) & ~m));
    }
};

// route: T trees in lockstep, as described above.  UNIT: the frame is at
// the forest's reference width (s = 1), so the offsets need no scaling (a
// product with 1.0f is exact).  The offset is clamped in float to the
// image's span around the pixel, which lands on the same probe as clamping
// the probe coordinate.  The first ktop levels may be read from a copy of
// the trees' top nodes (top: T x (2^ktop - 1) records, e.g. in LDS; ktop = 0
// reads every level from nodes).
template <int T, bool UNIT, class Probe>
__device__ __forceinline__ void route(const float4* __restrict__ nodes, int NT, int D, const Probe& pr, int w,
                                      int h, int x, int y, float d, float s, int leaf[T],
                                      const float4* top = nullptr, int ktop = 0)
{
    const float inv = 1.0f / d;
    typename Probe::Centre cen;
    pr.centre(x, y, cen);
    const float lox = (float)(-x), hix = (float)(w - 1 - x), loy = (float)(-y), hiy = (float)(h - 1 - y);
    int idx[T];
#pragma unroll
    for (int t = 0; t < T; ++t) idx[t] = 0;
    for (int lvl = 0; lvl < D; ++lvl) {
        float4 nd[T];
        if (lvl < ktop) {
            const int ntop = (1 << ktop) - 1;
#pragma unroll
            for (int t = 0; t < T; ++t) nd[t] = top[t * ntop + idx[t]];
        } else {
#pragma unroll
            for (int t = 0; t < T; ++t)   // 32-bit byte offsets (the forest is below 2^23 bytes)
                nd[t] = ldg(reinterpret_cast<const float4*>(reinterpret_cast<const char*>(nodes) +
                                                            (uint32_t)(t * NT + idx[t]) * 16u));
        }
        // every tree's probe is issued before any is used
        typename Probe::Word pv[T];
        uint32_t ch[T];
        bool dk[T];
#pragma unroll
        for (int t = 0; t < T; ++t) {
            dk[t] = __float_as_uint(nd[t].w) == 0u;
            float fox = rintf((UNIT ? nd[t].x : nd[t].x * s) * inv);
            float foy = rintf((UNIT ? nd[t].y : nd[t].y * s) * inv);
            fox = fminf(fmaxf(fox, lox), hix);
            foy = fminf(fmaxf(foy, loy), hiy);
            // kinds are validated at creation (<= 3); the clamp keeps the
            // colour read inside the pixel whatever the device memory holds
            ch[t] = min(__float_as_uint(nd[t].w) - 1u, 2u);
            pv[t] = pr.load(x + (int)fox, y + (int)foy, ch[t], dk[t]);
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float f = pr.feature(pv[t], dk[t], ch[t], d, cen);
            idx[t] = 2 * idx[t] + 1 + (f >= nd[t].z ? 1 : 0);
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) leaf[t] = idx[t] - NT;
}

// ---------------------------------------------------------------------------
// Rigid fit from the cross-covariance A = sum (x^C - c^C)(x^W - c^W)^T.
// Method: eigen-decomposition of A^T A by cyclic Jacobi rotations gives the
// right singular vectors v1, v2 (largest two); u_k follow from A v_k
// (Gram-Schmidt), and v3 = v1 x v2, u3 = u1 x u2 complete both bases as
// rotations, so R = V U^T is the optimal proper rotation (the signed-SVD
// form of the Kabsch solution).  Degenerate iff sigma_2 < 1e-4 sigma_1,
// i.e. lambda_2 < 1e-8 lambda_1.  R maps camera to world: x^W ~ R x^C + t.
template <int P, int Q>
__device__ __forceinline__ void jacobi_rotate(double (&B)[3][3], double (&V)[3][3])
{
    constexpr int R = 3 - P - Q;
    const double apq = B[P][Q];
    if (apq == 0.0) return;
    const double theta = (B[Q][Q] - B[P][P]) / (2.0 * apq);
    const double tt = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
    const double c = 1.0 / sqrt(tt * tt + 1.0), sn = tt * c;
    const double arp = B[R][P], arq = B[R][Q];
    B[P][P] -= tt * apq;
    B[Q][Q] += tt * apq;
    B[P][Q] = B[Q][P] = 0.0;
    B[R][P] = B[P][R] = c * arp - sn * arq;
    B[R][Q] = B[Q][R] = sn * arp + c * arq;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double vp = V[i][P], vq = V[i][Q];
        V[i][P] = c * vp - sn * vq;
        V[i][Q] = sn * vp + c * vq;
    }
}

// eigenpair (value, column) compare-swap so that the first is the larger
__device__ __forceinline__ void eig_order(double& la, double (&va)[3], double& lb, double (&vb)[3])
{
    if (lb > la) {
        const double tl = la;
        la = lb;
        lb = tl;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double tv = va[i];
            va[i] = vb[i];
            vb[i] = tv;
        }
    }
}

__device__ __forceinline__ bool rigid_from_cov(const double A[9], const double cc[3], const double cw[3],
                                               double R[9], double t[3])
{
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            B[i][j] = A[0 * 3 + i] * A[0 * 3 + j] + A[1 * 3 + i] * A[1 * 3 + j] + A[2 * 3 + i] * A[2 * 3 + j];
    double V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 32; ++sweep) {
        const double off = B[0][1] * B[0][1] + B[0][2] * B[0][2] + B[1][2] * B[1][2];
        const double dia = B[0][0] * B[0][0] + B[1][1] * B[1][1] + B[2][2] * B[2][2];
        if (off <= 1e-32 * dia || off == 0.0) break;
        jacobi_rotate<0, 1>(B, V);
        jacobi_rotate<0, 2>(B, V);
        jacobi_rotate<1, 2>(B, V);
    }
    double l[3] = {B[0][0], B[1][1], B[2][2]};
    double v1[3], v2[3], v3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        v1[i] = V[i][0];
        v2[i] = V[i][1];
        v3[i] = V[i][2];
    }
    eig_order(l[0], v1, l[1], v2);
    eig_order(l[1], v2, l[2], v3);
    eig_order(l[0], v1, l[1], v2);
    if (!(l[0] > 0.0) || l[1] < 1e-8 * l[0]) return false;
    v3[0] = v1[1] * v2[2] - v1[2] * v2[1];
    v3[1] = v1[2] * v2[0] - v1[0] * v2[2];
    v3[2] = v1[0] * v2[1] - v1[1] * v2[0];
    double u1[3], u2[3], u3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        u1[i] = A[i * 3 + 0] * v1[0] + A[i * 3 + 1] * v1[1] + A[i * 3 + 2] * v1[2];
        u2[i] = A[i * 3 + 0] * v2[0] + A[i * 3 + 1] * v2[1] + A[i * 3 + 2] * v2[2];
    }
    const double n1 = sqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    if (!(n1 > 0.0)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) u1[i] /= n1;
    const double pr = u1[0] * u2[0] + u1[1] * u2[1] + u1[2] * u2[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) u2[i] -= pr * u1[i];
    const double n2 = sqrt(u2[0] * u2[0] + u2[1] * u2[1] + u2[2] * u2[2]);
    if (!(n2 > 0.0)) return false;
#pragma unroll
    for (int i = 0; i < 3; ++i) u2[i] /= n2;
    u3[0] = u1[1] * u2[2] - u1[2] * u2[1];
    u3[1] = u1[2] * u2[0] - u1[0] * u2[2];
    u3[2] = u1[0] * u2[1] - u1[1] * u2[0];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i * 3 + j] = v1[i] * u1[j] + v2[i] * u2[j] + v3[i] * u3[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        t[i] = cw[i] - (R[i * 3 + 0] * cc[0] + R[i * 3 + 1] * cc[1] + R[i * 3 + 2] * cc[2]);
    return true;
}

// Per-pixel leaf record: 8 x uint16 leaves packed in a uint4, 8 x uint8 mode
// counts packed in a uint2.  Extraction by shifts keeps runtime tree indices
// in registers (no private-memory arrays).
__device__ __forceinline__ uint32_t leaf_of(uint4 lw, int t)
{
    const uint64_t v = t < 4 ? (((uint64_t)lw.y << 32) | lw.x) : (((uint64_t)lw.w << 32) | lw.z);
    return (uint32_t)(v >> (16 * (t & 3))) & 0xFFFFu;
}

__device__ __forceinline__ uint32_t count_of(uint2 nw, int t)
{
    const uint64_t v = ((uint64_t)nw.y << 32) | nw.x;
    return (uint32_t)(v >> (8 * t)) & 0xFFu;
}

// Eligible-pixel record, one per entry of the eligible list, ew 64-bit words:
//   word 0: |M(u)| (bits 0-7) and the colour-check bits of modes 0..55 of
//           M(u) (bits 8-63)
//   word k >= 1: colour-check bits of modes 56 + 64 (k - 1) ... (only when a
//           pixel can have more than 56 modes)
// The colour check of a (pixel, mode) pair does not depend on the iteration
// that draws it, so it is evaluated once per pair when the list is built; a
// generation iteration then reads one 8-byte word instead of gathering the
// pixel, its leaves, its colour and the mode row, and a frame's table (8 B
// per eligible pixel) stays resident in one XCD's L2.
__device__ __forceinline__ uint32_t erec_total(uint64_t h) { return (uint32_t)h & 0xFFu; }

__device__ __forceinline__ bool erec_bit(const uint64_t* rec, uint64_t h, uint32_t m)
{
    if (m < 56) return (h >> (8 + m)) & 1u;
    const uint32_t k = m - 56;
    return (ldg(rec + 1 + (k >> 6)) >> (k & 63)) & 1u;
}

// Colour box of a mode: per channel, the range [lo, hi] of integer pixel
// values v in 0..255 that pass the colour check !(|v - c| > theta) in float32
// (lo > hi: none).  (float)v - c is monotone in v and so is the rounding, so
// the passing values form an interval, found by testing the few integers
// around c - theta and c + theta.  Packed as lo bytes (R, G, B) in x, hi in y.
__device__ __forceinline__ bool colour_pass(float v, float c, float theta) { return !(fabsf(v - c) > theta); }

__device__ __forceinline__ void colour_range(float c, float theta, uint32_t& lo, uint32_t& hi)
{
    const int s = (int)fminf(fmaxf(floorf(c - theta) - 1.0f, 0.0f), 255.0f);
    const int e = (int)fminf(fmaxf(ceilf(c + theta) + 1.0f, 0.0f), 255.0f);
    lo = 1u;
    hi = 0u;
    for (int v = s; v <= min(s + 3, 255); ++v)
        if (colour_pass((float)v, c, theta)) {
            lo = (uint32_t)v;
            break;
        }
    for (int v = e; v >= max(e - 3, 0); --v)
        if (colour_pass((float)v, c, theta)) {
            hi = (uint32_t)v;
            break;
        }
    if (hi < lo) {
        lo = 1u;
        hi = 0u;
    }
}

// Colour boxes hold their three channel bounds in 10-bit fields
// (c0 | c1 << 10 | c2 << 20), so that all three comparisons of a box are two
// subtractions: with a guard bit 9 set in every field of the minuend, field
// k of (x | G) - lo keeps its guard bit iff x_k >= lo_k, and likewise for
// (hi | G) - x (no field borrows: every operand byte is below 256).
constexpr uint32_t kBoxGuard = (1u << 9) | (1u << 19) | (1u << 29);

__device__ __forceinline__ uint32_t spread3(uint32_t c0, uint32_t c1, uint32_t c2) { return c0 | (c1 << 10) | (c2 << 20); }

__device__ __forceinline__ uint2 colour_box(float r, float g, float b, float theta)
{
    uint32_t l0, h0, l1, h1, l2, h2;
    colour_range(r, theta, l0, h0);
    colour_range(g, theta, l1, h1);
    colour_range(b, theta, l2, h2);
    return make_uint2(spread3(l0, l1, l2), spread3(h0, h1, h2));
}

// the pixel's colour in box form, from R | G << 8 | B << 16
__device__ __forceinline__ uint32_t box_colour(uint32_t rgb)
{
    return spread3(rgb & 0xFFu, (rgb >> 8) & 0xFFu, (rgb >> 16) & 0xFFu);
}

// x: box_colour of the pixel
__device__ __forceinline__ bool box_pass(uint2 box, uint32_t x)
{
    return (((x | kBoxGuard) - box.x) & ((box.y | kBoxGuard) - x) & kBoxGuard) == kBoxGuard;
}

__device__ __forceinline__ int modes_total(uint2 nw, int T)
{
    int n = 0;
    for (int t = 0; t < T; ++t) n += (int)count_of(nw, t);
    return n;
}

// Mode row m of M(u), the tree-major concatenation of the leaves' modes.
__device__ __forceinline__ const float4* mode_row(const float4* __restrict__ modes, int T, int D,
                                                  int M, uint4 lw, uint2 nw, int m)
{
    int t = 0;
    for (; t < T - 1; ++t) {
        const int c = (int)count_of(nw, t);
        if (m < c) break;
        m -= c;
    }
    const size_t row = (((size_t)t << D) + leaf_of(lw, t)) * (size_t)M + (size_t)m;
    return modes + row * 4;
}

}  // namespace rl
