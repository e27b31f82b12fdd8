// rl_runtime.hip -- host runtime and C ABI of librl (see include/rl.h).
//
// All device state lives in caller-provided buffers; this file computes
// their layouts, validates every argument before any launch, fills the job
// tables and queues the kernel sequences on the caller's stream.  Batches
// can be captured into a HIP graph per batch shape and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "rl_internal.hpp"

#define RL_API extern "C" __attribute__((visibility("default")))

namespace rl {
hipError_t launch_prep(const Job* jobs, int njobs, int maxN, hipStream_t st);
hipError_t launch_traverse(const Job* jobs, int njobs, int maxP, int T, int top, hipStream_t st);
hipError_t launch_eligible(const Job* jobs, int njobs, int maxP, int T, hipStream_t st);
hipError_t launch_hyp_search(const Job* jobs, int njobs, int maxN, int maxIters, int ipt, hipStream_t st);
hipError_t launch_hyp_finalize(const Job* jobs, int njobs, int maxN, hipStream_t st);
hipError_t launch_score(const Job* jobs, int njobs, int round, int nptiles, int maxSurv,
                        hipStream_t st);
hipError_t launch_score_all(const Job* jobs, int njobs, int rounds, int nptiles, int fw, int window, hipStream_t st);
hipError_t launch_lm(const Job* jobs, int njobs, int round, int maxSurv, int maxEta, int maxRows, int maxIters,
                     bool split, hipStream_t st);
hipError_t launch_select(const Job* jobs, int njobs, int round, int nptiles, int maxN, hipStream_t st);
hipError_t launch_finalize(const Job* jobs, int njobs, int maxIlen, hipStream_t st);
hipError_t launch_depth_scores(const FrameView& src, int w, int h, float fx, float fy, float cx, float cy,
                               const float* surfaces, int n_surf, const float* poses, int n_poses, float zmin,
                               float zmax, double* partial, int* cnt, double* out, long long* counts,
                               hipStream_t st);
hipError_t launch_plane_scores(const FrameView& src, int w, int h, float fx, float fy, float cx, float cy,
                               const float* surfaces, int n_surf, const float* poses, int n_poses,
                               double* partial, int* cnt, double* scores, hipStream_t st);
hipError_t launch_adapt(const AdaptArgs& a, hipStream_t st);
hipError_t launch_rqs(const RqsArgs& a, int blocks, hipStream_t st);
hipError_t launch_adapt_jobs(const AdaptArgs* jobs, const AdaptArgs* hjobs, int njobs, hipStream_t st);
hipError_t launch_rqs_jobs(const RqsArgs* jobs, const RqsArgs* hjobs, int njobs, int blocks, hipStream_t st);

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, size_t n, uint8_t v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}
}  // namespace rl

using namespace rl;

namespace {

thread_local std::string g_err;

rl_status fail(rl_status s, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

rl_status hip_fail(hipError_t e, const char* what)
{
    return fail(RL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Carver {
    size_t cur = 0;
    size_t take(size_t bytes)
    {
        const size_t o = cur;
        cur += align256(bytes);
        return o;
    }
};

int rounds_for(int N, int n_cull, int n_out, std::vector<int>* entering = nullptr)
{
    int n = N, rounds = 0;
    bool first = true;
    while (first || n > n_out) {
        if (entering) entering->push_back(n);
        int keep = n;
        if (first && n_cull < n) keep = n_cull;
        else if (n > n_out) keep = (n + 1) / 2;
        n = keep;
        ++rounds;
        first = false;
        if (rounds > 64) break;
    }
    return rounds;
}

// Rounds any call on a room may need: N' <= N hypotheses, any cull, any
// n_out >= 1 take at most the rounds of N without cull down to one.
int rounds_capacity(const rl_params& p)
{
    return std::max(rounds_for(p.max_pose_candidates, p.max_pose_candidates_after_cull,
                               p.max_relocalisations_to_output),
                    rounds_for(p.max_pose_candidates, p.max_pose_candidates, 1));
}

// Pixels per scoring wave: every lane of a wave reads the same mode rows, so
// no shared memory is staged and the tile size does not depend on |M(u)|.
int score_tile(int) { return kScoreTile; }

// Per-frame (relocalisation) scratch of one job slot.
struct FrameLayout {
    size_t state, result, probe, leaves, nmt, nm, tile_count, eligible, ecold, erec, hyp_best, hyps, surv, E, partial,
        partial_all, pose64, lm_state, lm_part, Ie, lm_plan, lm_px, lm_rows,
        I, inl, trace_slots, trace_E, total;
    int ew;
    int lm_icap;
};

// 64-bit words per eligible-pixel record: |M(u)| and 56 colour-check bits in
// the first, 64 more bits per further word.
int erec_words(int rows_per_pixel)
{
    return 1 + (std::max(rows_per_pixel - 56, 0) + 63) / 64;
}

FrameLayout frame_layout(int maxP, int N, int eta, int rounds, int TP, int rows_per_pixel, size_t base)
{
    Carver c;
    c.cur = base;
    FrameLayout L;
    L.state = c.take(sizeof(JobState));
    L.result = c.take(sizeof(rl_result));
    L.probe = c.take((size_t)maxP * 8);                  // two planes of w h words
    L.leaves = c.take((size_t)maxP * 16);
    L.nmt = c.take((size_t)maxP * 8);
    L.nm = c.take((size_t)maxP);
    L.tile_count = c.take((size_t)((maxP + 255) / 256) * 4);
    L.eligible = c.take((size_t)maxP * 4);
    L.ecold = c.take((size_t)maxP * 32);
    L.ew = erec_words(rows_per_pixel);
    L.erec = c.take((size_t)maxP * L.ew * 8);
    L.hyp_best = c.take((size_t)N * 4);
    L.hyps = c.take((size_t)N * sizeof(Hyp));
    L.surv = c.take((size_t)N * 4);
    L.E = c.take((size_t)N * 8);
    L.pose64 = c.take((size_t)N * 96);
    // LM partials of round r >= 1: (survivor, tile) pairs, at most N / 2^(r-1)
    // (rounded up) survivors times the tiles of (r + 1) eta pixels
    size_t lm_pairs = 0;
    for (int r = 1, n = N; r < rounds; ++r, n = (n + 1) / 2)
        lm_pairs = std::max(lm_pairs, (size_t)n * (size_t)(((r + 1) * eta + kLmTile - 1) / kLmTile));
    L.lm_state = c.take((size_t)N * kLmStateDoubles * 8);
    L.lm_part = c.take(lm_pairs * kLmVals * 8);
    L.Ie = c.take((size_t)rounds * eta * 4);
    L.lm_plan = c.take((size_t)2 * (kMaxBatchFrames + 1) * 4);   // item plan, survivor plan
    L.lm_icap = rounds * eta;
    L.lm_px = c.take((size_t)rounds * eta * 32);
    L.lm_rows = c.take((size_t)rounds * eta * rows_per_pixel * 48);
    const int ptiles = (eta + TP - 1) / TP;
    L.partial = c.take((size_t)ptiles * N * 8);
    L.partial_all = c.take((size_t)rounds * ptiles * kFastStride * 8);
    L.I = c.take((size_t)rounds * eta * 4);
    L.inl = c.take((size_t)rounds * eta * 4);
    L.trace_slots = c.take((size_t)rounds * N * 4);
    L.trace_E = c.take((size_t)rounds * N * 8);
    L.total = c.cur - base;
    return L;
}

struct PersistLayout {
    size_t nodes, reservoir, seen, dirty, dirty_list, counters, modes, nmodes, cbox, total;
};

PersistLayout persist_layout(const rl_params& p)
{
    const size_t T = p.n_trees, L = (size_t)1 << p.depth, NT = L - 1;
    Carver c;
    PersistLayout P;
    P.nodes = c.take(T * NT * 16);
    P.reservoir = c.take(T * L * (size_t)p.reservoir_capacity * 16);
    P.seen = c.take(T * L * 4);
    P.dirty = c.take(T * L * 4);
    P.dirty_list = c.take(T * L * 4);
    P.counters = c.take(256);
    P.modes = c.take(T * L * (size_t)p.max_cluster_count * 64);
    P.nmodes = c.take(T * L);
    P.cbox = c.take(T * L * (size_t)p.max_cluster_count * 8);
    P.total = c.cur;
    return P;
}


// Scratch of the model-based score: surfaces, poses, per-tile partials, scores.
// host staging of the model scores: surfaces, poses, plane scores, depth
// scores (s, mu) and counts
constexpr size_t kModelHostBytes = (size_t)kMaxModelSurfaces * 64 + (size_t)kMaxModelPoses * (48 + 8 + 16 + 16);

struct ModelLayout {
    size_t surfaces, poses, partial, cnt, scores, dpartial, dcnt, dout, dcounts, total;
};

ModelLayout model_layout(int maxP, size_t base)
{
    Carver c;
    c.cur = base;
    ModelLayout L;
    const size_t ntiles = (size_t)(maxP + 1023) / 1024;
    L.surfaces = c.take((size_t)kMaxModelSurfaces * 64);
    L.poses = c.take((size_t)kMaxModelPoses * 48);
    L.partial = c.take(ntiles * kMaxModelPoses * 8);
    L.cnt = c.take(ntiles * 4);
    L.scores = c.take((size_t)kMaxModelPoses * 8);
    L.dpartial = c.take(ntiles * kMaxModelPoses * 8);
    L.dcnt = c.take(ntiles * kMaxModelPoses * 2 * 4);
    L.dout = c.take((size_t)kMaxModelPoses * 2 * 8);
    L.dcounts = c.take((size_t)kMaxModelPoses * 2 * 8);
    L.total = c.cur - base;
    return L;
}

struct AdaptLayout {
    size_t item_leaf, item_pt, item_run, item_lrank, item_n, item_slot, item_h, run_cnt, run_tl, run_next, run_pre,
        run_tot, head, hkey, hval, rr_rho, rr_parent, total;
    int Gp;
    uint32_t hsize;
};

// adaptation table entries: a power of two >= 2 T G (at least 256)
uint32_t adapt_table_size(int T, int G)
{
    uint32_t s = 256;
    while (s < 2u * (uint32_t)T * (uint32_t)G) s <<= 1;
    return s;
}

AdaptLayout adapt_layout(const rl_params& p, int G, size_t base)
{
    const size_t T = p.n_trees, L = (size_t)1 << p.depth;
    Carver c;
    c.cur = base;
    AdaptLayout A;
    A.Gp = (G + kAdaptChunk - 1) / kAdaptChunk * kAdaptChunk;
    A.hsize = adapt_table_size(p.n_trees, G);
    const size_t TG = T * (size_t)G, TGp = T * (size_t)A.Gp;
    A.item_leaf = c.take(TG * 2);
    A.item_pt = c.take((size_t)G * 16);
    A.item_run = c.take(TG * 4);
    A.item_lrank = c.take(TG * 2);
    A.item_n = c.take(TG * 4);
    A.item_slot = c.take(TG * 4);
    A.item_h = c.take(TG * 4);
    A.run_cnt = c.take(TGp * 4);
    A.run_tl = c.take(TGp * 4);
    A.run_next = c.take(TGp * 4);
    A.run_pre = c.take(TGp * 4);
    A.run_tot = c.take(TGp * 4);
    A.head = c.take(T * L * 4);
    A.hkey = c.take((size_t)A.hsize * 4);
    A.hval = c.take((size_t)A.hsize * 4);
    A.rr_rho = c.take((size_t)kRqsSplitLeaves * (size_t)p.reservoir_capacity * 8);
    A.rr_parent = c.take((size_t)kRqsSplitLeaves * (size_t)p.reservoir_capacity * 4);
    A.total = c.cur - base;
    return A;
}

int grid_items(int w, int h) { return (w / 4 - 1) * (h / 4 - 1); }

bool finite_f(float v) { return std::isfinite(v); }

rl_status validate_frame(const rl_frame* f, int max_w, int max_h)
{
    if (!f) return fail(RL_EINVAL, "frame is NULL");
    if (f->width <= 0 || f->height <= 0 || f->width % 4 || f->height % 4)
        return fail(RL_EINVAL, "frame size %dx%d: width and height must be positive multiples of 4",
                    f->width, f->height);
    if (f->width < 8 || f->height < 8) return fail(RL_EINVAL, "frame must be at least 8x8");
    if (f->width > max_w || f->height > max_h)
        return fail(RL_EINVAL, "frame %dx%d exceeds the %dx%d the scratch was sized for", f->width,
                    f->height, max_w, max_h);
    if (!f->depth || !f->rgb) return fail(RL_EINVAL, "frame depth/rgb pointer is NULL");
    if (f->rgb_channels != 0 && f->rgb_channels != 3 && f->rgb_channels != 4)
        return fail(RL_EINVAL, "rgb_channels must be 3 or 4 (0 = 3), got %d", f->rgb_channels);
    if (f->step != 0 && f->step != 1 && f->step != 2) return fail(RL_EINVAL, "step must be 1 or 2 (0 = 1)");
    const long long st = f->step ? f->step : 1, ch = f->rgb_channels ? f->rgb_channels : 3;
    if (f->depth_pitch_bytes != 0 && (f->depth_pitch_bytes < 4 * st * f->width || f->depth_pitch_bytes % 4))
        return fail(RL_EINVAL, "depth_pitch_bytes %d: at least %lld and a multiple of 4", f->depth_pitch_bytes,
                    4 * st * f->width);
    if (f->rgb_pitch_bytes != 0 && f->rgb_pitch_bytes < ch * st * f->width)
        return fail(RL_EINVAL, "rgb_pitch_bytes %d: at least %lld", f->rgb_pitch_bytes, ch * st * f->width);
    if (((uintptr_t)f->depth & 3) != 0) return fail(RL_EINVAL, "depth must be 4-byte aligned");
    const rl_intrinsics& K = f->K;
    if (!(finite_f(K.fx) && finite_f(K.fy) && finite_f(K.cx) && finite_f(K.cy)) || !(K.fx > 0) || !(K.fy > 0))
        return fail(RL_EINVAL, "invalid intrinsics");
    return RL_OK;
}

// The device view of a validated frame (zero fields take their defaults).
FrameView frame_view(const rl_frame* f)
{
    FrameView v;
    v.depth = f->depth;
    v.rgb = f->rgb;
    v.step = f->step ? (uint32_t)f->step : 1u;
    v.ch = f->rgb_channels ? (uint32_t)f->rgb_channels : 3u;
    v.dpitch = f->depth_pitch_bytes ? (uint32_t)f->depth_pitch_bytes : 4u * v.step * (uint32_t)f->width;
    v.rpitch = f->rgb_pitch_bytes ? (uint32_t)f->rgb_pitch_bytes : v.ch * v.step * (uint32_t)f->width;
    return v;
}

uint64_t stream_key64(uint64_t seed, uint64_t request_seed)
{
    return seed + request_seed * 0x9E3779B97F4A7C15ULL;
}

int device_lds_limit()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 65536;
    return v;
}

// Optional HIP-event pair recorded around one kernel of the sequence.
struct Timer {
    int kernel = RL_TIMER_NONE;
    hipEvent_t start = nullptr, stop = nullptr;
};

}  // namespace

// Launch shapes that leave every result unchanged (the search's and the
// scoring's arithmetic and summation orders do not depend on them): search
// iterations per thread, and the width in waves of the all-rounds scoring.
struct Schedule {
    int ipt = 4;
    int fw = 1;
    int top = kTopLevelsMax;   // tree levels the traversal reads from LDS
    int win = 0;   // rounds of the first all-rounds scoring pass (0: every remaining round in one pass)
    int screen = 1;   // the search rejects clearly degenerate triplets (else only the exact test does)
};

struct rl_room {
    rl_params p;
    int T, D, M, kappa, N, eta, rounds, TP;
    size_t L;
    int max_w, max_h, maxP, G;
    char* pers;
    char* scr;
    PersistLayout PL;
    FrameLayout FL;
    AdaptLayout AL;
    ModelLayout ML;
    size_t job_off;
    char* model_host;
    int rounds_cap;
    hipStream_t stream;
    hipEvent_t ev;
    // Access order of the room's persistent state by batches on other
    // streams: batches only read it (forest, modes); the mode update (RQS) is
    // the only writer they can race with.  wev marks the last mode update;
    // readers are events the room recorded on batch streams after batches
    // that read it since then (a pool, reused).
    hipEvent_t wev;
    bool wrote;
    // bev marks the work queued so far on the room's stream, for a batch that
    // adapts the room to wait on (the room's stream then waits for that batch)
    hipEvent_t bev;
    uint32_t mode_version;    // mode updates queued so far (each RQS launch)
    std::vector<hipEvent_t> readers, spare;
    Job* job_host;
    rl_result* res_host;
    int trace;
    bool modes_stale;         // leaves adapted since the last exact mode update
    int rr_leaves;            // 0: exact mode update before relocalising; K: K leaves per adapted frame
    uint32_t rr_cursor;       // next leaf of the round-robin schedule
    std::vector<int> entering;
    Schedule sched;
    Timer timer;
    std::map<std::vector<long long>, hipGraphExec_t> graphs;
};

// Pinned job tables of the batch path: a call fills one while the copies of
// earlier calls may still be queued behind running batches, so they rotate,
// and a table is refilled only after the event marking its last upload.
constexpr int kJobRing = 4;

struct rl_batch {
    rl_batch_params bp;
    char* ws;
    hipStream_t stream;
    hipEvent_t ev;
    hipEvent_t mark;          // end of the batch's adaptations, for the rooms' streams to wait on
    int TP, rows;
    size_t jobs_off, results_off, ad_off, rq_off;
    std::vector<FrameLayout> slots;
    Schedule sched;
    Timer timer;
    Job* job_ring[kJobRing];
    hipEvent_t up_ev[kJobRing];
    int ring;
    // adaptation job tables: pinned host copies ([max_frames] AdaptArgs, then
    // [max_frames] RqsArgs) and their upload events, a ring like job_ring
    char* ad_ring[kJobRing];
    hipEvent_t ad_ev[kJobRing];
    int ad_slot;
    rl_result* res_host;
    std::map<std::vector<long long>, hipGraphExec_t> graphs;
};

// ------------------------------------------------------------------------
RL_API const char* rl_last_error(void) { return g_err.c_str(); }
RL_API const char* rl_version(void) { return "librl 0.1 (gfx950)"; }

RL_API rl_status rl_params_preset(const char* name, rl_params* out)
{
    if (!name || !out) return fail(RL_EINVAL, "NULL argument");
    rl_params p;
    std::memset(&p, 0, sizeof(p));
    p.n_trees = 5;
    p.depth = 15;
    p.ref_width = 640;
    p.max_colour_linf = 30.0f;
    p.inlier_threshold = 0.05f;
    p.cov_regulariser = 1e-6f;
    p.clusterer_sigma = 0.1f;
    p.max_cluster_count = 50;
    p.max_pose_candidates_after_cull = 64;
    p.lm_iterations = 10;
    const std::string n(name);
    if (n == "default") {
        p.clusterer_tau = 0.05f; p.min_cluster_size = 20; p.reservoir_capacity = 1024;
        p.max_candidate_generation_iterations = 6000; p.max_pose_candidates = 1024;
        p.max_translation_error_for_correct_pose = 0.05f;
        p.min_squared_distance_between_sampled_modes = 0.09f; p.pose_update = 1;
        p.ransac_inliers_per_iteration = 512; p.use_prediction_covariance = 1;
        p.max_relocalisations_to_output = 16;
    } else if (n == "fast") {
        p.clusterer_tau = 0.2f; p.min_cluster_size = 5; p.reservoir_capacity = 2048;
        p.max_candidate_generation_iterations = 500; p.max_pose_candidates = 2048;
        p.max_translation_error_for_correct_pose = 0.05f;
        p.min_squared_distance_between_sampled_modes = 0.0f; p.pose_update = 0;
        p.ransac_inliers_per_iteration = 256; p.use_prediction_covariance = 0;
        p.max_relocalisations_to_output = 1;
    } else if (n == "intermediate") {
        p.clusterer_tau = 0.2f; p.min_cluster_size = 5; p.reservoir_capacity = 2048;
        p.max_candidate_generation_iterations = 1000; p.max_pose_candidates = 2048;
        p.max_translation_error_for_correct_pose = 0.1f;
        p.min_squared_distance_between_sampled_modes = 0.09f; p.pose_update = 1;
        p.ransac_inliers_per_iteration = 256; p.use_prediction_covariance = 0;
        p.max_relocalisations_to_output = 1;
    } else if (n == "slow") {
        p.clusterer_tau = 0.2f; p.min_cluster_size = 5; p.reservoir_capacity = 2048;
        p.max_candidate_generation_iterations = 250; p.max_pose_candidates = 2048;
        p.max_translation_error_for_correct_pose = 0.1f;
        p.min_squared_distance_between_sampled_modes = 0.0225f; p.pose_update = 1;
        p.ransac_inliers_per_iteration = 256; p.use_prediction_covariance = 0;
        p.max_relocalisations_to_output = 16;
    } else if (n == "c1" || n == "c2" || n == "c3" || n == "c4" || n == "c5") {
        p.clusterer_tau = 0.05f; p.min_cluster_size = 20; p.max_cluster_count = 10;
        p.reservoir_capacity = 1024; p.max_candidate_generation_iterations = 6000;
        p.max_pose_candidates = 1024; p.max_pose_candidates_after_cull = 1024;
        p.max_translation_error_for_correct_pose = 0.05f;
        p.min_squared_distance_between_sampled_modes = 0.09f; p.pose_update = 0;
        p.ransac_inliers_per_iteration = 500; p.use_prediction_covariance = 1;
        p.max_relocalisations_to_output = 1; p.final_refine = 1;
        if (n == "c1") {
            p.n_trees = 1; p.depth = 8; p.ref_width = 160; p.clusterer_tau = 0.2f;
            p.min_cluster_size = 5; p.max_cluster_count = 5; p.reservoir_capacity = 64;
            p.max_pose_candidates = 64; p.max_pose_candidates_after_cull = 64;
            p.ransac_inliers_per_iteration = 100; p.final_refine = 0;
        } else if (n == "c3") {
            p.max_pose_candidates = 4096; p.max_pose_candidates_after_cull = 4096;
            p.max_relocalisations_to_output = 16; p.final_refine = 0;
        }
    } else {
        return fail(RL_EINVAL, "unknown preset '%s'", name);
    }
    *out = p;
    return RL_OK;
}

RL_API rl_status rl_params_validate(const rl_params* p)
{
    if (!p) return fail(RL_EINVAL, "params is NULL");
    if (p->n_trees < 1 || p->n_trees > kMaxTrees) return fail(RL_EINVAL, "n_trees must be in 1..8");
    if (p->depth < 1 || p->depth > 15) return fail(RL_EINVAL, "depth must be in 1..15");
    if (p->ref_width < 1) return fail(RL_EINVAL, "ref_width must be positive");
    if (p->max_cluster_count < 1 || p->max_cluster_count > 64) return fail(RL_EINVAL, "max_cluster_count must be in 1..64");
    if (p->n_trees * p->max_cluster_count > 255) return fail(RL_EINVAL, "n_trees * max_cluster_count must be <= 255");
    if (p->min_cluster_size < 1) return fail(RL_EINVAL, "min_cluster_size must be >= 1");
    if (p->reservoir_capacity < 1 || p->reservoir_capacity > 4096) return fail(RL_EINVAL, "reservoir_capacity must be in 1..4096");
    if (p->max_candidate_generation_iterations < 1 || p->max_candidate_generation_iterations >= (1 << 30))
        return fail(RL_EINVAL, "max_candidate_generation_iterations must be in 1..2^30-1");
    if (p->max_pose_candidates < 1 || p->max_pose_candidates > 4096) return fail(RL_EINVAL, "max_pose_candidates must be in 1..4096");
    if (p->max_pose_candidates_after_cull < 1) return fail(RL_EINVAL, "max_pose_candidates_after_cull must be >= 1");
    if (p->ransac_inliers_per_iteration < 1 || p->ransac_inliers_per_iteration > 4096) return fail(RL_EINVAL, "ransac_inliers_per_iteration must be in 1..4096");
    if (p->max_relocalisations_to_output < 1) return fail(RL_EINVAL, "max_relocalisations_to_output must be >= 1");
    if (p->pose_update != 0 && p->pose_update != 1) return fail(RL_EINVAL, "pose_update must be 0 or 1");
    if (p->lm_iterations < 0 || p->lm_iterations > 64) return fail(RL_EINVAL, "lm_iterations must be in 0..64");
    if (p->use_prediction_covariance != 0 && p->use_prediction_covariance != 1)
        return fail(RL_EINVAL, "use_prediction_covariance must be 0 or 1");
    const float fs[] = {p->clusterer_sigma, p->clusterer_tau, p->min_squared_distance_between_sampled_modes,
                        p->max_translation_error_for_correct_pose, p->max_colour_linf, p->inlier_threshold,
                        p->cov_regulariser};
    for (float v : fs)
        if (!finite_f(v) || v < 0) return fail(RL_EINVAL, "float parameters must be finite and >= 0");
    if (!(p->clusterer_sigma > 0)) return fail(RL_EINVAL, "clusterer_sigma must be > 0");
    if ((long long)p->max_candidate_generation_iterations * p->max_pose_candidates > 0x7fffffffLL * 200LL)
        return fail(RL_EINVAL, "too many generation iterations");
    return RL_OK;
}

RL_API rl_status relocaliser_state_bytes(const rl_params* p, int32_t max_width, int32_t max_height,
                                         size_t* persistent, size_t* scratch)
{
    rl_status s = rl_params_validate(p);
    if (s != RL_OK) return s;
    if (max_width < 8 || max_height < 8 || max_width % 4 || max_height % 4)
        return fail(RL_EINVAL, "max frame size must be multiples of 4, at least 8x8");
    if ((long long)max_width * max_height >= kMaxPixels) return fail(RL_EINVAL, "max frame must have fewer than 2^24 pixels");
    if (!persistent || !scratch) return fail(RL_EINVAL, "NULL output");
    const int N = p->max_pose_candidates, eta = p->ransac_inliers_per_iteration;
    const int R = rounds_capacity(*p);
    const int TP = score_tile(p->n_trees * p->max_cluster_count);
    *persistent = persist_layout(*p).total;
    const size_t job = align256(sizeof(Job));
    const FrameLayout FL = frame_layout(max_width * max_height, N, eta, R, TP, p->n_trees * p->max_cluster_count, job);
    const AdaptLayout AL = adapt_layout(*p, grid_items(max_width, max_height), job + FL.total);
    const ModelLayout ML = model_layout(max_width * max_height, job + FL.total + AL.total);
    *scratch = job + FL.total + AL.total + ML.total;
    return RL_OK;
}

static Job make_job(const rl_room* r, char* scr, const FrameLayout& FL, const rl_frame* f,
                    uint64_t request_seed, int N)
{
    Job J;
    std::memset(&J, 0, sizeof(J));
    J.nodes = reinterpret_cast<const float4*>(r->pers + r->PL.nodes);
    J.modes = reinterpret_cast<const float4*>(r->pers + r->PL.modes);
    J.nmodes = reinterpret_cast<const uint8_t*>(r->pers + r->PL.nmodes);
    J.cbox = reinterpret_cast<const uint2*>(r->pers + r->PL.cbox);
    J.T = r->T;
    J.D = r->D;
    J.M = r->M;
    J.src = frame_view(f);
    J.mode_version = r->mode_version;
    J.w = f->width;
    J.h = f->height;
    J.fx = f->K.fx;
    J.fy = f->K.fy;
    J.cx = f->K.cx;
    J.cy = f->K.cy;
    J.s = (float)f->width / (float)r->p.ref_width;
    J.N = N;
    J.I_max = r->p.max_candidate_generation_iterations;
    J.eta = r->eta;
    J.n_cull = r->p.max_pose_candidates_after_cull;
    J.n_out = r->p.max_relocalisations_to_output;
    J.use_cov = r->p.use_prediction_covariance;
    J.final_refine = r->p.final_refine;
    J.trace = r->trace;
    J.theta_col = r->p.max_colour_linf;
    J.TP = r->TP;
    J.fast_max = 64 * r->sched.fw;
    J.screen = r->sched.screen;
    J.lm = r->p.pose_update;
    J.lm_iters = r->p.lm_iterations;
    J.min_sq_dist = r->p.min_squared_distance_between_sampled_modes;
    J.theta_rig = r->p.max_translation_error_for_correct_pose;
    J.theta_in = r->p.inlier_threshold;
    const uint64_t k = stream_key64(r->p.seed, request_seed);
    J.key0 = (uint32_t)k;
    J.key1 = (uint32_t)(k >> 32);
    J.probe = reinterpret_cast<uint32_t*>(scr + FL.probe);
    J.leaves = reinterpret_cast<uint16_t*>(scr + FL.leaves);
    J.nmt = reinterpret_cast<uint8_t*>(scr + FL.nmt);
    J.nm = reinterpret_cast<uint8_t*>(scr + FL.nm);
    J.tile_count = reinterpret_cast<int*>(scr + FL.tile_count);
    J.eligible = reinterpret_cast<int*>(scr + FL.eligible);
    J.ecold = reinterpret_cast<uint4*>(scr + FL.ecold);
    J.erec = reinterpret_cast<uint64_t*>(scr + FL.erec);
    J.ew = FL.ew;
    J.hyp_best = reinterpret_cast<int*>(scr + FL.hyp_best);
    J.hyps = reinterpret_cast<Hyp*>(scr + FL.hyps);
    J.surv = reinterpret_cast<int*>(scr + FL.surv);
    J.E = reinterpret_cast<double*>(scr + FL.E);
    J.pose64 = reinterpret_cast<double*>(scr + FL.pose64);
    J.lm_state = reinterpret_cast<double*>(scr + FL.lm_state);
    J.lm_part = reinterpret_cast<double*>(scr + FL.lm_part);
    J.Ie = reinterpret_cast<int*>(scr + FL.Ie);
    J.lm_plan = reinterpret_cast<int*>(scr + FL.lm_plan);
    J.lm_px = reinterpret_cast<double4*>(scr + FL.lm_px);
    J.lm_rows = reinterpret_cast<float4*>(scr + FL.lm_rows);
    J.lm_icap = FL.lm_icap;
    J.lm_split = 1;                         // one frame per launch: split rows (a batch resets it)
    J.partial = reinterpret_cast<double*>(scr + FL.partial);
    J.partial_all = reinterpret_cast<double*>(scr + FL.partial_all);
    J.I = reinterpret_cast<int*>(scr + FL.I);
    J.inl = reinterpret_cast<int*>(scr + FL.inl);
    J.trace_slots = reinterpret_cast<int*>(scr + FL.trace_slots);
    J.trace_E = reinterpret_cast<double*>(scr + FL.trace_E);
    J.st = reinterpret_cast<JobState*>(scr + FL.state);
    J.result = reinterpret_cast<rl_result*>(scr + FL.result);
    return J;
}

static RqsArgs rqs_args(rl_room* r)
{
    RqsArgs a;
    a.reservoir = reinterpret_cast<const float4*>(r->pers + r->PL.reservoir);
    a.seen = reinterpret_cast<const uint32_t*>(r->pers + r->PL.seen);
    a.dirty = reinterpret_cast<uint32_t*>(r->pers + r->PL.dirty);
    a.dirty_list = reinterpret_cast<const uint32_t*>(r->pers + r->PL.dirty_list);
    a.counters = reinterpret_cast<uint32_t*>(r->pers + r->PL.counters);
    a.modes = reinterpret_cast<float4*>(r->pers + r->PL.modes);
    a.nmodes = reinterpret_cast<uint8_t*>(r->pers + r->PL.nmodes);
    a.kappa = r->kappa;
    a.M = r->M;
    a.min_size = r->p.min_cluster_size;
    a.sigma = r->p.clusterer_sigma;
    a.tau = r->p.clusterer_tau;
    a.lambda = r->p.cov_regulariser;
    a.cbox = reinterpret_cast<uint2*>(r->pers + r->PL.cbox);
    a.theta_col = r->p.max_colour_linf;
    a.rr_first = 0;
    a.rr_count = 0;
    a.n_leaves = (uint32_t)(r->T * r->L);
    a.rr_rho = reinterpret_cast<double*>(r->scr + r->AL.rr_rho);
    a.rr_parent = reinterpret_cast<int*>(r->scr + r->AL.rr_parent);
    return a;
}

static rl_status fill_u32(void* p, size_t n, uint32_t v, hipStream_t st)
{
    if (n == 0) return RL_OK;
    k_fill_u32<<<dim3(1024), dim3(256), 0, st>>>(reinterpret_cast<uint32_t*>(p), n, v);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RL_OK : hip_fail(e, "fill");
}

static rl_status fill_u8(void* p, size_t n, uint8_t v, hipStream_t st)
{
    if (n == 0) return RL_OK;
    k_fill_u8<<<dim3(1024), dim3(256), 0, st>>>(reinterpret_cast<uint8_t*>(p), n, v);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RL_OK : hip_fail(e, "fill");
}

RL_API rl_status relocaliser_create(const rl_params* p, const rl_node* host_nodes, int32_t max_width,
                                    int32_t max_height, void* dev_persistent, void* dev_scratch,
                                    void* hip_stream, rl_room** out)
{
    if (!out) return fail(RL_EINVAL, "out is NULL");
    *out = nullptr;
    size_t pb = 0, sb = 0;
    rl_status s = relocaliser_state_bytes(p, max_width, max_height, &pb, &sb);
    if (s != RL_OK) return s;
    if (!host_nodes || !dev_persistent || !dev_scratch) return fail(RL_EINVAL, "NULL buffer");
    if (((uintptr_t)dev_persistent & 255) || ((uintptr_t)dev_scratch & 255))
        return fail(RL_EINVAL, "device buffers must be 256-byte aligned");
    const size_t NT = ((size_t)1 << p->depth) - 1;
    for (size_t i = 0; i < (size_t)p->n_trees * NT; ++i) {
        const rl_node& nd = host_nodes[i];
        if (nd.kind > 3 || !finite_f(nd.dx) || !finite_f(nd.dy) || !finite_f(nd.tau))
            return fail(RL_EINVAL, "node %zu: kind must be 0..3 and parameters finite", i);
    }
    const int lds = device_lds_limit();
    if ((size_t)36 * p->reservoir_capacity + 4096 > (size_t)lds)
        return fail(RL_EINVAL, "reservoir_capacity %d needs %zu bytes of LDS per workgroup; device allows %d",
                    p->reservoir_capacity, (size_t)36 * p->reservoir_capacity + 4096, lds);
    rl_room* r = new rl_room();
    r->p = *p;
    r->T = p->n_trees;
    r->D = p->depth;
    r->M = p->max_cluster_count;
    r->kappa = p->reservoir_capacity;
    r->N = p->max_pose_candidates;
    r->eta = p->ransac_inliers_per_iteration;
    r->rounds = rounds_for(r->N, p->max_pose_candidates_after_cull, p->max_relocalisations_to_output, &r->entering);
    r->TP = score_tile(r->T * r->M);
    r->L = (size_t)1 << r->D;
    r->max_w = max_width;
    r->max_h = max_height;
    r->maxP = max_width * max_height;
    r->G = grid_items(max_width, max_height);
    r->pers = reinterpret_cast<char*>(dev_persistent);
    r->scr = reinterpret_cast<char*>(dev_scratch);
    r->PL = persist_layout(*p);
    r->job_off = 0;
    r->rounds_cap = rounds_capacity(*p);
    r->FL = frame_layout(r->maxP, r->N, r->eta, r->rounds_cap, r->TP, r->T * r->M, align256(sizeof(Job)));
    r->AL = adapt_layout(*p, r->G, align256(sizeof(Job)) + r->FL.total);
    r->ML = model_layout(r->maxP, align256(sizeof(Job)) + r->FL.total + r->AL.total);
    r->stream = reinterpret_cast<hipStream_t>(hip_stream);
    r->trace = 0;
    r->modes_stale = false;
    r->rr_leaves = 0;
    r->rr_cursor = 0;
    r->mode_version = 0;
    hipError_t e = hipEventCreateWithFlags(&r->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->wev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r->bev, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipEvent_t ev : {r->ev, r->wev, r->bev})
            if (ev) (void)hipEventDestroy(ev);
        delete r;
        return hip_fail(e, "hipEventCreate");
    }
    r->wrote = false;
    e = hipHostMalloc(reinterpret_cast<void**>(&r->job_host), sizeof(Job), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&r->res_host), sizeof(rl_result), hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&r->model_host),
                          kModelHostBytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        for (void* hp : {(void*)r->job_host, (void*)r->res_host, (void*)r->model_host})
            if (hp) (void)hipHostFree(hp);
        for (hipEvent_t ev : {r->ev, r->wev, r->bev}) (void)hipEventDestroy(ev);
        delete r;
        return fail(RL_ENOMEM, "pinned host allocation failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(r->pers + r->PL.nodes, host_nodes, (size_t)r->T * NT * sizeof(rl_node),
                       hipMemcpyHostToDevice, r->stream);
    if (e != hipSuccess) {
        relocaliser_destroy(r);
        return hip_fail(e, "copy nodes");
    }
    const size_t TL = (size_t)r->T * r->L;
    rl_status fs = RL_OK;
    if (fs == RL_OK) fs = fill_u32(r->pers + r->PL.seen, TL, 0, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->pers + r->PL.dirty, TL, 0, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->pers + r->PL.counters, 64, 0, r->stream);
    if (fs == RL_OK) fs = fill_u8(r->pers + r->PL.nmodes, TL, 0, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->scr + r->AL.head, TL, kNone32, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->scr + r->AL.hkey, r->AL.hsize, kNone32, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->scr + r->AL.hval, r->AL.hsize, 0, r->stream);
    if (fs == RL_OK) fs = fill_u32(r->scr + r->FL.state, sizeof(JobState) / 4, 0, r->stream);
    if (fs != RL_OK) {
        relocaliser_destroy(r);
        return fs;
    }
    e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) {
        relocaliser_destroy(r);
        return hip_fail(e, "create");
    }
    *out = r;
    return RL_OK;
}

RL_API rl_status relocaliser_destroy(rl_room* r)
{
    if (!r) return RL_OK;
    for (auto& kv : r->graphs) (void)hipGraphExecDestroy(kv.second);
    if (r->job_host) (void)hipHostFree(r->job_host);
    if (r->res_host) (void)hipHostFree(r->res_host);
    if (r->model_host) (void)hipHostFree(r->model_host);
    for (hipEvent_t ev : {r->ev, r->wev, r->bev})
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : r->readers) {
        (void)hipEventSynchronize(ev);      // recorded on a batch stream that may still run
        (void)hipEventDestroy(ev);
    }
    for (hipEvent_t ev : r->spare) (void)hipEventDestroy(ev);
    delete r;
    return RL_OK;
}

// ------------------------------------------------------------------------
// random forest (host)

// Philox4x32-10 on the host (the device version is in rl_internal.hpp)
static void philox_host(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1, n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static float uniform_range(uint32_t u, float a, float b)
{
    const double x = ((double)u + 0.5) * (1.0 / 4294967296.0);
    return (float)((double)a + ((double)b - (double)a) * x);
}

RL_API rl_status rl_forest_generate(const rl_forest_params* fp, rl_node* nodes, size_t* bytes)
{
    if (!fp || !bytes) return fail(RL_EINVAL, "NULL argument");
    if (fp->n_trees < 1 || fp->n_trees > kMaxTrees) return fail(RL_EINVAL, "n_trees must be in 1..%d", kMaxTrees);
    if (fp->depth < 1 || fp->depth > 15) return fail(RL_EINVAL, "depth must be in 1..15");
    if (!(fp->p_depth >= 0.0f && fp->p_depth <= 1.0f)) return fail(RL_EINVAL, "p_depth must be in [0, 1]");
    if (!(fp->offset_range >= 0.0f) || !(fp->tau_depth >= 0.0f) || !(fp->tau_colour >= 0.0f) ||
        !finite_f(fp->offset_range) || !finite_f(fp->tau_depth) || !finite_f(fp->tau_colour))
        return fail(RL_EINVAL, "ranges must be finite and >= 0");
    const size_t NT = ((size_t)1 << fp->depth) - 1;
    *bytes = (size_t)fp->n_trees * NT * sizeof(rl_node);
    if (!nodes) return RL_OK;
    const uint32_t k0 = (uint32_t)fp->seed, k1 = (uint32_t)(fp->seed >> 32);
    for (int t = 0; t < fp->n_trees; ++t)
        for (size_t i = 0; i < NT; ++i) {
            uint32_t a[4], b[4];
            const uint32_t c0[4] = {(uint32_t)t, (uint32_t)i, 0u, 0u}, c1[4] = {(uint32_t)t, (uint32_t)i, 1u, 0u};
            philox_host(c0, k0, k1, a);
            philox_host(c1, k0, k1, b);
            rl_node& n = nodes[(size_t)t * NT + i];
            const bool depth = ((double)a[0] + 0.5) * (1.0 / 4294967296.0) < (double)fp->p_depth;
            const uint32_t chan = (uint32_t)(((uint64_t)a[1] * 3u) >> 32);
            n.kind = depth ? 0u : 1u + chan;
            n.dx = uniform_range(a[2], -fp->offset_range, fp->offset_range);
            n.dy = uniform_range(a[3], -fp->offset_range, fp->offset_range);
            n.tau = depth ? uniform_range(b[0], -fp->tau_depth, fp->tau_depth)
                          : uniform_range(b[0], -fp->tau_colour, fp->tau_colour);
        }
    return RL_OK;
}

// ------------------------------------------------------------------------
// room persistence

struct SaveHeader {
    char magic[8];            // "RLROOM01"
    int32_t n_trees, depth, max_cluster_count, reservoir_capacity;
    uint64_t bytes;           // persistent state that follows
    uint32_t rr_cursor;
    int32_t modes_stale;
};

static const size_t kStageBytes = (size_t)64 << 20;

RL_API rl_status relocaliser_save(rl_room* r, const char* path)
{
    if (!r || !path) return fail(RL_EINVAL, "NULL argument");
    SaveHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, "RLROOM01", 8);
    h.n_trees = r->p.n_trees;
    h.depth = r->p.depth;
    h.max_cluster_count = r->p.max_cluster_count;
    h.reservoir_capacity = r->p.reservoir_capacity;
    h.bytes = r->PL.total;
    h.rr_cursor = r->rr_cursor;
    h.modes_stale = r->modes_stale ? 1 : 0;
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(RL_EINVAL, "cannot open %s for writing", path);
    char* stage = nullptr;
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&stage), kStageBytes, hipHostMallocDefault);
    bool ok = e == hipSuccess && std::fwrite(&h, sizeof(h), 1, f) == 1;
    for (size_t off = 0; ok && off < h.bytes; off += kStageBytes) {
        const size_t n = std::min(kStageBytes, (size_t)h.bytes - off);
        e = hipMemcpyAsync(stage, r->pers + off, n, hipMemcpyDeviceToHost, r->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
        ok = e == hipSuccess && std::fwrite(stage, 1, n, f) == n;
    }
    if (stage) (void)hipHostFree(stage);
    ok = (std::fclose(f) == 0) && ok;
    if (e != hipSuccess) return hip_fail(e, "room save");
    if (!ok) return fail(RL_EINVAL, "writing %s failed", path);
    return RL_OK;
}

RL_API rl_status relocaliser_load(rl_room* r, const char* path)
{
    if (!r || !path) return fail(RL_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(RL_EINVAL, "cannot open %s", path);
    SaveHeader h;
    if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, "RLROOM01", 8) != 0) {
        std::fclose(f);
        return fail(RL_EINVAL, "%s is not a saved room", path);
    }
    if (h.n_trees != r->p.n_trees || h.depth != r->p.depth || h.max_cluster_count != r->p.max_cluster_count ||
        h.reservoir_capacity != r->p.reservoir_capacity || h.bytes != r->PL.total) {
        std::fclose(f);
        return fail(RL_EINVAL, "%s holds a room of another forest shape", path);
    }
    // the load writes everything batches read: after the batches that read the room
    hipError_t e = hipSuccess;
    for (hipEvent_t ev : r->readers) {
        if (e == hipSuccess) e = hipStreamWaitEvent(r->stream, ev, 0);
        r->spare.push_back(ev);
    }
    r->readers.clear();
    char* stage = nullptr;
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&stage), kStageBytes, hipHostMallocDefault);
    bool ok = e == hipSuccess;
    for (size_t off = 0; ok && off < h.bytes; off += kStageBytes) {
        const size_t n = std::min(kStageBytes, (size_t)h.bytes - off);
        ok = std::fread(stage, 1, n, f) == n;
        if (ok) e = hipMemcpyAsync(r->pers + off, stage, n, hipMemcpyHostToDevice, r->stream);
        if (ok && e == hipSuccess) e = hipStreamSynchronize(r->stream);
        ok = ok && e == hipSuccess;
    }
    std::fclose(f);
    if (stage) (void)hipHostFree(stage);
    if (e == hipSuccess) e = hipEventRecord(r->wev, r->stream);
    if (e != hipSuccess) return hip_fail(e, "room load");
    r->wrote = true;      // also after a truncated file: later readers wait for what was copied
    if (!ok) return fail(RL_EINVAL, "%s is truncated (the room's state is partly overwritten)", path);
    r->rr_cursor = h.rr_cursor;
    r->modes_stale = h.modes_stale != 0;
    return RL_OK;
}

RL_API rl_status relocaliser_set_trace(rl_room* r, int32_t on)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    r->trace = on ? 1 : 0;
    return RL_OK;
}

static rl_status check_pose(const float* H)
{
    if (!H) return fail(RL_EINVAL, "pose is NULL");
    for (int i = 0; i < 16; ++i)
        if (!finite_f(H[i])) return fail(RL_EINVAL, "pose has a non-finite entry");
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double dot = 0;
            for (int k = 0; k < 3; ++k) dot += (double)H[4 * k + i] * H[4 * k + j];
            if (std::fabs(dot - (i == j ? 1.0 : 0.0)) > 1e-3) return fail(RL_EINVAL, "pose is not rigid");
        }
    if (std::fabs(H[12]) > 1e-6f || std::fabs(H[13]) > 1e-6f || std::fabs(H[14]) > 1e-6f || std::fabs(H[15] - 1.0f) > 1e-6f)
        return fail(RL_EINVAL, "pose last row must be 0 0 0 1");
    return RL_OK;
}

// Arguments of one adaptation of room r by frame f at pose H (validated).
static AdaptArgs adapt_args(const rl_room* r, const rl_frame* f, const float H[16])
{
    AdaptArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nodes = reinterpret_cast<const float4*>(r->pers + r->PL.nodes);
    a.T = r->T;
    a.D = r->D;
    a.L = (int)r->L;
    a.kappa = r->kappa;
    a.src = frame_view(f);
    a.w = f->width;
    a.h = f->height;
    a.gw = f->width / 4 - 1;
    a.G = grid_items(f->width, f->height);
    a.fx = f->K.fx;
    a.fy = f->K.fy;
    a.cx = f->K.cx;
    a.cy = f->K.cy;
    a.s = (float)f->width / (float)r->p.ref_width;
    for (int i = 0; i < 12; ++i) a.H[i] = (double)H[i];
    const uint64_t k = stream_key64(r->p.seed, 0);
    a.key0 = (uint32_t)k;
    a.key1 = (uint32_t)(k >> 32);
    a.reservoir = reinterpret_cast<float4*>(r->pers + r->PL.reservoir);
    a.seen = reinterpret_cast<uint32_t*>(r->pers + r->PL.seen);
    a.dirty = reinterpret_cast<uint32_t*>(r->pers + r->PL.dirty);
    a.dirty_list = reinterpret_cast<uint32_t*>(r->pers + r->PL.dirty_list);
    a.counters = reinterpret_cast<uint32_t*>(r->pers + r->PL.counters);
    char* sc = r->scr;
    const AdaptLayout& A = r->AL;
    a.item_leaf = reinterpret_cast<uint16_t*>(sc + A.item_leaf);
    a.item_pt = reinterpret_cast<float4*>(sc + A.item_pt);
    a.item_run = reinterpret_cast<uint32_t*>(sc + A.item_run);
    a.item_lrank = reinterpret_cast<uint16_t*>(sc + A.item_lrank);
    a.item_n = reinterpret_cast<uint32_t*>(sc + A.item_n);
    a.item_slot = reinterpret_cast<int*>(sc + A.item_slot);
    a.item_h = reinterpret_cast<uint32_t*>(sc + A.item_h);
    a.run_cnt = reinterpret_cast<uint32_t*>(sc + A.run_cnt);
    a.run_tl = reinterpret_cast<uint32_t*>(sc + A.run_tl);
    a.run_next = reinterpret_cast<uint32_t*>(sc + A.run_next);
    a.run_pre = reinterpret_cast<uint32_t*>(sc + A.run_pre);
    a.run_tot = reinterpret_cast<uint32_t*>(sc + A.run_tot);
    a.head = reinterpret_cast<uint32_t*>(sc + A.head);
    a.hkey = reinterpret_cast<uint32_t*>(sc + A.hkey);
    a.hval = reinterpret_cast<uint32_t*>(sc + A.hval);
    a.Gp = (a.G + kAdaptChunk - 1) / kAdaptChunk * kAdaptChunk;
    a.hmask = A.hsize - 1;
    a.result = nullptr;
    return a;
}

static rl_status round_robin_step(rl_room* r, hipStream_t st);

RL_API rl_status relocaliser_adapt(rl_room* r, const rl_frame* f, const float H[16], int32_t reliable)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    rl_status s = validate_frame(f, r->max_w, r->max_h);
    if (s != RL_OK) return s;
    s = check_pose(H);
    if (s != RL_OK) return s;
    if (!reliable) return RL_OK;
    const hipError_t e = launch_adapt(adapt_args(r, f, H), r->stream);
    if (e != hipSuccess) return hip_fail(e, "adapt launch");
    r->modes_stale = true;
    return r->rr_leaves ? round_robin_step(r, r->stream) : RL_OK;
}

static rl_status write_modes(rl_room* r, const RqsArgs& a, hipStream_t st)
{
    hipError_t e = hipSuccess;
    for (hipEvent_t ev : r->readers) {
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
        r->spare.push_back(ev);
    }
    r->readers.clear();
    if (e == hipSuccess) e = launch_rqs(a, 1024, st);
    if (e == hipSuccess) e = hipEventRecord(r->wev, st);
    ++r->mode_version;
    if (e != hipSuccess) return hip_fail(e, "mode update launch");
    r->wrote = true;
    return RL_OK;
}

// exact update: every leaf adapted since the last one
static rl_status update_dirty_modes(rl_room* r)
{
    if (!r->modes_stale) return RL_OK;
    const rl_status s = write_modes(r, rqs_args(r), r->stream);
    if (s == RL_OK) r->modes_stale = false;
    return s;
}

// Before a relocalisation: the exact schedule brings every adapted leaf up
// to date; the round-robin schedule uses the modes as they are.
static rl_status ensure_modes(rl_room* r)
{
    return r->rr_leaves ? RL_OK : update_dirty_modes(r);
}

// Round-robin schedule (Sec. 3.2.2): after each adapted frame, the next K
// leaves of the forest in index order, wrapping around.
static rl_status round_robin_step(rl_room* r, hipStream_t st)
{
    RqsArgs a = rqs_args(r);
    a.rr_first = r->rr_cursor;
    a.rr_count = (uint32_t)r->rr_leaves;
    const rl_status s = write_modes(r, a, st);
    if (s == RL_OK) r->rr_cursor = (uint32_t)((r->rr_cursor + (uint64_t)r->rr_leaves) % a.n_leaves);
    return s;
}

// A batch on stream st is about to read the room: order it after the last
// mode update.
static rl_status room_read_begin(rl_room* r, hipStream_t st)
{
    rl_status s = ensure_modes(r);
    if (s != RL_OK) return s;
    if (r->wrote && st != r->stream) {
        const hipError_t e = hipStreamWaitEvent(st, r->wev, 0);
        if (e != hipSuccess) return hip_fail(e, "batch ordering");
    }
    return RL_OK;
}

// ... and has been queued: remember it as a reader of the current modes.
static rl_status room_read_end(rl_room* r, hipStream_t st)
{
    if (st == r->stream) return RL_OK;
    hipEvent_t ev = nullptr;
    hipError_t e = hipSuccess;
    if (!r->spare.empty()) {
        ev = r->spare.back();
        r->spare.pop_back();
    } else {
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventRecord(ev, st);
    if (e != hipSuccess) {
        if (ev) (void)hipEventDestroy(ev);
        return hip_fail(e, "batch ordering");
    }
    r->readers.push_back(ev);
    return RL_OK;
}

RL_API rl_status relocaliser_update_modes(rl_room* r)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    return update_dirty_modes(r);
}

RL_API rl_status relocaliser_set_mode_schedule(rl_room* r, int32_t leaves_per_frame)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    const long long TL = (long long)r->T * (long long)r->L;
    if (leaves_per_frame < 0 || leaves_per_frame > TL)
        return fail(RL_EINVAL, "leaves_per_frame must be in 0..%lld", TL);
    r->rr_leaves = leaves_per_frame;
    return RL_OK;
}

static rl_status check_schedule(int ipt, int fast_waves, int lds_levels, int score_window)
{
    if (score_window < 0 || score_window > 3) return fail(RL_EINVAL, "score_window must be in 0..3");
    if (ipt != 2 && ipt != 4 && ipt != 8) return fail(RL_EINVAL, "iterations per thread must be 2, 4 or 8");
    if (fast_waves != 1 && fast_waves != 2 && fast_waves != 4) return fail(RL_EINVAL, "fast_waves must be 1, 2 or 4");
    if (lds_levels != kTopLevelsMin && lds_levels != kTopLevelsMax)
        return fail(RL_EINVAL, "lds_levels must be %d or %d", kTopLevelsMin, kTopLevelsMax);
    return RL_OK;
}

RL_API rl_status relocaliser_set_schedule(rl_room* r, int32_t ipt, int32_t fast_waves, int32_t lds_levels,
                                         int32_t score_window)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    rl_status s = check_schedule(ipt, fast_waves, lds_levels, score_window);
    if (s != RL_OK) return s;
    r->sched.ipt = ipt;
    r->sched.fw = fast_waves;
    r->sched.top = lds_levels;
    r->sched.win = score_window;
    return RL_OK;
}

RL_API rl_status rl_batch_set_schedule(rl_batch* b, int32_t ipt, int32_t fast_waves, int32_t lds_levels,
                                       int32_t score_window)
{
    if (!b) return fail(RL_EINVAL, "batch is NULL");
    rl_status s = check_schedule(ipt, fast_waves, lds_levels, score_window);
    if (s != RL_OK) return s;
    b->sched.ipt = ipt;
    b->sched.fw = fast_waves;
    b->sched.top = lds_levels;
    b->sched.win = score_window;
    return RL_OK;
}

RL_API rl_status relocaliser_set_degeneracy_screen(rl_room* r, int32_t on)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    r->sched.screen = on ? 1 : 0;
    return RL_OK;
}

RL_API rl_status rl_batch_set_degeneracy_screen(rl_batch* b, int32_t on)
{
    if (!b) return fail(RL_EINVAL, "batch is NULL");
    b->sched.screen = on ? 1 : 0;
    return RL_OK;
}

static hipError_t launch_sequence(const Job* jobs, int njobs, int maxP, int maxN, int maxIters, int T,
                                  const std::vector<int>& entering, int nptiles, int maxEta, int maxRows, bool any_lm,
                                  int lm_iters, bool lm_split, const Schedule& sc, const Timer& tm, hipStream_t st)
{
    hipError_t e;
#define RL_TRY(x) do { e = (x); if (e != hipSuccess) return e; } while (0)
#define RL_MARK(k, ev) do { if (tm.kernel == (k)) RL_TRY(hipEventRecord(tm.ev, st)); } while (0)
    RL_TRY(launch_prep(jobs, njobs, maxN, st));
    RL_MARK(RL_TIMER_TRAVERSE, start);
    RL_TRY(launch_traverse(jobs, njobs, maxP, T, sc.top, st));
    RL_MARK(RL_TIMER_TRAVERSE, stop);
    RL_TRY(launch_eligible(jobs, njobs, maxP, T, st));
    RL_MARK(RL_TIMER_HYP_SEARCH, start);
    RL_TRY(launch_hyp_search(jobs, njobs, maxN, maxIters, sc.ipt, st));
    RL_MARK(RL_TIMER_HYP_SEARCH, stop);
    RL_TRY(launch_hyp_finalize(jobs, njobs, maxN, st));
    RL_MARK(RL_TIMER_RANSAC, start);
    // rounds with more than 64 * fw survivors one at a time, the rest at once;
    // with LM refinement (which re-scores every round after the first) all
    // rounds one at a time
    for (int r = 0; r < (int)entering.size() && (any_lm || entering[r] > 64 * sc.fw); ++r) {
        RL_TRY(launch_score(jobs, njobs, r, nptiles, entering[r], st));
        if (any_lm && r > 0) RL_TRY(launch_lm(jobs, njobs, r, entering[r], maxEta, maxRows, lm_iters, lm_split, st));
        RL_TRY(launch_select(jobs, njobs, r, nptiles, maxN, st));
    }
    RL_TRY(launch_score_all(jobs, njobs, (int)entering.size(), nptiles, sc.fw, sc.win, st));
    RL_MARK(RL_TIMER_RANSAC, stop);
    RL_TRY(launch_finalize(jobs, njobs, (int)entering.size() * maxEta, st));
#undef RL_MARK
#undef RL_TRY
    return hipSuccess;
}

// Replays the launch sequence from a graph cached under `key` (captured on
// first use).  Streams that cannot be captured (the legacy default stream)
// and active kernel timers use direct launches.
template <class F>
static hipError_t run_sequence(std::map<std::vector<long long>, hipGraphExec_t>& cache,
                               const std::vector<long long>& key, bool graph_ok, hipStream_t st, F&& launch)
{
    if (!graph_ok || st == nullptr) return launch();
    auto it = cache.find(key);
    if (it == cache.end()) {
        hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipError_t le = launch();
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(st, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return le != hipSuccess ? le : e;
        }
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return e;
        it = cache.emplace(key, ex).first;
    }
    return hipGraphLaunch(it->second, st);
}

RL_API rl_status relocaliser_relocalise_opts(rl_room* r, const rl_frame* f, uint64_t request_seed,
                                             const rl_reloc_opts* opts, rl_result* out)
{
    if (!r || !out) return fail(RL_EINVAL, "NULL argument");
    rl_status s = validate_frame(f, r->max_w, r->max_h);
    if (s != RL_OK) return s;
    const int N = opts && opts->n_hypotheses > 0 ? opts->n_hypotheses : r->N;
    const int n_cull = opts && opts->n_cull > 0 ? opts->n_cull : r->p.max_pose_candidates_after_cull;
    const int n_out = opts && opts->n_out > 0 ? opts->n_out : r->p.max_relocalisations_to_output;
    const int refine = opts && opts->final_refine >= 0 ? (opts->final_refine ? 1 : 0) : r->p.final_refine;
    const int lm = opts && opts->pose_update >= 0 ? (opts->pose_update ? 1 : 0) : r->p.pose_update;
    const int iters = opts && opts->max_iterations > 0 ? opts->max_iterations : r->p.max_candidate_generation_iterations;
    const int eta = opts && opts->eta > 0 ? opts->eta : r->eta;
    const int cov = opts && opts->use_covariance >= 0 ? (opts->use_covariance ? 1 : 0) : r->p.use_prediction_covariance;
    if (opts && (!finite_f(opts->min_squared_distance) || !finite_f(opts->max_translation_error)))
        return fail(RL_EINVAL, "non-finite per-call threshold");
    const double min_sq = opts && opts->min_squared_distance >= 0.0f ? opts->min_squared_distance
                                                                     : r->p.min_squared_distance_between_sampled_modes;
    const double rig = opts && opts->max_translation_error >= 0.0f ? opts->max_translation_error
                                                                   : r->p.max_translation_error_for_correct_pose;
    if (eta > r->eta) return fail(RL_EINVAL, "eta %d exceeds the room's %d", eta, r->eta);
    if (iters >= (1 << 30)) return fail(RL_EINVAL, "max_iterations must be below 2^30");
    if (N > r->N) return fail(RL_EINVAL, "%d hypotheses exceed the room's maximum %d", N, r->N);
    std::vector<int> entering;
    const int R = rounds_for(N, n_cull, n_out, &entering);
    if (R > r->rounds_cap) return fail(RL_EINVAL, "%d rounds exceed the room's capacity %d", R, r->rounds_cap);
    s = ensure_modes(r);
    if (s != RL_OK) return s;
    Job J = make_job(r, r->scr, r->FL, f, request_seed, N);
    J.n_cull = n_cull;
    J.n_out = n_out;
    J.final_refine = refine;
    J.lm = lm;
    J.I_max = iters;
    J.eta = eta;
    J.use_cov = cov;
    J.min_sq_dist = min_sq;
    J.theta_rig = rig;
    *r->job_host = J;
    Job* jd = reinterpret_cast<Job*>(r->scr + r->job_off);
    hipError_t e = hipMemcpyAsync(jd, r->job_host, sizeof(Job), hipMemcpyHostToDevice, r->stream);
    if (e != hipSuccess) return hip_fail(e, "job upload");
    const int nptiles = (eta + r->TP - 1) / r->TP;
    const int P = f->width * f->height;
    std::vector<long long> key = {P, N, r->sched.ipt, r->sched.fw, r->sched.top, r->sched.win, lm, r->p.lm_iterations, iters, eta};
    for (int v : entering) key.push_back(v);
    e = run_sequence(r->graphs, key, r->timer.kernel == RL_TIMER_NONE, r->stream, [&]() {
        return launch_sequence(jd, 1, P, N, iters, r->T, entering, nptiles, eta, r->T * r->M, lm != 0,
                               r->p.lm_iterations, J.lm_split != 0, r->sched, r->timer, r->stream);
    });
    if (e != hipSuccess) return hip_fail(e, "relocalise launch");
    e = hipMemcpyAsync(r->res_host, r->scr + r->FL.result, sizeof(rl_result), hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "relocalise");
    *out = *r->res_host;
    return out->status == RL_OK ? RL_OK : RL_NO_POSE;
}

RL_API rl_status relocaliser_relocalise_ex(rl_room* r, const rl_frame* f, uint64_t request_seed, rl_result* out)
{
    return relocaliser_relocalise_opts(r, f, request_seed, nullptr, out);
}

RL_API rl_status rl_plane_scores(rl_room* r, const rl_frame* f, const rl_surface* surfaces, int32_t n_surf,
                                 const float* poses, int32_t n_poses, double* scores)
{
    if (!r || !surfaces || !poses || !scores) return fail(RL_EINVAL, "NULL argument");
    rl_status s = validate_frame(f, r->max_w, r->max_h);
    if (s != RL_OK) return s;
    if (n_surf < 1 || n_surf > kMaxModelSurfaces) return fail(RL_EINVAL, "n_surfaces must be in 1..%d", kMaxModelSurfaces);
    if (n_poses < 1 || n_poses > kMaxModelPoses) return fail(RL_EINVAL, "n_poses must be in 1..%d", kMaxModelPoses);
    for (int i = 0; i < n_surf * 16; ++i)
        if (!finite_f(reinterpret_cast<const float*>(surfaces)[i])) return fail(RL_EINVAL, "non-finite surface");
    for (int i = 0; i < n_poses * 12; ++i)
        if (!finite_f(poses[i])) return fail(RL_EINVAL, "non-finite pose");
    char* hs = r->model_host;
    std::memcpy(hs, surfaces, (size_t)n_surf * 64);
    std::memcpy(hs + kMaxModelSurfaces * 64, poses, (size_t)n_poses * 48);
    hipError_t e = hipMemcpyAsync(r->scr + r->ML.surfaces, hs, (size_t)n_surf * 64, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->scr + r->ML.poses, hs + kMaxModelSurfaces * 64, (size_t)n_poses * 48,
                           hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess)
        e = launch_plane_scores(frame_view(f), f->width, f->height, f->K.fx, f->K.fy, f->K.cx, f->K.cy,
                                reinterpret_cast<const float*>(r->scr + r->ML.surfaces), n_surf,
                                reinterpret_cast<const float*>(r->scr + r->ML.poses), n_poses,
                                reinterpret_cast<double*>(r->scr + r->ML.partial),
                                reinterpret_cast<int*>(r->scr + r->ML.cnt),
                                reinterpret_cast<double*>(r->scr + r->ML.scores), r->stream);
    double* hscores = reinterpret_cast<double*>(hs + kMaxModelSurfaces * 64 + kMaxModelPoses * 48);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hscores, r->scr + r->ML.scores, (size_t)n_poses * 8, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "plane scores");
    std::memcpy(scores, hscores, (size_t)n_poses * 8);
    return RL_OK;
}

RL_API rl_status rl_depth_scores(rl_room* r, const rl_frame* f, const rl_surface* surfaces, int32_t n_surf,
                                 const float* poses, int32_t n_poses, float min_depth, float max_depth,
                                 double* scores, double* mu, int64_t* counts)
{
    if (!r || !surfaces || !poses || !scores) return fail(RL_EINVAL, "NULL argument");
    rl_status s = validate_frame(f, r->max_w, r->max_h);
    if (s != RL_OK) return s;
    if (n_surf < 1 || n_surf > kMaxModelSurfaces) return fail(RL_EINVAL, "n_surfaces must be in 1..%d", kMaxModelSurfaces);
    if (n_poses < 1 || n_poses > kMaxModelPoses) return fail(RL_EINVAL, "n_poses must be in 1..%d", kMaxModelPoses);
    if (!finite_f(min_depth) || !finite_f(max_depth) || min_depth < 0.0f)
        return fail(RL_EINVAL, "min_depth must be finite and >= 0, max_depth finite");
    for (int i = 0; i < n_surf * 16; ++i)
        if (!finite_f(reinterpret_cast<const float*>(surfaces)[i])) return fail(RL_EINVAL, "non-finite surface");
    for (int i = 0; i < n_poses * 12; ++i)
        if (!finite_f(poses[i])) return fail(RL_EINVAL, "non-finite pose");
    char* hs = r->model_host;
    char* hp = hs + kMaxModelSurfaces * 64;
    char* hout = hp + kMaxModelPoses * (48 + 8);
    char* hcnt = hout + kMaxModelPoses * 16;
    std::memcpy(hs, surfaces, (size_t)n_surf * 64);
    std::memcpy(hp, poses, (size_t)n_poses * 48);
    hipError_t e = hipMemcpyAsync(r->scr + r->ML.surfaces, hs, (size_t)n_surf * 64, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->scr + r->ML.poses, hp, (size_t)n_poses * 48, hipMemcpyHostToDevice, r->stream);
    if (e == hipSuccess)
        e = launch_depth_scores(frame_view(f), f->width, f->height, f->K.fx, f->K.fy, f->K.cx, f->K.cy,
                                reinterpret_cast<const float*>(r->scr + r->ML.surfaces), n_surf,
                                reinterpret_cast<const float*>(r->scr + r->ML.poses), n_poses, min_depth, max_depth,
                                reinterpret_cast<double*>(r->scr + r->ML.dpartial),
                                reinterpret_cast<int*>(r->scr + r->ML.dcnt),
                                reinterpret_cast<double*>(r->scr + r->ML.dout),
                                reinterpret_cast<long long*>(r->scr + r->ML.dcounts), r->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hout, r->scr + r->ML.dout, (size_t)n_poses * 16, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hcnt, r->scr + r->ML.dcounts, (size_t)n_poses * 16, hipMemcpyDeviceToHost, r->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(r->stream);
    if (e != hipSuccess) return hip_fail(e, "depth scores");
    const double* o = reinterpret_cast<const double*>(hout);
    const long long* c = reinterpret_cast<const long long*>(hcnt);
    for (int k = 0; k < n_poses; ++k) {
        scores[k] = o[2 * k];
        if (mu) mu[k] = o[2 * k + 1];
        if (counts) {
            counts[2 * k] = c[2 * k];
            counts[2 * k + 1] = c[2 * k + 1];
        }
    }
    return RL_OK;
}

// ------------------------------------------------------------------------
// Depth-raycast scores without caller work space (for callers that cannot
// allocate): the surfaces, poses, per-tile partial sums and counts and the
// outputs live in one fixed device array of this library, whose address on
// each device is looked up once, with that device current.

namespace {

constexpr size_t align256c(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr int kStaticScoreMaxPixels = 1 << 21;     // 2048 tiles of 1024 pixels
constexpr size_t kStaticScoreTiles = ((size_t)kStaticScoreMaxPixels + 1023) / 1024;
constexpr size_t kSsSurfaces = 0;
constexpr size_t kSsPoses = align256c(kSsSurfaces + (size_t)kMaxModelSurfaces * 64);
constexpr size_t kSsPartial = align256c(kSsPoses + (size_t)kMaxModelPoses * 48);
constexpr size_t kSsCnt = align256c(kSsPartial + kStaticScoreTiles * kMaxModelPoses * 8);
constexpr size_t kSsOut = align256c(kSsCnt + kStaticScoreTiles * kMaxModelPoses * 2 * 4);
constexpr size_t kSsCounts = align256c(kSsOut + (size_t)kMaxModelPoses * 2 * 8);
constexpr size_t kStaticScoreBytes = align256c(kSsCounts + (size_t)kMaxModelPoses * 2 * 8);
constexpr int kStaticScoreDevices = 64;

// Host code never passes this name to a kernel or a copy: the address it
// stands for on a device comes from hipGetSymbolAddress (g_score_scratch_ptr).
static __device__ __align__(256) unsigned char score_scratch[kStaticScoreBytes];

std::mutex g_score_scratch_mu[kStaticScoreDevices];
std::mutex g_score_scratch_init_mu;
void* g_score_scratch_ptr[kStaticScoreDevices] = {};

// The current device's copy of score_scratch (looked up on its first use).
rl_status score_scratch_address(int* dev_out, char** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kStaticScoreDevices)
        return fail(RL_EDEVICE, "device %d is beyond the %d devices the fixed work space supports", dev,
                    kStaticScoreDevices);
    std::lock_guard<std::mutex> lk(g_score_scratch_init_mu);
    if (!g_score_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(score_scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "work space lookup");
        g_score_scratch_ptr[dev] = p;
    }
    *dev_out = dev;
    *out = static_cast<char*>(g_score_scratch_ptr[dev]);
    return RL_OK;
}

}  // namespace

RL_API rl_status rl_depth_scores_noalloc(const rl_frame* f, const rl_surface* surfaces, int32_t n_surf,
                                         const float* poses, int32_t n_poses, float min_depth, float max_depth,
                                         void* hip_stream, double* scores, double* mu, int64_t* counts)
{
    if (!f || !surfaces || !poses || !scores) return fail(RL_EINVAL, "NULL argument");
    if ((long long)f->width * f->height > kStaticScoreMaxPixels)
        return fail(RL_EINVAL, "frame %dx%d exceeds the %d pixels of the fixed work space", f->width, f->height,
                    kStaticScoreMaxPixels);
    rl_status s = validate_frame(f, 1 << 30, 1 << 30);
    if (s != RL_OK) return s;
    if (n_surf < 1 || n_surf > kMaxModelSurfaces) return fail(RL_EINVAL, "n_surfaces must be in 1..%d", kMaxModelSurfaces);
    if (n_poses < 1 || n_poses > kMaxModelPoses) return fail(RL_EINVAL, "n_poses must be in 1..%d", kMaxModelPoses);
    if (!finite_f(min_depth) || !finite_f(max_depth) || min_depth < 0.0f)
        return fail(RL_EINVAL, "min_depth must be finite and >= 0, max_depth finite");
    for (int i = 0; i < n_surf * 16; ++i)
        if (!finite_f(reinterpret_cast<const float*>(surfaces)[i])) return fail(RL_EINVAL, "non-finite surface");
    for (int i = 0; i < n_poses * 12; ++i)
        if (!finite_f(poses[i])) return fail(RL_EINVAL, "non-finite pose");
    int dev = 0;
    char* ws = nullptr;
    s = score_scratch_address(&dev, &ws);
    if (s != RL_OK) return s;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double hout[kMaxModelPoses * 2];
    long long hcnt[kMaxModelPoses * 2];
    // one call at a time per device: the work space is shared by every call
    std::lock_guard<std::mutex> lk(g_score_scratch_mu[dev]);
    hipError_t e = hipMemcpyAsync(ws + kSsSurfaces, surfaces, (size_t)n_surf * 64, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + kSsPoses, poses, (size_t)n_poses * 48, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_depth_scores(frame_view(f), f->width, f->height, f->K.fx, f->K.fy, f->K.cx, f->K.cy,
                                reinterpret_cast<const float*>(ws + kSsSurfaces), n_surf,
                                reinterpret_cast<const float*>(ws + kSsPoses), n_poses, min_depth, max_depth,
                                reinterpret_cast<double*>(ws + kSsPartial), reinterpret_cast<int*>(ws + kSsCnt),
                                reinterpret_cast<double*>(ws + kSsOut), reinterpret_cast<long long*>(ws + kSsCounts),
                                st);
    if (e == hipSuccess) e = hipMemcpyAsync(hout, ws + kSsOut, (size_t)n_poses * 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hcnt, ws + kSsCounts, (size_t)n_poses * 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "depth scores (fixed work space)");
    for (int k = 0; k < n_poses; ++k) {
        scores[k] = hout[2 * k];
        if (mu) mu[k] = hout[2 * k + 1];
        if (counts) {
            counts[2 * k] = hcnt[2 * k];
            counts[2 * k + 1] = hcnt[2 * k + 1];
        }
    }
    return RL_OK;
}

RL_API rl_status relocaliser_relocalise(rl_room* r, const rl_frame* f, uint64_t request_seed, float H[16],
                                        float* energy, float* mean_energy)
{
    rl_result res;
    const rl_status s = relocaliser_relocalise_ex(r, f, request_seed, &res);
    if (s < 0) return s;
    if (H) std::memcpy(H, res.cam_to_world, sizeof(float) * 16);
    if (energy) *energy = res.energy;
    if (mean_energy) *mean_energy = res.mean_energy;
    return s;
}

RL_API rl_status relocaliser_buffer(const rl_room* r, int32_t which, size_t* offset, size_t* bytes, int32_t* region)
{
    if (!r || !offset || !bytes || !region) return fail(RL_EINVAL, "NULL argument");
    const size_t TL = (size_t)r->T * r->L;
    switch (which) {
        case RL_BUF_NODES: *offset = r->PL.nodes; *bytes = TL / r->L * (r->L - 1) * 16; *region = 0; break;
        case RL_BUF_RESERVOIR: *offset = r->PL.reservoir; *bytes = TL * r->kappa * 16; *region = 0; break;
        case RL_BUF_SEEN: *offset = r->PL.seen; *bytes = TL * 4; *region = 0; break;
        case RL_BUF_MODES: *offset = r->PL.modes; *bytes = TL * r->M * 64; *region = 0; break;
        case RL_BUF_NMODES: *offset = r->PL.nmodes; *bytes = TL; *region = 0; break;
        case RL_BUF_DIRTY: *offset = r->PL.dirty; *bytes = TL * 4; *region = 0; break;
        case RL_BUF_LEAVES: *offset = r->FL.leaves; *bytes = (size_t)r->maxP * 16; *region = 1; break;
        case RL_BUF_NM: *offset = r->FL.nm; *bytes = (size_t)r->maxP; *region = 1; break;
        case RL_BUF_ELIGIBLE: *offset = r->FL.eligible; *bytes = (size_t)r->maxP * 4; *region = 1; break;
        case RL_BUF_HYPS: *offset = r->FL.hyps; *bytes = (size_t)r->N * sizeof(Hyp); *region = 1; break;
        case RL_BUF_ILIST: *offset = r->FL.I; *bytes = (size_t)r->rounds_cap * r->eta * 4; *region = 1; break;
        case RL_BUF_TRACE_SLOTS: *offset = r->FL.trace_slots; *bytes = (size_t)r->rounds_cap * r->N * 4; *region = 1; break;
        case RL_BUF_TRACE_ENERGY: *offset = r->FL.trace_E; *bytes = (size_t)r->rounds_cap * r->N * 8; *region = 1; break;
        case RL_BUF_SURVIVORS: *offset = r->FL.surv; *bytes = (size_t)r->N * 4; *region = 1; break;
        case RL_BUF_ENERGY: *offset = r->FL.E; *bytes = (size_t)r->N * 8; *region = 1; break;
        case RL_BUF_CBOX: *offset = r->PL.cbox; *bytes = TL * r->M * 8; *region = 0; break;
        case RL_BUF_EREC: *offset = r->FL.erec; *bytes = (size_t)r->maxP * r->FL.ew * 8; *region = 1; break;
        case RL_BUF_POSE64: *offset = r->FL.pose64; *bytes = (size_t)r->N * 96; *region = 1; break;
        default: return fail(RL_EINVAL, "unknown buffer %d", which);
    }
    return RL_OK;
}

// ------------------------------------------------------------------------
// batches

static int batch_rounds(const rl_batch_params& bp) { return bp.max_rounds; }

RL_API rl_status rl_batch_workspace_bytes(const rl_batch_params* bp, size_t* bytes)
{
    if (!bp || !bytes) return fail(RL_EINVAL, "NULL argument");
    if (bp->max_frames < 1 || bp->max_frames > kMaxBatchFrames) return fail(RL_EINVAL, "max_frames must be in 1..%d", kMaxBatchFrames);
    if (bp->max_width < 8 || bp->max_height < 8 || bp->max_width % 4 || bp->max_height % 4)
        return fail(RL_EINVAL, "max frame size must be multiples of 4, at least 8x8");
    if ((long long)bp->max_width * bp->max_height >= kMaxPixels) return fail(RL_EINVAL, "max frame must have fewer than 2^24 pixels");
    if (bp->max_hypotheses < 1 || bp->max_hypotheses > 4096) return fail(RL_EINVAL, "max_hypotheses must be in 1..4096");
    if (bp->max_eta < 1 || bp->max_eta > 4096) return fail(RL_EINVAL, "max_eta must be in 1..4096");
    if (bp->max_rounds < 1 || bp->max_rounds > 64) return fail(RL_EINVAL, "max_rounds must be in 1..64");
    if (bp->n_trees < 1 || bp->n_trees > kMaxTrees) return fail(RL_EINVAL, "n_trees must be in 1..8");
    if (bp->max_modes_per_pixel < 1 || bp->max_modes_per_pixel > 255) return fail(RL_EINVAL, "max_modes_per_pixel must be in 1..255");
    const int TP = score_tile(bp->max_modes_per_pixel);
    Carver c;
    c.take((size_t)bp->max_frames * sizeof(Job));
    c.take((size_t)bp->max_frames * sizeof(rl_result));
    c.take((size_t)bp->max_frames * sizeof(AdaptArgs));
    c.take((size_t)bp->max_frames * sizeof(RqsArgs));
    const FrameLayout FL = frame_layout(bp->max_width * bp->max_height, bp->max_hypotheses, bp->max_eta,
                                        batch_rounds(*bp), TP, bp->max_modes_per_pixel, 0);
    *bytes = c.cur + (size_t)bp->max_frames * align256(FL.total);
    return RL_OK;
}

RL_API rl_status rl_batch_create(const rl_batch_params* bp, void* ws, void* hip_stream, rl_batch** out)
{
    if (!out) return fail(RL_EINVAL, "out is NULL");
    *out = nullptr;
    size_t bytes = 0;
    rl_status s = rl_batch_workspace_bytes(bp, &bytes);
    if (s != RL_OK) return s;
    if (!ws || ((uintptr_t)ws & 255)) return fail(RL_EINVAL, "workspace must be a 256-byte aligned device buffer");
    rl_batch* b = new rl_batch();
    b->bp = *bp;
    b->ws = reinterpret_cast<char*>(ws);
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->TP = score_tile(bp->max_modes_per_pixel);
    b->rows = bp->max_modes_per_pixel;
    // many frames per launch: scoring the first two all-rounds rounds apart
    // from the rest saves more waves than its extra launches cost
    b->sched.win = 2;
    Carver c;
    b->jobs_off = c.take((size_t)bp->max_frames * sizeof(Job));
    b->results_off = c.take((size_t)bp->max_frames * sizeof(rl_result));
    b->ad_off = c.take((size_t)bp->max_frames * sizeof(AdaptArgs));
    b->rq_off = c.take((size_t)bp->max_frames * sizeof(RqsArgs));
    const FrameLayout proto = frame_layout(bp->max_width * bp->max_height, bp->max_hypotheses, bp->max_eta,
                                           batch_rounds(*bp), b->TP, bp->max_modes_per_pixel, 0);
    for (int i = 0; i < bp->max_frames; ++i) {
        const size_t base = c.take(proto.total);
        b->slots.push_back(frame_layout(bp->max_width * bp->max_height, bp->max_hypotheses, bp->max_eta,
                                        batch_rounds(*bp), b->TP, bp->max_modes_per_pixel, base));
    }
    b->ring = 0;
    b->ad_slot = 0;
    for (int k = 0; k < kJobRing; ++k) {
        b->job_ring[k] = nullptr;
        b->up_ev[k] = nullptr;
        b->ad_ring[k] = nullptr;
        b->ad_ev[k] = nullptr;
    }
    hipError_t e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->mark, hipEventDisableTiming);
    for (int k = 0; k < kJobRing && e == hipSuccess; ++k) {
        e = hipEventCreateWithFlags(&b->up_ev[k], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&b->job_ring[k]), (size_t)bp->max_frames * sizeof(Job),
                              hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ad_ev[k], hipEventDisableTiming);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void**>(&b->ad_ring[k]),
                              (size_t)bp->max_frames * (sizeof(AdaptArgs) + sizeof(RqsArgs)), hipHostMallocDefault);
    }
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->res_host), (size_t)bp->max_frames * sizeof(rl_result), hipHostMallocDefault);
    if (e != hipSuccess) {
        rl_batch_destroy(b);
        return fail(RL_ENOMEM, "batch host allocation failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return RL_OK;
}

RL_API rl_status rl_batch_destroy(rl_batch* b)
{
    if (!b) return RL_OK;
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    for (int k = 0; k < kJobRing; ++k) {
        if (b->up_ev[k]) {
            (void)hipEventSynchronize(b->up_ev[k]);
            (void)hipEventDestroy(b->up_ev[k]);
        }
        if (b->job_ring[k]) (void)hipHostFree(b->job_ring[k]);
        if (b->ad_ev[k]) {
            (void)hipEventSynchronize(b->ad_ev[k]);
            (void)hipEventDestroy(b->ad_ev[k]);
        }
        if (b->ad_ring[k]) (void)hipHostFree(b->ad_ring[k]);
    }
    if (b->res_host) (void)hipHostFree(b->res_host);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->mark) (void)hipEventDestroy(b->mark);
    delete b;
    return RL_OK;
}

// The relocalisation requests of a batch (indices reloc into reqs) as one
// launch sequence on the batch's stream.
static rl_status batch_relocalise_queue(rl_batch* b, const rl_request* reqs, const std::vector<int>& reloc,
                                        rl_result* dev_results, int maxN, int maxIters, int maxEta, bool any_lm,
                                        int lm_iters, const std::vector<int>& entering, int32_t use_graph)
{
    // Launch shapes come in few classes so that few graphs are captured:
    // grids cover the batch's largest frame, and the job count is padded to
    // a power of two with empty jobs (no pixels, no hypotheses), which every
    // kernel leaves at once.
    const int maxP = b->bp.max_width * b->bp.max_height;
    const int n = (int)reloc.size();
    int nq = 1;
    while (nq < n) nq *= 2;
    nq = std::min(nq, b->bp.max_frames);
    // each room: mode update if stale (on the room's stream, after the batches
    // that read the old modes), and this batch after the last update
    std::vector<rl_room*> rooms;
    for (int i : reloc)
        if (std::find(rooms.begin(), rooms.end(), reqs[i].room) == rooms.end()) rooms.push_back(reqs[i].room);
    for (rl_room* r : rooms) {
        rl_status s = room_read_begin(r, b->stream);
        if (s != RL_OK) return s;
    }
    // the pinned table to fill: its previous upload (kJobRing calls ago) has
    // to have been read by the copy engine first
    const int slot_k = b->ring;
    Job* job_host = b->job_ring[slot_k];
    hipError_t e = hipEventSynchronize(b->up_ev[slot_k]);
    if (e != hipSuccess) return hip_fail(e, "job table reuse");
    // job slot -> request (position in reloc), -1 for an empty job.  The
    // search runs job j's blocks on XCD j % 8 (eight jobs or more).  When the
    // jobs carry equal search work (hypotheses x iterations), the requests
    // are grouped by room and dealt to the XCDs in equal contiguous runs: an
    // XCD's L2 then holds few rooms' tables, and each XCD gets a run of
    // consecutive requests rather than every eighth.  Jobs of unequal work
    // keep request order, which balances the XCDs better than runs by count.
    // A job's slot changes no result.
    std::vector<int> at(nq, -1);
    std::vector<long long> work(n);
    bool equal_work = true;
    for (int k = 0; k < n; ++k) {
        const rl_request& q = reqs[reloc[k]];
        work[k] = (long long)(q.n_hypotheses > 0 ? q.n_hypotheses : q.room->N) *
                  q.room->p.max_candidate_generation_iterations;
        equal_work = equal_work && work[k] == work[0];
    }
    if (nq >= 8 && nq % 8 == 0 && equal_work) {
        std::vector<int> order;
        for (rl_room* r : rooms)
            for (int k = 0; k < n; ++k)
                if (reqs[reloc[k]].room == r) order.push_back(k);
        int k = 0;
        for (int x = 0; x < 8; ++x)
            for (int i = 0; i < n / 8 + (x < n % 8 ? 1 : 0); ++i) at[i * 8 + x] = order[k++];
    } else if (nq >= 8 && nq % 8 == 0) {
        // unequal work: longest first, each to the least loaded XCD with a
        // free slot (on a tie, one that already holds the job's room)
        std::vector<int> order(n);
        for (int k = 0; k < n; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
        long long load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        int used[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        std::vector<rl_room*> held[8];
        for (int k : order) {
            rl_room* r = reqs[reloc[k]].room;
            int best = -1;
            bool best_room = false;
            for (int x = 0; x < 8; ++x) {
                if (used[x] * 8 + x >= nq) continue;
                const bool has = std::find(held[x].begin(), held[x].end(), r) != held[x].end();
                if (best < 0 || load[x] < load[best] || (load[x] == load[best] && has && !best_room)) {
                    best = x;
                    best_room = has;
                }
            }
            at[used[best]++ * 8 + best] = k;
            load[best] += work[k];
            if (std::find(held[best].begin(), held[best].end(), r) == held[best].end()) held[best].push_back(r);
        }
    } else {
        for (int k = 0; k < n; ++k) at[k] = k;
    }
    for (int i = 0; i < nq; ++i) {
        Job J;
        if (at[i] >= 0) {
            const rl_request& q = reqs[reloc[at[i]]];
            const int N = q.n_hypotheses > 0 ? q.n_hypotheses : q.room->N;
            J = make_job(q.room, b->ws, b->slots[i], &q.frame, q.request_seed, N);
            J.lm_split = 0;                 // the batch's passes are launched for this layout
            J.result = dev_results + reloc[at[i]];
            if (q.pose_update != 0) J.lm = q.pose_update > 0 ? 1 : 0;
        } else {
            std::memset(&J, 0, sizeof(J));
            J.T = b->bp.n_trees;
            J.st = reinterpret_cast<JobState*>(b->ws + b->slots[i].state);
            J.result = reinterpret_cast<rl_result*>(b->ws + b->slots[i].result);
        }
        J.TP = b->TP;
        J.fast_max = 64 * b->sched.fw;
        J.screen = b->sched.screen;
        J.lm_plan = reinterpret_cast<int*>(b->ws + b->slots[0].lm_plan);   // one plan per launch
        J.trace = 0;
        job_host[i] = J;
    }
    Job* jd = reinterpret_cast<Job*>(b->ws + b->jobs_off);
    e = hipMemcpyAsync(jd, job_host, (size_t)nq * sizeof(Job), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->up_ev[slot_k], b->stream);
    if (e != hipSuccess) return hip_fail(e, "job upload");
    b->ring = (slot_k + 1) % kJobRing;
    const int nptiles = (maxEta + b->TP - 1) / b->TP;
    if (use_graph && b->stream == nullptr)
        return fail(RL_EINVAL, "graph replay needs a batch created on a non-default stream");
    std::vector<long long> key = {nq, maxN, maxIters, nptiles, maxEta, b->bp.n_trees, b->sched.ipt, b->sched.fw, b->sched.top,
                                  b->sched.win, any_lm ? 1 : 0, lm_iters};
    for (int v : entering) key.push_back(v);
    e = run_sequence(b->graphs, key, use_graph && b->timer.kernel == RL_TIMER_NONE, b->stream, [&]() {
        return launch_sequence(jd, nq, maxP, maxN, maxIters, b->bp.n_trees, entering, nptiles, maxEta, b->rows,
                               any_lm, lm_iters, false, b->sched, b->timer, b->stream);
    });
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    // the next mode update of each room waits for this batch
    for (rl_room* r : rooms) {
        rl_status s = room_read_end(r, b->stream);
        if (s != RL_OK) return s;
    }
    return RL_OK;
}

// The adaptation requests of a batch, on the batch's stream after its
// relocalisations and after the work queued so far on each room's stream.
// Round k holds the k-th adaptation of every room (so a room's adaptations
// keep their request order) and is one launch sequence over those rooms
// (split by tree count), followed by one launch for the rooms' round-robin
// mode steps, which first wait for the batches still reading the old modes.
// Each room's stream, and every later reader of its modes, is then ordered
// after the batch.
static rl_status batch_adapt(rl_batch* b, const rl_request* reqs, const std::vector<int>& adapt,
                             rl_result* dev_results)
{
    std::vector<rl_room*> rooms;
    std::vector<int> seen_count;
    std::vector<std::vector<int>> rounds;
    for (int i : adapt) {
        rl_room* r = reqs[i].room;
        const auto it = std::find(rooms.begin(), rooms.end(), r);
        const size_t ri = (size_t)(it - rooms.begin());
        if (it == rooms.end()) {
            rooms.push_back(r);
            seen_count.push_back(0);
        }
        const size_t k = (size_t)seen_count[ri]++;
        if (k >= rounds.size()) rounds.emplace_back();
        rounds[k].push_back(i);
    }
    hipError_t e = hipSuccess;
    for (rl_room* r : rooms) {
        e = hipEventRecord(r->bev, r->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, r->bev, 0);
        if (e == hipSuccess && r->rr_leaves) {
            for (hipEvent_t ev : r->readers) {
                if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
                r->spare.push_back(ev);
            }
            r->readers.clear();
        }
        if (e != hipSuccess) return hip_fail(e, "batched adaptation ordering");
    }
    // the pinned tables to fill: their previous upload has to have been read
    const int slot_k = b->ad_slot;
    e = hipEventSynchronize(b->ad_ev[slot_k]);
    if (e != hipSuccess) return hip_fail(e, "adaptation table reuse");
    AdaptArgs* ha = reinterpret_cast<AdaptArgs*>(b->ad_ring[slot_k]);
    RqsArgs* hr = reinterpret_cast<RqsArgs*>(b->ad_ring[slot_k] + (size_t)b->bp.max_frames * sizeof(AdaptArgs));
    struct Step { int a0, na, r0, nr; };
    std::vector<Step> steps;
    int na = 0, nr = 0;
    for (const std::vector<int>& rd : rounds) {
        std::vector<int> trees;
        for (int i : rd)
            if (std::find(trees.begin(), trees.end(), reqs[i].room->T) == trees.end()) trees.push_back(reqs[i].room->T);
        for (int T : trees) {
            Step st{na, 0, nr, 0};
            for (int i : rd) {
                rl_room* r = reqs[i].room;
                if (r->T != T) continue;
                AdaptArgs a = adapt_args(r, &reqs[i].frame, reqs[i].cam_to_world);
                a.result = dev_results + i;
                a.mode_version = r->mode_version + (r->rr_leaves ? 1u : 0u);   // after its own round-robin step
                ha[na++] = a;
                ++st.na;
                r->modes_stale = true;
                if (r->rr_leaves) {
                    RqsArgs q = rqs_args(r);
                    q.rr_first = r->rr_cursor;
                    q.rr_count = (uint32_t)r->rr_leaves;
                    r->rr_cursor = (uint32_t)((r->rr_cursor + (uint64_t)r->rr_leaves) % q.n_leaves);
                    ++r->mode_version;
                    hr[nr++] = q;
                    ++st.nr;
                }
            }
            steps.push_back(st);
        }
    }
    AdaptArgs* da = reinterpret_cast<AdaptArgs*>(b->ws + b->ad_off);
    RqsArgs* dr = reinterpret_cast<RqsArgs*>(b->ws + b->rq_off);
    e = hipMemcpyAsync(da, ha, (size_t)na * sizeof(AdaptArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && nr > 0) e = hipMemcpyAsync(dr, hr, (size_t)nr * sizeof(RqsArgs), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->ad_ev[slot_k], b->stream);
    if (e != hipSuccess) return hip_fail(e, "adaptation table upload");
    b->ad_slot = (slot_k + 1) % kJobRing;
    for (const Step& st : steps) {
        e = launch_adapt_jobs(da + st.a0, ha + st.a0, st.na, b->stream);
        if (e == hipSuccess && st.nr > 0) e = launch_rqs_jobs(dr + st.r0, hr + st.r0, st.nr, 1024, b->stream);
        if (e != hipSuccess) return hip_fail(e, "batched adaptation");
    }
    e = hipEventRecord(b->mark, b->stream);
    for (rl_room* r : rooms) {
        if (e == hipSuccess) e = hipStreamWaitEvent(r->stream, b->mark, 0);
        if (e == hipSuccess && r->rr_leaves) {
            e = hipEventRecord(r->wev, b->stream);
            r->wrote = true;
        }
    }
    if (e != hipSuccess) return hip_fail(e, "batched adaptation ordering");
    return RL_OK;
}

RL_API rl_status rl_batch_relocalise_async(rl_batch* b, const rl_request* reqs, int32_t n, rl_result* dev_results,
                                           int32_t use_graph)
{
    if (!b || !reqs || !dev_results) return fail(RL_EINVAL, "NULL argument");
    if (n < 1 || n > b->bp.max_frames) return fail(RL_EINVAL, "batch of %d requests (1..%d allowed)", n, b->bp.max_frames);
    int maxN = 0, maxIters = 0, maxEta = 0;
    bool any_lm = false;
    int lm_iters = 0;
    std::vector<int> entering, reloc, adapt;
    for (int i = 0; i < n; ++i) {
        const rl_request& q = reqs[i];
        rl_room* r = q.room;
        if (!r) return fail(RL_EINVAL, "request %d: room is NULL", i);
        if (q.kind == RL_REQ_ADAPT) {
            rl_status s = validate_frame(&q.frame, r->max_w, r->max_h);
            if (s == RL_OK) s = check_pose(q.cam_to_world);
            if (s != RL_OK) return fail(s, "request %d: %s", i, g_err.c_str());
            adapt.push_back(i);
            continue;
        }
        if (q.kind != RL_REQ_RELOCALISE) return fail(RL_EINVAL, "request %d: kind must be 0 or 1", i);
        reloc.push_back(i);
        rl_status s = validate_frame(&q.frame, b->bp.max_width, b->bp.max_height);
        if (s != RL_OK) return fail(s, "request %d: %s", i, g_err.c_str());
        if (r->T != b->bp.n_trees) return fail(RL_EINVAL, "request %d: room has %d trees, batch %d", i, r->T, b->bp.n_trees);
        if (r->T * r->M > b->rows) return fail(RL_EINVAL, "request %d: room has up to %d modes per pixel, batch %d", i, r->T * r->M, b->rows);
        const int N = q.n_hypotheses > 0 ? q.n_hypotheses : r->N;
        if (N > b->bp.max_hypotheses || N > 4096) return fail(RL_EINVAL, "request %d: %d hypotheses exceed the batch maximum", i, N);
        if (r->eta > b->bp.max_eta) return fail(RL_EINVAL, "request %d: eta exceeds the batch maximum", i);
        std::vector<int> ent;
        const int R = rounds_for(N, r->p.max_pose_candidates_after_cull, r->p.max_relocalisations_to_output, &ent);
        if (R > b->bp.max_rounds) return fail(RL_EINVAL, "request %d: %d rounds exceed the batch maximum", i, R);
        if (ent.size() > entering.size()) entering.resize(ent.size(), 0);
        for (size_t k = 0; k < ent.size(); ++k) entering[k] = std::max(entering[k], ent[k]);
        maxN = std::max(maxN, N);
        maxIters = std::max(maxIters, r->p.max_candidate_generation_iterations);
        maxEta = std::max(maxEta, r->eta);
        if (q.pose_update < -1 || q.pose_update > 1) return fail(RL_EINVAL, "request %d: pose_update must be -1, 0 or 1", i);
        const bool lm = q.pose_update == 0 ? r->p.pose_update != 0 : q.pose_update > 0;
        any_lm = any_lm || lm;
        if (lm) lm_iters = std::max(lm_iters, r->p.lm_iterations);
    }
    if (!reloc.empty()) {
        const rl_status s = batch_relocalise_queue(b, reqs, reloc, dev_results, maxN, maxIters, maxEta, any_lm,
                                                   lm_iters, entering, use_graph);
        if (s != RL_OK) return s;
    }
    // adaptations after every relocalisation of the batch
    if (!adapt.empty()) {
        const rl_status s = batch_adapt(b, reqs, adapt, dev_results);
        if (s != RL_OK) return s;
    }
    const hipError_t e = hipEventRecord(b->ev, b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch event");
    return RL_OK;
}

RL_API rl_status rl_batch_relocalise(rl_batch* b, const rl_request* reqs, int32_t n, rl_result* results,
                                     int32_t use_graph)
{
    if (!b || !results) return fail(RL_EINVAL, "NULL argument");
    rl_result* dres = reinterpret_cast<rl_result*>(b->ws + b->results_off);
    rl_status s = rl_batch_relocalise_async(b, reqs, n, dres, use_graph);
    if (s != RL_OK) return s;
    hipError_t e = hipMemcpyAsync(b->res_host, dres, (size_t)n * sizeof(rl_result), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "batch relocalise");
    std::memcpy(results, b->res_host, (size_t)n * sizeof(rl_result));
    return RL_OK;
}

static rl_status set_timer(Timer* t, int32_t kernel, void* start_event, void* stop_event)
{
    if (kernel < RL_TIMER_NONE || kernel > RL_TIMER_RANSAC) return fail(RL_EINVAL, "unknown timer kernel %d", kernel);
    if (kernel != RL_TIMER_NONE && (!start_event || !stop_event)) return fail(RL_EINVAL, "timer events are NULL");
    t->kernel = kernel;
    t->start = reinterpret_cast<hipEvent_t>(start_event);
    t->stop = reinterpret_cast<hipEvent_t>(stop_event);
    return RL_OK;
}

RL_API rl_status relocaliser_set_timer(rl_room* r, int32_t kernel, void* start_event, void* stop_event)
{
    if (!r) return fail(RL_EINVAL, "room is NULL");
    return set_timer(&r->timer, kernel, start_event, stop_event);
}

RL_API rl_status rl_batch_set_timer(rl_batch* b, int32_t kernel, void* start_event, void* stop_event)
{
    if (!b) return fail(RL_EINVAL, "batch is NULL");
    return set_timer(&b->timer, kernel, start_event, stop_event);
}
