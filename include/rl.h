/*
 * rl.h -- C ABI of the MI355X relocaliser library (librl.so).
 *
 * The library implements the per-frame hot path of the adaptive
 * regression-forest camera relocaliser of Cavallari et al., "Real-Time RGB-D
 * Camera Pose Estimation in Novel Scenes using a Relocalisation Cascade"
 * (TPAMI 2019, arXiv 1810.12163):
 *   - Depth and DA-RGB features and routing through every tree (Eq. 1-3,
 *     Sec. 3.2.1), leaf indexing of an implicit complete binary tree;
 *   - online adaptation into bounded per-leaf reservoirs and Really Quick
 *     Shift modes (Sec. 3.2.2);
 *   - pose estimation: Kabsch hypotheses from pixel triplets with the three
 *     checks, Eq. 5 energies on growing pixel sets, preemptive halving
 *     (Sec. 3.2.3), plus an optional closed-form refit over the inliers.
 *
 * Conventions (all entry points):
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary CPU memory.  The library never frees caller
 *     memory and never allocates device memory after relocaliser_create /
 *     rl_batch_create (those allocate nothing on the device either: all
 *     device state lives in caller-provided buffers).
 *   - Poses are camera->world, 4x4 row-major float32, metres, last row
 *     0 0 0 1 (the paper's hypotheses map camera space to world space).
 *   - Camera frame: x right, y down, z forward; x^C = D(u) K^-1 (u, v, 1)^T on
 *     integer pixel coordinates.  Depth: float32 metres, 0 = invalid.
 *   - Errors are returned as rl_status; negative values are errors, and
 *     rl_last_error() gives a thread-local message.  RL_NO_POSE is not an
 *     error: no hypothesis survived (energy = +inf, pose = identity).
 *   - A room handle is bound to one HIP stream and is not thread-safe;
 *     different rooms may be used concurrently from different threads.
 */
#ifndef RL_H_
#define RL_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RL_OK = 0,
    RL_NO_POSE = 1,
    RL_EINVAL = -1,
    RL_ENOMEM = -2,
    RL_EDEVICE = -3,
    RL_EBUSY = -4
} rl_status;

typedef struct { float fx, fy, cx, cy; } rl_intrinsics;

/*
 * One RGB-D frame in device memory, read in place (no copy is required of
 * the caller).  width and height (multiples of 4) and K describe the frame as
 * relocalised.  Pixel (x, y) is sample (step * x, step * y) of the buffers:
 *   depth: float32 metres (0 = invalid) at byte offset
 *          step * y * depth_pitch_bytes + step * x * 4;
 *   rgb:   channel c (0 = R, 1 = G, 2 = B) at byte offset
 *          step * y * rgb_pitch_bytes + step * x * rgb_channels + c.
 * step 2 relocalises the 2x decimated frame of Sec. 3.2.5's cascade in place
 * (K then is the decimated frame's: the full frame's fx, fy, cx, cy halved).
 * Zero fields take defaults: rgb_channels 3, step 1, pitches of tightly
 * packed rows of the buffers (width * step * 4 and width * step *
 * rgb_channels bytes).  RL_EINVAL for rgb_channels other than 3 or 4, step
 * other than 1 or 2, or pitches below those of packed rows.
 */
typedef struct {
    int32_t width, height;
    const float* depth;      /* device, float32 metres, 0 = invalid              */
    const uint8_t* rgb;      /* device, uint8 R, G, B[, unused]                  */
    rl_intrinsics K;
    int32_t rgb_channels;    /* 3 (RGB) or 4 (RGBA, the fourth byte unused); 0 = 3 */
    int32_t rgb_pitch_bytes; /* bytes from one buffer row to the next; 0 = packed  */
    int32_t depth_pitch_bytes; /* bytes from one buffer row to the next; 0 = packed */
    int32_t step;            /* 1: every pixel; 2: every second pixel and row; 0 = 1 */
} rl_frame;

/*
 * Parameters.  Names follow the paper's parameter table (Table 8) in
 * snake_case; the remaining fields are settings the paper leaves open.
 */
typedef struct {
    /* forest structure (nodes are supplied by the caller) */
    int32_t n_trees;                 /* 1..8                                            */
    int32_t depth;                   /* split levels, 1..15; 2^depth leaves per tree     */
    int32_t ref_width;               /* image width the offsets are expressed for        */
    /* Table 8, Forest */
    float clusterer_sigma;           /* RQS Gaussian kernel width (m)                    */
    float clusterer_tau;             /* RQS maximum link distance (m)                    */
    int32_t max_cluster_count;       /* M_max, 1..64, n_trees * M_max <= 255             */
    int32_t min_cluster_size;
    int32_t reservoir_capacity;      /* kappa, 1..4096                                   */
    /* Table 8, RANSAC */
    int32_t max_candidate_generation_iterations;
    int32_t max_pose_candidates;     /* N_max, 1..4096                                   */
    int32_t max_pose_candidates_after_cull;  /* N_cull; >= N_max disables the initial cull */
    int32_t ransac_inliers_per_iteration;    /* eta, 1..4096                             */
    int32_t max_relocalisations_to_output;   /* >= 1                                     */
    int32_t use_prediction_covariance;       /* Mahalanobis (1) or Euclidean (0) Eq. 5   */
    int32_t pose_update;                     /* 1: LM refinement in se(3) every round    */
    int32_t final_refine;                    /* 1: Kabsch refit over the inliers         */
    int32_t lm_iterations;                   /* LM iterations per survivor per round, 0..64 */
    float min_squared_distance_between_sampled_modes;   /* check 2 (m^2)                */
    float max_translation_error_for_correct_pose;       /* check 3 tolerance (m)        */
    float max_colour_linf;           /* check 1 threshold, 0..255 scale                  */
    float inlier_threshold;          /* refit inlier distance (m)                        */
    float cov_regulariser;           /* lambda added to every mode covariance (m^2)      */
    uint64_t seed;                   /* generator seed of the room                       */
} rl_params;

typedef struct rl_room rl_room;

/* Forest node record as supplied by the caller: 16 bytes per branch node,
 * (2^depth - 1) nodes per tree in implicit complete-tree order, tree-major.
 * kind 0 = Depth feature, 1 + c = DA-RGB feature on colour channel c. */
typedef struct { float dx, dy, tau; uint32_t kind; } rl_node;

/*
 * A random forest (the paper's "Is Pre-Training Necessary?" section: complete
 * trees with random split functions, adapted online, relocalise as well as
 * trained ones).  For every branch node: a Depth feature with probability
 * p_depth, else a DA-RGB feature on a uniformly drawn channel; offsets
 * uniform in +-offset_range (pixel-metres); thresholds uniform in
 * +-tau_depth (metres) for Depth nodes, +-tau_colour (0..255 scale) for
 * DA-RGB nodes.  Draws: Philox4x32-10 keyed by seed (two words, low first),
 * counters (tree, node, 0, 0) -> (kind, channel, dx, dy) and (tree, node, 1, 0)
 * -> tau; a uniform in [a, b) is a + (b - a) * (u + 0.5) * 2^-32 in double,
 * rounded to float; channel = (u * 3) >> 32.
 * host_nodes: n_trees * (2^depth - 1) records, tree-major (NULL: only *bytes
 * is set).  RL_EINVAL for n_trees outside 1..8, depth outside 1..15, a
 * probability outside [0, 1] or negative ranges.
 */
typedef struct {
    int32_t n_trees, depth;
    float p_depth;                   /* probability of a Depth feature (0.4 in the paper) */
    float offset_range;              /* pixel-metres */
    float tau_depth;                 /* metres */
    float tau_colour;                /* 0..255 scale */
    uint64_t seed;
} rl_forest_params;
rl_status rl_forest_generate(const rl_forest_params* fp, rl_node* host_nodes, size_t* bytes);

/*
 * Fills *out with a named preset: "default", "fast", "intermediate", "slow"
 * (Table 8 of the paper) or one of the synthetic workloads: "c1" (160x120,
 * one depth-8 tree, kappa 64, 64 hypotheses, eta 100), "c2" (640x480, five
 * depth-15 trees, kappa 1024, at most 10 modes per leaf, 1024 hypotheses,
 * eta 500, refit), "c3" (the c2 forest with room for the cascade's widest
 * stage: 4096 hypotheses, 16 outputs; its stages are per-call settings),
 * "c4" and "c5" (the c2 room of the batching and serving workloads).
 * RL_EINVAL for an unknown name.
 */
rl_status rl_params_preset(const char* name, rl_params* out);

/*
 * Checks a parameter block (RL_EINVAL with a message when invalid).
 */
rl_status rl_params_validate(const rl_params* p);

/*
 * Device bytes a room needs.  persistent: forest, reservoirs, counters and
 * modes (must outlive the room).  scratch: per-frame work space for frames up
 * to max_width x max_height (multiples of 4, at least 8x8, fewer than 2^24
 * pixels; RL_EINVAL otherwise).  Both must be 256-byte aligned.
 */
rl_status relocaliser_state_bytes(const rl_params* p, int32_t max_width, int32_t max_height,
                                  size_t* persistent, size_t* scratch);

/*
 * Creates a room.  host_nodes: n_trees * (2^depth - 1) rl_node records (host);
 * they are copied into dev_persistent, whose reservoirs and modes are cleared.
 * dev_persistent / dev_scratch: caller-owned device buffers of at least the
 * sizes relocaliser_state_bytes reported.  hip_stream: the hipStream_t all
 * work of this room is queued on (NULL = default stream).
 */
rl_status relocaliser_create(const rl_params* p, const rl_node* host_nodes, int32_t max_width,
                             int32_t max_height, void* dev_persistent, void* dev_scratch,
                             void* hip_stream, rl_room** out);

/* Destroys the handle (the caller's buffers are left untouched). */
rl_status relocaliser_destroy(rl_room* room);

/*
 * Room persistence.  relocaliser_save writes the room's whole persistent
 * state (forest, reservoirs, arrival counters, dirty flags, modes, colour
 * boxes) and its mode-schedule position to path, after the work queued on
 * the room's stream; relocaliser_load reads such a file into a room created
 * with the same forest shape (n_trees, depth, max_cluster_count,
 * reservoir_capacity), after every batch that reads the room.  Both are
 * synchronous; they stage through a 64 MiB pinned host buffer.  RL_EINVAL for
 * a file that cannot be opened, read or written, a bad header or a shape
 * mismatch (the room is unchanged then, except after a short read).
 */
rl_status relocaliser_save(rl_room* room, const char* path);
rl_status relocaliser_load(rl_room* room, const char* path);

/*
 * Online adaptation (Sec. 3.2.2): when reliable != 0, the pixels on the
 * 4-pixel grid {(4i, 4j), i, j >= 1} with valid depth are routed through every
 * tree and their world points x^W = H x^C (with colour) enter the reached
 * leaves' reservoirs by Algorithm R; reliable == 0 is a no-op (the paper skips
 * frames whose tracking is unreliable).  cam_to_world: host, 16 floats, must
 * be rigid (|R^T R - I| <= 1e-3).  Asynchronous on the room's stream; the
 * frame buffers must stay valid until that work has completed.
 */
rl_status relocaliser_adapt(rl_room* room, const rl_frame* frame, const float cam_to_world[16],
                            int32_t reliable);

/* Re-clusters every leaf whose reservoir changed since the last call (RQS).
 * Under the exact schedule (the default) every relocalisation does this
 * implicitly.  Asynchronous. */
rl_status relocaliser_update_modes(rl_room* room);

/*
 * Mode-update schedule (Sec. 3.2.2).  leaves_per_frame = 0 (default): exact,
 * every adapted leaf is re-clustered before the next relocalisation, so modes
 * are a function of the reservoirs.  leaves_per_frame = K > 0: amortised as
 * in the paper, each adapted frame is followed by RQS of the next K leaves of
 * the forest (leaf index t * 2^D + leaf, in order, wrapping around; the first
 * call starts at leaf 0), and relocalisation uses the modes as they are.
 * K <= n_trees * 2^depth, else RL_EINVAL.  Takes effect at the next adapt;
 * relocaliser_update_modes still performs an exact update when called.
 */
rl_status relocaliser_set_mode_schedule(rl_room* room, int32_t leaves_per_frame);

/*
 * Relocalises one frame (Sec. 3.2.3): synchronous on the room's stream.  On
 * a non-default stream the launch sequence is captured once per frame size
 * into a HIP graph and replayed (direct launches while a kernel timer is set).
 * request_seed selects the generator stream of this request (results do not
 * depend on anything else).  Outputs (host): cam_to_world_out[16], energy_out
 * = Eq. 5 energy of the winning hypothesis over the final pixel set (before
 * any refit), mean_energy_out = energy / |I|.  Returns RL_OK, RL_NO_POSE or
 * an error.
 */
rl_status relocaliser_relocalise(rl_room* room, const rl_frame* frame, uint64_t request_seed,
                                 float cam_to_world_out[16], float* energy_out,
                                 float* mean_energy_out);

/* Per-call hypothesis-generation and RANSAC settings (the parameters of
 * Table 8 that differ between the relocalisers of a cascade sharing one
 * forest).  0 (or a negative value where stated) keeps the room's own value.
 * n_hypotheses may not exceed the room's max_pose_candidates, nor eta the
 * room's ransac_inliers_per_iteration, which size its scratch. */
typedef struct {
    int32_t n_hypotheses;     /* N_max for this call                          */
    int32_t n_cull;           /* N_cull for this call                         */
    int32_t n_out;            /* maxRelocalisationsToOutput for this call     */
    int32_t final_refine;     /* -1 = room's value, 0 = off, 1 = on           */
    int32_t pose_update;      /* LM refinement: -1 = room's value, 0 = off, 1 = on */
    int32_t max_iterations;   /* maxCandidateGenerationIterations             */
    int32_t eta;              /* ransacInliersPerIteration                    */
    int32_t use_covariance;   /* -1 = room's value, 0 = Euclidean, 1 = Mahalanobis */
    float min_squared_distance;   /* minSquaredDistanceBetweenSampledModes; < 0 = room's */
    float max_translation_error;  /* maxTranslationErrorForCorrectPose; < 0 = room's     */
} rl_reloc_opts;

/* Result record (also the device-side layout written by the batch path). */
typedef struct {
    float cam_to_world[16];
    float energy, mean_energy;
    int32_t status;          /* RL_OK or RL_NO_POSE */
    int32_t n_valid;         /* hypotheses that passed generation */
    int32_t n_inliers;       /* refit inliers (0 without refit) */
    int32_t winner;          /* winning hypothesis slot, -1 if none */
    int32_t refitted;
    int32_t n_eligible;      /* pixels with depth and at least one mode */
    int32_t rounds;          /* RANSAC rounds run */
    int32_t n_out;           /* hypotheses returned in the survivor list */
    uint32_t mode_version;   /* mode updates the room had received when this request read its modes
                                (relocalisation), or after this adaptation's own (adaptation): a
                                relocalisation sees exactly the adaptations whose mode updates it
                                counts; counted from 0 at relocaliser_create */
    int32_t pad;
} rl_result;

/* Like relocaliser_relocalise but returns the full result record (host). */
rl_status relocaliser_relocalise_ex(rl_room* room, const rl_frame* frame, uint64_t request_seed,
                                    rl_result* out);

/* relocaliser_relocalise_ex with per-call RANSAC settings (opts may be NULL).
 * The cascade of the paper (Sec. 3.2.5) runs differently-tuned relocalisers
 * backed by the same forest: one room, one call per stage. */
rl_status relocaliser_relocalise_opts(rl_room* room, const rl_frame* frame, uint64_t request_seed,
                                      const rl_reloc_opts* opts, rl_result* out);

/*
 * Analytic scene surface: a point p0, unit normal n, in-plane unit axes e1,
 * e2 and half-extents (half_a <= 0 marks an infinite plane).  64 bytes.
 */
typedef struct {
    float p0[3], n[3], e1[3], e2[3];
    float half_a, half_b, pad[2];
} rl_surface;

/*
 * Model-based pose score on an analytic scene model, the stand-in here for the
 * paper's depth-raycast comparison of Sec. 3.2.4 (used to rank the final
 * hypotheses and to decide cascade fallbacks): for each pose (host, 12 floats
 * per pose: R row-major, t; camera -> world), the mean over pixels with valid
 * depth of the distance from H x^C(u) to the nearest surface (FP64).
 * n_surfaces <= 64, n_poses <= 64; host_scores receives n_poses doubles
 * (+inf when the frame has no valid depth).  Synchronous on the room's stream;
 * uses the room's scratch.
 */
rl_status rl_plane_scores(rl_room* room, const rl_frame* frame, const rl_surface* host_surfaces,
                          int32_t n_surfaces, const float* host_poses, int32_t n_poses,
                          double* host_scores);

/*
 * Model-based hypothesis score of Sec. 3.2.4 (Eq. 6-7), with the scene model
 * given as analytic surfaces.  For each pose (host, 12 floats: R row-major,
 * t; camera -> world) the library raycasts the surfaces through every pixel
 * u = (x, y) (integer coordinates; camera ray ((x-cx)/fx, (y-cy)/fy, 1)) and
 * takes the nearest hit's camera-space depth D~(u), valid when
 * min_depth <= D~(u) <= max_depth (max_depth <= 0: no upper limit).  With
 * live depth valid when positive:
 *   mu(xi) = mean over pixels valid in both of |D_l(u) - D~(u)|   (Eq. 6)
 *   s(xi)  = mu(xi) if 10 * |valid D~| >= w * h, else +inf       (Eq. 7)
 * and s = +inf when no pixel is valid in both.  The caller takes the argmin
 * (Eq. 8).  FP64; hit tests in a fixed operation order without contraction.
 * n_surfaces <= 64, n_poses <= 64.  host_scores: n_poses doubles; host_mu
 * (may be NULL): n_poses doubles (NaN when no pixel is valid in both);
 * host_counts (may be NULL): 2 per pose, (|valid D~|, |valid in both|).
 * Synchronous on the room's stream; uses the room's scratch.  RL_EINVAL for
 * NULL, out-of-range counts, non-finite inputs or min_depth < 0.
 */
rl_status rl_depth_scores(rl_room* room, const rl_frame* frame, const rl_surface* host_surfaces,
                          int32_t n_surfaces, const float* host_poses, int32_t n_poses, float min_depth,
                          float max_depth, double* host_scores, double* host_mu, int64_t* host_counts);

/*
 * rl_depth_scores without caller work space, for callers that cannot allocate
 * device memory (no room, no workspace argument).  Same computation, limits
 * on n_surfaces / n_poses / depths, outputs and errors as rl_depth_scores,
 * for a frame of at most 2^21 pixels (RL_EINVAL beyond; also for sizes that
 * are not multiples of 4 or below 8x8, and NULL depth or rgb pointers; rgb is
 * not read).  The work space is a fixed device array of this library (about
 * 2.01 MiB per device, held until the process ends); it allocates nothing
 * (no hipMalloc / hipFree, no allocating library call).  hip_stream: the
 * stream the copies and kernels run on (NULL = default stream), ordered after
 * the caller's earlier work on it.  Synchronous.  Every call on a device
 * shares that device's array, which keeps the last call's contents: calls
 * from threads of one process are serialised per device by a lock held for
 * the whole call, so they never overlap.  RL_EDEVICE on devices numbered 64
 * or above.
 */
rl_status rl_depth_scores_noalloc(const rl_frame* frame, const rl_surface* host_surfaces, int32_t n_surfaces,
                                  const float* host_poses, int32_t n_poses, float min_depth, float max_depth,
                                  void* hip_stream, double* host_scores, double* host_mu,
                                  int64_t* host_counts);

/*
 * Introspection for tests and tools: byte offset and size of an internal
 * array inside the caller's persistent (*region = 0) or scratch (*region = 1)
 * buffer.  which: see RL_BUF_* below.  Contents are valid after the stream
 * work that produced them has completed.
 */
enum {
    RL_BUF_NODES = 0,      /* rl_node[T][2^D-1]                                   persistent */
    RL_BUF_RESERVOIR = 1,  /* float4[T][L][kappa]: x, y, z, colour bits             persistent */
    RL_BUF_SEEN = 2,       /* uint32[T][L] arrivals per leaf                        persistent */
    RL_BUF_MODES = 3,      /* float[T][L][M][16] mode rows                          persistent */
    RL_BUF_NMODES = 4,     /* uint8[T][L]                                           persistent */
    RL_BUF_LEAVES = 5,     /* uint16[w*h][8] leaf per tree, 0xFFFF = none           scratch    */
    RL_BUF_NM = 6,         /* uint8[w*h] |M(u)|                                     scratch    */
    RL_BUF_ELIGIBLE = 7,   /* int32[w*h] eligible pixels, raster order              scratch    */
    RL_BUF_HYPS = 8,       /* hypothesis records (see rl_hypothesis)                scratch    */
    RL_BUF_ILIST = 9,      /* int32[rounds*eta] scoring pixels I                    scratch    */
    RL_BUF_TRACE_SLOTS = 10, /* int32[rounds][N] survivors after each round          scratch    */
    RL_BUF_TRACE_ENERGY = 11,/* double[rounds][N] their energies                      scratch    */
    RL_BUF_SURVIVORS = 12, /* int32[N] current survivor slots, best first           scratch    */
    RL_BUF_ENERGY = 13,    /* double[N] energy per slot                             scratch    */
    RL_BUF_DIRTY = 14,     /* uint8[T][L] leaves awaiting re-clustering             persistent */
    RL_BUF_CBOX = 15,      /* uint32[T][L][M][2] per mode: lowest R,G,B values passing the colour
                              check, then highest, as R | G << 10 | B << 20 (a channel with
                              lo > hi passes nothing)                               persistent */
    RL_BUF_EREC = 16,      /* uint64[w*h][ew] per eligible-list entry: |M(u)| in bits 0-7, the
                              colour-check bit of mode m of M(u) in bit 8 + m (m < 56), then 64
                              bits per further word                                 scratch    */
    RL_BUF_POSE64 = 17     /* double[N][12] per slot: pose after LM refinement (R row-major, t);
                              valid for the survivors of the last call with pose_update scratch */
};
rl_status relocaliser_buffer(const rl_room* room, int32_t which, size_t* offset, size_t* bytes,
                             int32_t* region);

/* Hypothesis record layout of RL_BUF_HYPS (80 bytes). */
typedef struct {
    float R[9];       /* row-major rotation (camera -> world), rounded to float32 */
    float t[3];
    int32_t pix[3];   /* pixel indices y*w + x of the triplet */
    int32_t mode[3];  /* index of the sampled mode within M(u) */
    int32_t iter;     /* generation iteration that passed; -1 if none */
    int32_t valid;
} rl_hypothesis;

/* Records survivors and energies of every RANSAC round (off by default). */
rl_status relocaliser_set_trace(rl_room* room, int32_t on);

/* ---------------------------------------------------------------------- */
/* Batched relocalisation: many frames (any mix of rooms and resolutions)
 * through one sequence of launches, optionally replayed from a HIP graph.  */

typedef struct rl_batch rl_batch;

typedef struct {
    int32_t max_frames;      /* frames per submission                          */
    int32_t max_width, max_height;
    int32_t max_hypotheses;  /* largest N of any request                       */
    int32_t max_eta;         /* largest eta                                    */
    int32_t max_rounds;      /* largest number of RANSAC rounds                */
    int32_t n_trees;         /* every room of a batch has this many trees      */
    int32_t max_modes_per_pixel; /* largest n_trees * M_max                    */
} rl_batch_params;

/* Request kinds of a batch. */
enum { RL_REQ_RELOCALISE = 0, RL_REQ_ADAPT = 1 };

/*
 * One request of a batch.  kind RL_REQ_RELOCALISE: relocalise frame in room
 * (Sec. 3.2.3); cam_to_world is ignored.  kind RL_REQ_ADAPT: online
 * adaptation of room by frame at the reliable pose cam_to_world (Sec. 3.2.2,
 * as relocaliser_adapt with reliable != 0; camera->world, 4x4 row-major, must
 * be rigid); request_seed, n_hypotheses and pose_update are ignored.
 */
typedef struct {
    rl_room* room;
    rl_frame frame;
    uint64_t request_seed;
    int32_t n_hypotheses;    /* 0 = the room's max_pose_candidates              */
    int32_t pose_update;     /* LM refinement: 0 = the room's value, 1 = on, -1 = off */
    int32_t kind;            /* RL_REQ_RELOCALISE or RL_REQ_ADAPT               */
    float cam_to_world[16];  /* RL_REQ_ADAPT: the frame's pose                  */
} rl_request;

/* Device workspace bytes of a batch context (256-byte aligned buffer); the
 * frame limits are those of relocaliser_state_bytes. */
rl_status rl_batch_workspace_bytes(const rl_batch_params* bp, size_t* bytes);

rl_status rl_batch_create(const rl_batch_params* bp, void* dev_workspace, void* hip_stream,
                          rl_batch** out);
rl_status rl_batch_destroy(rl_batch* b);

/*
 * Runs n <= max_frames requests on the batch's stream: the relocalisations
 * as one launch sequence, then the adaptations in request order (a snapshot:
 * every relocalisation of the batch sees the rooms as they were before the
 * batch's adaptations).  Every room's modes are brought up to date first.
 * The result for relocalisation request i is identical to
 * relocaliser_relocalise_ex on the same room, frame and request_seed, and the
 * rooms afterwards equal those of relocaliser_adapt calls of the adaptation
 * requests in order (under either mode schedule); the record of an
 * adaptation request has status RL_OK, winner -1 and the identity pose.
 * The adaptations run on the batch's stream after its relocalisations and
 * after the work already queued on each adapted room's stream, as rounds of
 * multi-room launches (round k adapts the k-th frame of each room, so a
 * room's adaptations keep request order); each room's stream, and every
 * later reader of its modes, is ordered after them, and the batch completes
 * after all of them.  results: host array of n records; the call is
 * synchronous.  use_graph != 0 captures the relocalisations' launch sequence
 * for this batch shape once and replays it on later calls with the same
 * shape (adaptations are launched directly).  RL_EINVAL for an unknown kind,
 * a frame beyond the batch's limits (relocalisation) or the room's
 * (adaptation), or a pose that is not rigid.
 */
rl_status rl_batch_relocalise(rl_batch* b, const rl_request* reqs, int32_t n, rl_result* results,
                              int32_t use_graph);

/* Asynchronous form: results are written to dev_results (device, n records);
 * completion is ordered on the batch's stream.  The requests are read during
 * the call; calls may be queued back to back with different requests (each
 * call's job table is kept until its upload has completed, and the batch's
 * work space is reused in stream order).  Frame buffers and dev_results must
 * stay valid until the batch has completed. */
rl_status rl_batch_relocalise_async(rl_batch* b, const rl_request* reqs, int32_t n,
                                    rl_result* dev_results, int32_t use_graph);

/*
 * Kernel timing: when kernel != RL_TIMER_NONE, the library records
 * start_event just before and stop_event just after that kernel (or kernel
 * group) on the stream it launches it on, in every later relocalisation of
 * this room / batch (such calls launch directly, not from a graph).  The events are the
 * caller's hipEvent_t handles, created with timing enabled; read them with
 * hipEventElapsedTime after the call has completed.
 */
enum {
    RL_TIMER_NONE = 0,
    RL_TIMER_TRAVERSE = 1,     /* features + routing of every pixel             */
    RL_TIMER_HYP_SEARCH = 2,   /* hypothesis generation search                  */
    RL_TIMER_RANSAC = 3        /* all scoring and selection rounds              */
};
rl_status relocaliser_set_timer(rl_room* room, int32_t kernel, void* start_event, void* stop_event);
rl_status rl_batch_set_timer(rl_batch* b, int32_t kernel, void* start_event, void* stop_event);

/*
 * Launch schedule (for callers that tune it to their device and workload):
 * ipt = hypothesis-search iterations per thread (2, 4 or 8); fast_waves =
 * width in 64-lane waves (1, 2 or 4) of the scoring that, once a request has
 * at most 64 * fast_waves surviving hypotheses, scores all its remaining
 * rounds at once; lds_levels = tree levels the traversal reads from a
 * per-workgroup LDS copy instead of global memory (6 or 8); score_window =
 * 0 to score all those remaining rounds in one pass, or 1..3 to score that
 * many rounds first, select, and then score the rest for the survivors only
 * (less scoring work, one more pass).  None changes any result: each
 * hypothesis draws from its own Philox counters whichever thread runs it,
 * every energy is summed in the same order, and a node record is the same
 * bits wherever it is read from.  Defaults: ipt 4, fast_waves 1, lds_levels
 * 8, score_window 0 for a room (one frame per call: fewer launches) and 2
 * for a batch.  Applies to later calls; RL_EINVAL for other values.
 * Not thread-safe against concurrent calls on the same room / batch.
 */
rl_status relocaliser_set_schedule(rl_room* room, int32_t ipt, int32_t fast_waves, int32_t lds_levels,
                                   int32_t score_window);
rl_status rl_batch_set_schedule(rl_batch* b, int32_t ipt, int32_t fast_waves, int32_t lds_levels,
                                int32_t score_window);

/*
 * Degeneracy screen of the hypothesis search (result-invariant, on by
 * default).  A hypothesis needs a non-degenerate Kabsch fit (Sec. 3.2.3): the
 * exact test rejects a triplet whose cross-covariance has sigma_2 < 1e-4
 * sigma_1.  With the screen on, the parallel search already skips triplets
 * that are degenerate by a wide margin; with it off, every iteration passing
 * checks 1-3 reaches the exact test, which rejects degenerate ones and
 * continues the slot's scan from there.  Either way each slot keeps its first
 * iteration passing every check, so results are identical; off only costs
 * time (the exact test's scan is serial per slot).  Applies to later calls.
 */
rl_status relocaliser_set_degeneracy_screen(rl_room* room, int32_t on);
rl_status rl_batch_set_degeneracy_screen(rl_batch* b, int32_t on);

/* Thread-local message of the last error. */
const char* rl_last_error(void);

/* Library version string. */
const char* rl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RL_H_ */
