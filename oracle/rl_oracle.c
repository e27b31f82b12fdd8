/*
 * rl_oracle.c -- plain, slow CPU oracle of the relocaliser's per-frame path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing but the test-suite, the package smoke
 * check and the CPU-baseline leg of the benchmark may load this library.  It
 * shares no code with the GPU path and must never serve as a fallback for it.
 *
 * Method: Cavallari et al., "Real-Time RGB-D Camera Pose Estimation in Novel
 * Scenes using a Relocalisation Cascade" (TPAMI 2019, arXiv 1810.12163).
 * Every function cites the passage it follows.  Arithmetic is FP64 except
 * feature evaluation and tree routing, which are defined in float32 so that
 * leaf indices are well defined bit for bit (see oracle_traverse).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 *        (contraction off: every expression is evaluated as written).
 *        Loops over independent pixels (routing) and hypotheses (generation,
 *        scoring, refinement) may run on several threads (oracle_set_threads);
 *        each iteration writes only its own outputs, so results do not depend
 *        on the thread count.
 *
 * Parity status of each function is stated in its header comment.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define EXPORT __attribute__((visibility("default")))

/* Threads of the parallel loops (1 = serial); returns the count in effect. */
EXPORT int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
 * random numbers: as easy as 1, 2, 3", SC'11).  Written from the paper's
 * definition: 10 rounds, each multiplying counter words 0 and 2 by the two
 * round multipliers (32x32 -> 64 bits) and mixing in the round key, which is
 * bumped by the Weyl constants between rounds.
 * Pinned: bit-identical to rocRAND's philox4x32_10 engine (an independent
 * implementation) on arbitrary counters and keys.
 */
static const uint32_t PH_M0 = 0xD2511F53u;
static const uint32_t PH_M1 = 0xCD9E8D57u;
static const uint32_t PH_W0 = 0x9E3779B9u;
static const uint32_t PH_W1 = 0xBB67AE85u;

EXPORT void oracle_philox4x32(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += PH_W0; k1 += PH_W1; }
        uint64_t p0 = (uint64_t)PH_M0 * c0;
        uint64_t p1 = (uint64_t)PH_M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The 64-bit generator key of a stream: seed + request_seed * 0x9E3779B97F4A7C15
 * (mod 2^64), split into (low, high) 32-bit words. */
static void stream_key(uint64_t seed, uint64_t request_seed, uint32_t key[2])
{
    uint64_t k = seed + request_seed * 0x9E3779B97F4A7C15ULL;
    key[0] = (uint32_t)k;
    key[1] = (uint32_t)(k >> 32);
}

/* One block of four 32-bit draws for counter (tag<<28 | sub, a, b, c). */
static void philox_block(uint32_t tag, uint32_t sub, uint32_t a, uint32_t b, uint32_t c,
                         const uint32_t key[2], uint32_t r[4])
{
    uint32_t ctr[4] = {(tag << 28) | sub, a, b, c};
    oracle_philox4x32(ctr, key, r);
}

/* integer in [0, n): floor(r * n / 2^32) */
static uint32_t uniform_below(uint32_t r, uint32_t n)
{
    return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

enum { TAG_RES = 1, TAG_HYP = 2, TAG_SCORE = 3 };

/* ------------------------------------------------------------------------ */
/* Forest node record: see rlsynth/forest.py (16 bytes). */
typedef struct { float dx, dy, tau; uint32_t kind; } node_t;

static int depth_valid(float d) { return d > 0.0f && d <= 3.0e38f; }

/*
 * Features and routing, Eq. 1-3 (Sec. 3.2.1) and tree descent (Sec. 3.2.2 step 2).
 * Depth feature  f = D(p) - D(p + delta / D(p));
 * DA-RGB feature f = C(p, c) - C(p + delta / D(p), c);
 * split: f >= tau sends the example right (child 2i+2), otherwise left (2i+1).
 * Readings: offset = rint(delta * s * (1/D(p))) in float32, ties to even, with
 * s = w / w_ref; the probe is clamped to the image; a probe with invalid depth
 * reads the raw 0.  Leaves are numbered i - (2^D - 1).  An invalid centre
 * pixel reaches no leaf (0xFFFF).
 * Parity: hand-built images and trees with hand-derived leaves.
 */
static int route(const float* depth, const uint8_t* rgb, int w, int h, int x, int y,
                 const node_t* tree, int D, float s)
{
    float d = depth[(size_t)y * w + x];
    if (!depth_valid(d)) return -1;
    float inv = 1.0f / d;
    int i = 0;
    for (int lvl = 0; lvl < D; ++lvl) {
        node_t nd = tree[i];
        float dxs = nd.dx * s;
        float dys = nd.dy * s;
        float fox = rintf(dxs * inv);
        float foy = rintf(dys * inv);
        if (fox > 1048576.0f) fox = 1048576.0f;
        if (fox < -1048576.0f) fox = -1048576.0f;
        if (foy > 1048576.0f) foy = 1048576.0f;
        if (foy < -1048576.0f) foy = -1048576.0f;
        int qx = x + (int)fox, qy = y + (int)foy;
        if (qx < 0) qx = 0;
        if (qx > w - 1) qx = w - 1;
        if (qy < 0) qy = 0;
        if (qy > h - 1) qy = h - 1;
        size_t q = (size_t)qy * w + qx;
        float f;
        if (nd.kind == 0) {
            f = d - depth[q];
        } else {
            int c = (int)nd.kind - 1;
            f = (float)rgb[((size_t)y * w + x) * 3 + c] - (float)rgb[q * 3 + c];
        }
        i = 2 * i + 1 + (f >= nd.tau ? 1 : 0);
    }
    return i - ((1 << D) - 1);
}

/* leaves_out[p*T + t] for every pixel listed in pix (or all pixels if pix == NULL) */
EXPORT void oracle_traverse(const float* depth, const uint8_t* rgb, int w, int h,
                            const void* nodes, int T, int D, int ref_width,
                            const int32_t* pix, int npix, uint16_t* leaves_out)
{
    const node_t* nd = (const node_t*)nodes;
    size_t per_tree = ((size_t)1 << D) - 1;
    float s = (float)w / (float)ref_width;
    int n = pix ? npix : w * h;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        int p = pix ? pix[k] : k;
        int x = p % w, y = p / w;
        for (int t = 0; t < T; ++t) {
            int leaf = route(depth, rgb, w, h, x, y, nd + per_tree * t, D, s);
            leaves_out[(size_t)k * T + t] = leaf < 0 ? 0xFFFF : (uint16_t)leaf;
        }
    }
}

/* Back-projection x^C = D(u) K^-1 (u, v, 1)^T (Sec. 3.2.3), in FP64. */
static void backproject(float d, int x, int y, const float K[4], double out[3])
{
    out[0] = (double)d * (((double)x - (double)K[2]) / (double)K[0]);
    out[1] = (double)d * (((double)y - (double)K[3]) / (double)K[1]);
    out[2] = (double)d;
}

/* ------------------------------------------------------------------------ */
/*
 * Online adaptation (Sec. 3.2.2, steps 1-2): pixels on the 4-pixel grid
 * {(4i, 4j) : i, j >= 1} in raster order, x^W = H x^C (H camera->world),
 * stored float32 with the pixel's colour in the reservoir of the leaf reached
 * in each tree.  Reservoirs follow Vitter's Algorithm R (the paper's
 * reservoir sampling): the n-th arrival at a leaf fills slot n-1 while
 * n <= kappa, else replaces slot j = floor(u * n) if j < kappa, u drawn from
 * Philox with counter (RES, tree, leaf, n) and the stream key of (seed, 0).
 * Reservoir entry: float x, y, z and uint32 colour r | g<<8 | b<<16.
 * Returns the number of reservoir writes; dirty[t*L+leaf] is set on a write.
 * Parity: n <= kappa exact; n > kappa inclusion frequency kappa/n.
 */
EXPORT long oracle_adapt(const float* depth, const uint8_t* rgb, int w, int h, const float K[4],
                         const float H[16], const void* nodes, int T, int D, int ref_width,
                         int kappa, uint64_t seed, float* reservoir, uint32_t* seen,
                         uint8_t* dirty)
{
    const node_t* nd = (const node_t*)nodes;
    size_t per_tree = ((size_t)1 << D) - 1;
    size_t L = (size_t)1 << D;
    float s = (float)w / (float)ref_width;
    long writes = 0;
    for (int y = 4; y < h; y += 4) {
        for (int x = 4; x < w; x += 4) {
            float d = depth[(size_t)y * w + x];
            if (!depth_valid(d)) continue;
            double xc[3];
            backproject(d, x, y, K, xc);
            float xw[3];
            for (int a = 0; a < 3; ++a) {
                double v = (double)H[4 * a + 0] * xc[0] + (double)H[4 * a + 1] * xc[1];
                v = v + (double)H[4 * a + 2] * xc[2];
                v = v + (double)H[4 * a + 3];
                xw[a] = (float)v;
            }
            const uint8_t* c = rgb + ((size_t)y * w + x) * 3;
            uint32_t col = (uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16);
            for (int t = 0; t < T; ++t) {
                int leaf = route(depth, rgb, w, h, x, y, nd + per_tree * t, D, s);
                size_t tl = (size_t)t * L + (size_t)leaf;
                uint32_t n = ++seen[tl];
                long slot = -1;
                if (n <= (uint32_t)kappa) {
                    slot = (long)n - 1;
                } else {
                    uint32_t r[4], key[2];
                    stream_key(seed, 0, key);
                    philox_block(TAG_RES, 0, (uint32_t)t, (uint32_t)leaf, n, key, r);
                    uint32_t j = uniform_below(r[0], n);
                    if (j < (uint32_t)kappa) slot = (long)j;
                }
                if (slot >= 0) {
                    float* e = reservoir + (tl * (size_t)kappa + (size_t)slot) * 4;
                    e[0] = xw[0]; e[1] = xw[1]; e[2] = xw[2];
                    memcpy(&e[3], &col, 4);
                    dirty[tl] = 1;
                    ++writes;
                }
            }
        }
    }
    return writes;
}

/* ------------------------------------------------------------------------ */
/*
 * Mode finding in one leaf reservoir: Really Quick Shift (Fulkerson & Soatto
 * 2010), as the paper uses (Sec. 3.2.2 step 3, parameters in Table 8).
 *   density rho_k = sum_j exp(-|P_k - P_j|^2 / (2 sigma^2))   (sigma = clustererSigma)
 *   parent(k) = nearest j with (rho_j, j) > (rho_k, k) and |P_k - P_j| < tau
 *               (tau = clustererTau); none => k is a root
 *   clusters = trees of the parent forest; keep those with >= minClusterSize
 *   points, sorted by (size desc, root asc), at most maxClusterCount of them.
 * Per kept cluster: mean, population covariance, mean colour, and the inverse
 * of the covariance regularised by lambda * I.
 * Mode row (16 float32): mean xyz, size, inv-cov xx xy xz yy yz zz,
 * colour rgb, 0, 0, 0.  detail (optional, FP64, 16 per mode): mean[3],
 * cov xx xy xz yy yz zz, colour[3], size, root, 0, 0, 0.
 * Returns the number of modes.
 * Parity: separated blobs => one mode each with the blob's mean and
 * numpy.cov(bias=True) covariance; too-small clusters dropped; order by size.
 */
EXPORT int oracle_rqs_leaf(const float* entries, int n, double sigma, double tau_c,
                           int min_size, int max_modes, double lambda,
                           float* modes_out, double* detail)
{
    if (n <= 0) return 0;
    double* rho = (double*)calloc((size_t)n, sizeof(double));
    int* parent = (int*)malloc((size_t)n * sizeof(int));
    int* root = (int*)malloc((size_t)n * sizeof(int));
    int* size = (int*)calloc((size_t)n, sizeof(int));
    double two_s2 = 2.0 * sigma * sigma;
    double tau2 = tau_c * tau_c;
#define DIST2(a, b) ({ double _dx = (double)entries[4*(a)] - (double)entries[4*(b)];       \
                       double _dy = (double)entries[4*(a)+1] - (double)entries[4*(b)+1];   \
                       double _dz = (double)entries[4*(a)+2] - (double)entries[4*(b)+2];   \
                       _dx * _dx + _dy * _dy + _dz * _dz; })
    for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int j = 0; j < n; ++j) acc += exp(-DIST2(k, j) / two_s2);
        rho[k] = acc;
    }
    for (int k = 0; k < n; ++k) {
        int best = -1;
        double bestd = INFINITY;
        for (int j = 0; j < n; ++j) {
            int higher = rho[j] > rho[k] || (rho[j] == rho[k] && j > k);
            if (!higher) continue;
            double d2 = DIST2(k, j);
            if (d2 < tau2 && d2 < bestd) { bestd = d2; best = j; }
        }
        parent[k] = best;
    }
#undef DIST2
    for (int k = 0; k < n; ++k) {
        int r = k;
        while (parent[r] >= 0) r = parent[r];
        root[k] = r;
        size[r] += 1;
    }
    /* candidate roots, selection by (size desc, root asc) */
    int nm = 0;
    int* chosen = (int*)malloc((size_t)(max_modes > 0 ? max_modes : 1) * sizeof(int));
    for (int m = 0; m < max_modes; ++m) {
        int best = -1;
        for (int r = 0; r < n; ++r) {
            if (parent[r] >= 0 || size[r] < min_size) continue;
            int taken = 0;
            for (int q = 0; q < nm; ++q) taken |= (chosen[q] == r);
            if (taken) continue;
            if (best < 0 || size[r] > size[best]) best = r;   /* ties: lower root kept */
        }
        if (best < 0) break;
        chosen[nm++] = best;
    }
    for (int m = 0; m < nm; ++m) {
        int r = chosen[m];
        double cnt = 0, mu[3] = {0, 0, 0}, col[3] = {0, 0, 0};
        for (int k = 0; k < n; ++k) {
            if (root[k] != r) continue;
            cnt += 1.0;
            for (int a = 0; a < 3; ++a) mu[a] += (double)entries[4 * k + a];
            uint32_t c;
            memcpy(&c, &entries[4 * k + 3], 4);
            col[0] += (double)(c & 0xFF);
            col[1] += (double)((c >> 8) & 0xFF);
            col[2] += (double)((c >> 16) & 0xFF);
        }
        for (int a = 0; a < 3; ++a) { mu[a] /= cnt; col[a] /= cnt; }
        double S[6] = {0, 0, 0, 0, 0, 0};   /* xx xy xz yy yz zz */
        for (int k = 0; k < n; ++k) {
            if (root[k] != r) continue;
            double dx = (double)entries[4 * k] - mu[0];
            double dy = (double)entries[4 * k + 1] - mu[1];
            double dz = (double)entries[4 * k + 2] - mu[2];
            S[0] += dx * dx; S[1] += dx * dy; S[2] += dx * dz;
            S[3] += dy * dy; S[4] += dy * dz; S[5] += dz * dz;
        }
        for (int a = 0; a < 6; ++a) S[a] /= cnt;
        /* (S + lambda I)^-1 by the adjugate */
        double a_ = S[0] + lambda, b_ = S[1], c_ = S[2], d_ = S[3] + lambda, e_ = S[4], f_ = S[5] + lambda;
        double A = d_ * f_ - e_ * e_;
        double B = c_ * e_ - b_ * f_;
        double C = b_ * e_ - c_ * d_;
        double Dd = a_ * f_ - c_ * c_;
        double E = b_ * c_ - a_ * e_;
        double F = a_ * d_ - b_ * b_;
        double det = a_ * A + b_ * B + c_ * C;
        double inv[6] = {A / det, B / det, C / det, Dd / det, E / det, F / det};
        float* row = modes_out + (size_t)m * 16;
        row[0] = (float)mu[0]; row[1] = (float)mu[1]; row[2] = (float)mu[2];
        row[3] = (float)cnt;
        for (int a = 0; a < 6; ++a) row[4 + a] = (float)inv[a];
        row[10] = (float)col[0]; row[11] = (float)col[1]; row[12] = (float)col[2];
        row[13] = row[14] = row[15] = 0.0f;
        if (detail) {
            double* dd = detail + (size_t)m * 16;
            dd[0] = mu[0]; dd[1] = mu[1]; dd[2] = mu[2];
            for (int a = 0; a < 6; ++a) dd[3 + a] = S[a];
            dd[9] = col[0]; dd[10] = col[1]; dd[11] = col[2];
            dd[12] = cnt; dd[13] = (double)r; dd[14] = dd[15] = 0.0;
        }
    }
    free(chosen); free(rho); free(parent); free(root); free(size);
    return nm;
}

/* Re-cluster every dirty leaf of a room (all leaves if all != 0). */
EXPORT long oracle_update_modes(const float* reservoir, const uint32_t* seen, uint8_t* dirty,
                                int T, int D, int kappa, double sigma, double tau_c, int min_size,
                                int max_modes, double lambda, float* modes, uint8_t* nmodes, int all)
{
    size_t L = (size_t)1 << D;
    long done = 0;
    for (size_t tl = 0; tl < (size_t)T * L; ++tl) {
        if (!all && !dirty[tl]) continue;
        int n = seen[tl] < (uint32_t)kappa ? (int)seen[tl] : kappa;
        int nm = oracle_rqs_leaf(reservoir + tl * (size_t)kappa * 4, n, sigma, tau_c, min_size,
                                 max_modes, lambda, modes + tl * (size_t)max_modes * 16, NULL);
        nmodes[tl] = (uint8_t)nm;
        dirty[tl] = 0;
        ++done;
    }
    return done;
}

/*
 * Amortised mode update (Sec. 3.2.2): re-cluster `count` leaves in leaf-index
 * order starting at `first`, wrapping around the T * 2^D leaves of the
 * forest; dirty flags are not used or changed.  Returns the next first leaf.
 */
EXPORT long oracle_update_modes_range(const float* reservoir, const uint32_t* seen, int T, int D, int kappa,
                                      double sigma, double tau_c, int min_size, int max_modes, double lambda,
                                      float* modes, uint8_t* nmodes, long first, long count)
{
    const long n_leaves = (long)T << D;
    for (long i = 0; i < count; ++i) {
        const size_t tl = (size_t)((first + i) % n_leaves);
        int n = seen[tl] < (uint32_t)kappa ? (int)seen[tl] : kappa;
        nmodes[tl] = (uint8_t)oracle_rqs_leaf(reservoir + tl * (size_t)kappa * 4, n, sigma, tau_c, min_size,
                                              max_modes, lambda, modes + tl * (size_t)max_modes * 16, NULL);
    }
    return (first + count) % n_leaves;
}

/* ------------------------------------------------------------------------ */
/*
 * Singular value decomposition of a 3x3 matrix by one-sided (Hestenes)
 * Jacobi rotations: columns of G = A V are orthogonalised pairwise until no
 * pair has a relative inner product above 1e-15; then sigma_k = |g_k| and
 * u_k = g_k / sigma_k.  Singular values are returned in descending order; a
 * column with sigma = 0 is completed as the cross product of the others.
 * A is row-major; U, V column vectors are stored as columns (row-major).
 */
static void svd3(const double A[9], double U[9], double S[3], double V[9])
{
    double G[9];
    memcpy(G, A, sizeof(G));
    double W[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (int sweep = 0; sweep < 60; ++sweep) {
        int rotated = 0;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                double al = 0, be = 0, ga = 0;
                for (int i = 0; i < 3; ++i) {
                    al += G[3 * i + p] * G[3 * i + p];
                    be += G[3 * i + q] * G[3 * i + q];
                    ga += G[3 * i + p] * G[3 * i + q];
                }
                if (ga == 0.0 || fabs(ga) <= 1e-15 * sqrt(al * be)) continue;
                rotated = 1;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < 3; ++i) {
                    double gp = G[3 * i + p], gq = G[3 * i + q];
                    G[3 * i + p] = c * gp - s * gq;
                    G[3 * i + q] = s * gp + c * gq;
                    double wp = W[3 * i + p], wq = W[3 * i + q];
                    W[3 * i + p] = c * wp - s * wq;
                    W[3 * i + q] = s * wp + c * wq;
                }
            }
        }
        if (!rotated) break;
    }
    double sv[3];
    for (int k = 0; k < 3; ++k)
        sv[k] = sqrt(G[k] * G[k] + G[3 + k] * G[3 + k] + G[6 + k] * G[6 + k]);
    int ord[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (sv[ord[b]] > sv[ord[a]]) { int tmp = ord[a]; ord[a] = ord[b]; ord[b] = tmp; }
    for (int k = 0; k < 3; ++k) {
        int o = ord[k];
        S[k] = sv[o];
        for (int i = 0; i < 3; ++i) {
            V[3 * i + k] = W[3 * i + o];
            U[3 * i + k] = sv[o] > 0 ? G[3 * i + o] / sv[o] : 0.0;
        }
    }
    double tiny = 1e-300;
    for (int k = 0; k < 3; ++k) {
        if (S[k] > tiny && S[k] > 1e-13 * S[0]) continue;
        /* complete U's column k from the other two (only possible for k = 2,
           or k = 1 when the matrix has rank <= 1, which callers reject) */
        int a = (k + 1) % 3, b = (k + 2) % 3;
        double ua[3] = {U[a], U[3 + a], U[6 + a]}, ub[3] = {U[b], U[3 + b], U[6 + b]};
        double cr[3] = {ua[1] * ub[2] - ua[2] * ub[1], ua[2] * ub[0] - ua[0] * ub[2],
                        ua[0] * ub[1] - ua[1] * ub[0]};
        double nr = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        for (int i = 0; i < 3; ++i) U[3 * i + k] = nr > 0 ? cr[i] / nr : 0.0;
    }
}

static double det3(const double M[9])
{
    return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6])
         + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

/*
 * Kabsch (Kabsch 1976), used by the paper for pose hypotheses from 3 point
 * pairs (Sec. 3.2.3): with centroids c^C, c^W and A = sum (x^C - c^C)(x^W - c^W)^T
 * = U S V^T, R = V diag(1, 1, sign det(V U^T)) U^T and t = c^W - R c^C, so that
 * x^W ~ R x^C + t.  Returns 0 (degenerate) iff sigma_2 < 1e-4 sigma_1.
 * R row-major, sv = singular values (descending).
 * Parity: exact recovery of known transforms; R^T R = I, det R = +1;
 * least-squares optimality against perturbed rotations; collinear => 0.
 */
EXPORT int oracle_kabsch(const double* xc, const double* xw, int n, double R[9], double t[3],
                         double sv[3])
{
    double cc[3] = {0, 0, 0}, cw[3] = {0, 0, 0};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) { cc[a] += xc[3 * i + a]; cw[a] += xw[3 * i + a]; }
    for (int a = 0; a < 3; ++a) { cc[a] /= n; cw[a] /= n; }
    double A[9] = {0};
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                A[3 * a + b] += (xc[3 * i + a] - cc[a]) * (xw[3 * i + b] - cw[b]);
    double U[9], S[3], V[9];
    svd3(A, U, S, V);
    if (sv) { sv[0] = S[0]; sv[1] = S[1]; sv[2] = S[2]; }
    double VUt[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            VUt[3 * i + j] = V[3 * i + 0] * U[3 * j + 0] + V[3 * i + 1] * U[3 * j + 1]
                           + V[3 * i + 2] * U[3 * j + 2];
    double dsign = det3(VUt) < 0 ? -1.0 : 1.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[3 * i + j] = V[3 * i + 0] * U[3 * j + 0] + V[3 * i + 1] * U[3 * j + 1]
                         + dsign * V[3 * i + 2] * U[3 * j + 2];
    for (int a = 0; a < 3; ++a)
        t[a] = cw[a] - (R[3 * a] * cc[0] + R[3 * a + 1] * cc[1] + R[3 * a + 2] * cc[2]);
    if (!(S[0] > 0.0) || S[1] < 1e-4 * S[0]) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Per-frame view of a room for pose estimation. */
typedef struct {
    const float* depth; const uint8_t* rgb; int w, h; float K[4];
    const uint16_t* leaves;      /* [w*h][T], 0xFFFF = none */
    const uint8_t* nmodes;       /* [T*L] */
    const float* modes;          /* [T*L*M][16] */
    int T, D, M;
    const int32_t* eligible; int n_elig;
} view_t;

static int modes_of(const view_t* v, int pix)
{
    size_t L = (size_t)1 << v->D;
    int total = 0;
    for (int t = 0; t < v->T; ++t) {
        uint16_t lf = v->leaves[(size_t)pix * v->T + t];
        if (lf != 0xFFFF) total += v->nmodes[(size_t)t * L + lf];
    }
    return total;
}

/* m-th element of M(u): the tree-major concatenation of the leaves' modes */
static const float* mode_row(const view_t* v, int pix, int m)
{
    size_t L = (size_t)1 << v->D;
    for (int t = 0; t < v->T; ++t) {
        uint16_t lf = v->leaves[(size_t)pix * v->T + t];
        if (lf == 0xFFFF) continue;
        int cnt = v->nmodes[(size_t)t * L + lf];
        if (m < cnt) return v->modes + (((size_t)t * L + lf) * v->M + (size_t)m) * 16;
        m -= cnt;
    }
    return NULL;
}

/*
 * Pose hypothesis generation (Sec. 3.2.3).  Slot h tries iterations
 * it = 0, 1, ... < max_iters; iteration it draws two Philox blocks with
 * counters (HYP | blk, h, it, 0), blk = 0, 1, under the stream key of
 * (seed, request_seed).  Block 0 serves the pair the colour check looks at:
 * a0 picks that pair k* in {0, 1, 2}, a1 its pixel (uniform over the
 * raster-ordered eligible list) and a2 its mode (uniform over the tree-major
 * concatenation M(u)).  Block 1 serves the other two pairs in increasing
 * order: b0, b1 their pixels, b2, b3 their modes.  Checks, in the paper's
 * order: (1) L-infinity colour distance between pixel k* and its mode's
 * colour centroid must not exceed max_colour_linf (float32); (2) every
 * pairwise squared distance between the world points must be >=
 * min_sq_dist; (3) for every pair, | |x^C_a - x^C_b| - |x^W_a - x^W_b| | must not
 * exceed max_rigid; then Kabsch must not be degenerate.  The first passing
 * iteration is the slot's hypothesis; none => the slot is invalid.
 * Outputs per slot: valid, it, pix[3], mode[3] (index in M(u)), pose[12]
 * (R row-major then t, rounded to float32), pose64[12] (FP64).
 * Parity: triplets and iterations bit-exact, poses to 1e-5.
 */
EXPORT void oracle_hypotheses(const float* depth, const uint8_t* rgb, int w, int h, const float K[4],
                              const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                              int T, int D, int M, const int32_t* eligible, int n_elig,
                              int n_slots, int max_iters, float max_colour_linf,
                              double min_sq_dist, double max_rigid, uint64_t seed,
                              uint64_t request_seed, uint8_t* valid, int32_t* iter_out,
                              int32_t* pix_out, int32_t* mode_out, float* pose_out,
                              double* pose64_out)
{
    view_t v = {depth, rgb, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M,
                eligible, n_elig};
    uint32_t key[2];
    stream_key(seed, request_seed, key);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < n_slots; ++s) {
        valid[s] = 0;
        iter_out[s] = -1;
        if (n_elig <= 0) continue;
        for (int it = 0; it < max_iters; ++it) {
            uint32_t ra[4], rb[4];
            philox_block(TAG_HYP, 0, (uint32_t)s, (uint32_t)it, 0, key, ra);
            philox_block(TAG_HYP, 1, (uint32_t)s, (uint32_t)it, 0, key, rb);
            int kc = (int)uniform_below(ra[0], 3);
            uint32_t rpix[3], rmode[3];
            for (int k = 0, other = 0; k < 3; ++k) {
                if (k == kc) {
                    rpix[k] = ra[1];
                    rmode[k] = ra[2];
                } else {
                    rpix[k] = rb[other];
                    rmode[k] = rb[2 + other];
                    ++other;
                }
            }
            int pix[3], mi[3];
            const float* row[3];
            double xc[9], xw[9];
            for (int k = 0; k < 3; ++k) {
                pix[k] = eligible[uniform_below(rpix[k], (uint32_t)n_elig)];
                int nm = modes_of(&v, pix[k]);
                mi[k] = (int)uniform_below(rmode[k], (uint32_t)nm);
                row[k] = mode_row(&v, pix[k], mi[k]);
                backproject(depth[pix[k]], pix[k] % w, pix[k] / w, K, xc + 3 * k);
                for (int a = 0; a < 3; ++a) xw[3 * k + a] = (double)row[k][a];
            }
            /* check 1: colour of one randomly chosen pair */
            int ok = 1;
            for (int c = 0; c < 3; ++c) {
                float diff = fabsf((float)rgb[(size_t)pix[kc] * 3 + c] - row[kc][10 + c]);
                if (diff > max_colour_linf) ok = 0;
            }
            if (!ok) continue;
            /* check 2: scene points pairwise far enough apart */
            static const int PA[3] = {0, 0, 1}, PB[3] = {1, 2, 2};
            double dw2[3], dc2[3];
            for (int q = 0; q < 3; ++q) {
                const double* a = xw + 3 * PA[q];
                const double* b = xw + 3 * PB[q];
                double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
                dw2[q] = dx * dx + dy * dy + dz * dz;
                a = xc + 3 * PA[q];
                b = xc + 3 * PB[q];
                dx = a[0] - b[0]; dy = a[1] - b[1]; dz = a[2] - b[2];
                dc2[q] = dx * dx + dy * dy + dz * dz;
                if (dw2[q] < min_sq_dist) ok = 0;
            }
            if (!ok) continue;
            /* check 3: rigid enough */
            for (int q = 0; q < 3; ++q)
                if (fabs(sqrt(dc2[q]) - sqrt(dw2[q])) > max_rigid) ok = 0;
            if (!ok) continue;
            double R[9], t[3];
            if (!oracle_kabsch(xc, xw, 3, R, t, NULL)) continue;
            valid[s] = 1;
            iter_out[s] = it;
            for (int k = 0; k < 3; ++k) { pix_out[3 * s + k] = pix[k]; mode_out[3 * s + k] = mi[k]; }
            for (int a = 0; a < 9; ++a) {
                pose_out[12 * s + a] = (float)R[a];
                if (pose64_out) pose64_out[12 * s + a] = R[a];
            }
            for (int a = 0; a < 3; ++a) {
                pose_out[12 * s + 9 + a] = (float)t[a];
                if (pose64_out) pose64_out[12 * s + 9 + a] = t[a];
            }
            break;
        }
    }
}

/*
 * Per-pixel energy term of Eq. 5 (Sec. 3.2.3):
 *   e_i(H) = min over (mu, Sigma) in M(u_i) of | Sigma^-1/2 (H x_i - mu) |
 *          = sqrt(min_m d_m^T Sigma_m^-1 d_m), d_m = R x_i + t - mu_m,
 * with Sigma^-1 the stored regularised inverse; Euclidean |d_m| when the
 * covariance is not used.  Also returns the minimising mode (ties -> lower m).
 */
static double pixel_energy(const view_t* v, const double R[9], const double t[3], int pix,
                           int use_cov, int* argmin)
{
    double x[3];
    backproject(v->depth[pix], pix % v->w, pix / v->w, v->K, x);
    double y[3];
    for (int a = 0; a < 3; ++a)
        y[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2] + t[a];
    int nm = modes_of(v, pix);
    double best = INFINITY;
    int bi = -1;
    for (int m = 0; m < nm; ++m) {
        const float* row = mode_row(v, pix, m);
        double d0 = y[0] - (double)row[0], d1 = y[1] - (double)row[1], d2 = y[2] - (double)row[2];
        double q;
        if (use_cov) {
            double sxx = row[4], sxy = row[5], sxz = row[6], syy = row[7], syz = row[8], szz = row[9];
            q = d0 * (sxx * d0 + sxy * d1 + sxz * d2) + d1 * (sxy * d0 + syy * d1 + syz * d2)
              + d2 * (sxz * d0 + syz * d1 + szz * d2);
        } else {
            q = d0 * d0 + d1 * d1 + d2 * d2;
        }
        if (q < 0) q = 0;
        if (q < best) { best = q; bi = m; }
    }
    if (argmin) *argmin = bi;
    return sqrt(best);
}

EXPORT double oracle_pixel_energy(const float* depth, int w, int h, const float K[4],
                                  const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                                  int T, int D, int M, const float pose[12], int pix, int use_cov)
{
    view_t v = {depth, NULL, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M, NULL, 0};
    double R[9], t[3];
    for (int a = 0; a < 9; ++a) R[a] = pose[a];
    for (int a = 0; a < 3; ++a) t[a] = pose[9 + a];
    return pixel_energy(&v, R, t, pix, use_cov, NULL);
}

/*
 * Levenberg-Marquardt refinement of one pose in se(3) on the energy E of
 * Eq. 5 over a pixel set (Sec. 3.2.3, step (ii) of each preemptive-RANSAC
 * iteration).  The paper names the method and the parametrisation only;
 * the readings here:
 *  - the minimised function is E itself over the cumulative set I (with
 *    multiplicity), in the metric of Eq. 5 (Sigma^-1 when the covariance is
 *    used, else Euclidean);
 *  - update H <- exp(xi^) H with xi = (omega, v), acting on world points;
 *  - each iteration linearises at the current pose: per pixel its nearest
 *    mode m_i (ties to the lower m), r_i = H x_i - mu_{m_i}, e_i = |r_i|_A,
 *    the Jacobian J_i = [-[y_i]x | I] of exp(xi^) y_i at xi = 0 (y_i = H x_i),
 *    and the weight w_i = 1 / max(e_i, 1e-6), which makes
 *    sum_i w_i |r_i + J_i d|_A^2 / 2 share E's gradient at d = 0:
 *    N = sum_i w_i J_i^T A J_i, g = sum_i w_i J_i^T A r_i;
 *  - the step d solves (N + lambda diag(N)) d = -g by Cholesky (a
 *    non-positive or non-finite pivot rejects the step); the candidate
 *    exp(d^) H is accepted iff its energy (nearest modes chosen afresh) is
 *    lower; lambda starts at 1e-3, is divided by 10 on acceptance and
 *    multiplied by 10 on rejection;
 *  - a fixed number of iterations.
 * Returns the energy at the final pose; R, t are updated in place.
 */
static void se3_exp(const double xi[6], double Rd[9], double td[3])
{
    const double wx = xi[0], wy = xi[1], wz = xi[2];
    const double th2 = wx * wx + wy * wy + wz * wz;
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-2) {   /* Taylor series of sin(th)/th, (1-cos th)/th^2, (th-sin th)/th^3 to th^4 */
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        A = sin(th) / th;
        B = (1.0 - cos(th)) / th2;
        C = (1.0 - A) / th2;
    }
    const double W[9] = {0.0, -wz, wy, wz, 0.0, -wx, -wy, wx, 0.0};
    double W2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            W2[3 * i + j] = W[3 * i] * W[j] + W[3 * i + 1] * W[3 + j] + W[3 * i + 2] * W[6 + j];
    double V[9];
    for (int i = 0; i < 9; ++i) {
        const double id = (i % 4 == 0) ? 1.0 : 0.0;
        Rd[i] = id + A * W[i] + B * W2[i];
        V[i] = id + B * W[i] + C * W2[i];
    }
    for (int i = 0; i < 3; ++i) td[i] = V[3 * i] * xi[3] + V[3 * i + 1] * xi[4] + V[3 * i + 2] * xi[5];
}

/* E over I at (R, t); with N, g non-NULL also the weighted normal equations */
static double lm_linearise(const view_t* v, const int* I, int nI, int use_cov, const double R[9],
                           const double t[3], double N[36], double g[6])
{
    if (N) {
        for (int i = 0; i < 36; ++i) N[i] = 0.0;
        for (int i = 0; i < 6; ++i) g[i] = 0.0;
    }
    double E = 0.0;
    for (int k = 0; k < nI; ++k) {
        const int pix = I[k];
        int m = -1;
        const double e = pixel_energy(v, R, t, pix, use_cov, &m);
        E += e;
        if (!N || m < 0) continue;
        double x[3], y[3];
        backproject(v->depth[pix], pix % v->w, pix / v->w, v->K, x);
        for (int a = 0; a < 3; ++a)
            y[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2] + t[a];
        const float* row = mode_row(v, pix, m);
        const double r[3] = {y[0] - (double)row[0], y[1] - (double)row[1], y[2] - (double)row[2]};
        double A[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
        if (use_cov) {
            A[0] = row[4]; A[1] = row[5]; A[2] = row[6];
            A[3] = row[5]; A[4] = row[7]; A[5] = row[8];
            A[6] = row[6]; A[7] = row[8]; A[8] = row[9];
        }
        /* J = [-[y]x | I] */
        const double J[18] = {0.0, y[2], -y[1], 1.0, 0.0, 0.0,
                              -y[2], 0.0, y[0], 0.0, 1.0, 0.0,
                              y[1], -y[0], 0.0, 0.0, 0.0, 1.0};
        double AJ[18], Ar[3];
        for (int a = 0; a < 3; ++a) {
            Ar[a] = A[3 * a] * r[0] + A[3 * a + 1] * r[1] + A[3 * a + 2] * r[2];
            for (int j = 0; j < 6; ++j)
                AJ[6 * a + j] = A[3 * a] * J[j] + A[3 * a + 1] * J[6 + j] + A[3 * a + 2] * J[12 + j];
        }
        const double wgt = 1.0 / (e > 1e-6 ? e : 1e-6);
        for (int i = 0; i < 6; ++i) {
            g[i] += wgt * (J[i] * Ar[0] + J[6 + i] * Ar[1] + J[12 + i] * Ar[2]);
            for (int j = 0; j < 6; ++j)
                N[6 * i + j] += wgt * (J[i] * AJ[j] + J[6 + i] * AJ[6 + j] + J[12 + i] * AJ[12 + j]);
        }
    }
    return E;
}

/* solves M d = b for symmetric positive definite M (6x6); 0 when a pivot is
 * not positive and finite */
static int cholesky_solve6(const double M[36], const double b[6], double d[6])
{
    double L[36] = {0};
    for (int j = 0; j < 6; ++j) {
        double s = M[6 * j + j];
        for (int k = 0; k < j; ++k) s -= L[6 * j + k] * L[6 * j + k];
        if (!(s > 0.0) || !isfinite(s)) return 0;
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
    return 1;
}

static double lm_refine(const view_t* v, const int* I, int nI, int use_cov, int iters, double R[9], double t[3])
{
    double N[36], g[6];
    double E = lm_linearise(v, I, nI, use_cov, R, t, N, g);
    double lambda = 1e-3;
    for (int it = 0; it < iters; ++it) {
        double M[36], b[6], d[6];
        for (int i = 0; i < 36; ++i) M[i] = N[i];
        for (int i = 0; i < 6; ++i) {
            M[6 * i + i] = N[6 * i + i] + lambda * N[6 * i + i];
            b[i] = -g[i];
        }
        if (!cholesky_solve6(M, b, d)) {
            lambda *= 10.0;
            continue;
        }
        double Rd[9], td[3], Rc[9], tc[3];
        se3_exp(d, Rd, td);
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j)
                Rc[3 * i + j] = Rd[3 * i] * R[j] + Rd[3 * i + 1] * R[3 + j] + Rd[3 * i + 2] * R[6 + j];
            tc[i] = Rd[3 * i] * t[0] + Rd[3 * i + 1] * t[1] + Rd[3 * i + 2] * t[2] + td[i];
        }
        double Nc[36], gc[6];
        const double Ec = lm_linearise(v, I, nI, use_cov, Rc, tc, Nc, gc);
        if (Ec < E) {
            E = Ec;
            for (int i = 0; i < 9; ++i) R[i] = Rc[i];
            for (int i = 0; i < 3; ++i) t[i] = tc[i];
            for (int i = 0; i < 36; ++i) N[i] = Nc[i];
            for (int i = 0; i < 6; ++i) g[i] = gc[i];
            lambda /= 10.0;
        } else {
            lambda *= 10.0;
        }
    }
    return E;
}

EXPORT double oracle_lm_refine(const float* depth, int w, int h, const float K[4],
                               const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                               int T, int D, int M, const int32_t* I, int nI, int use_cov, int iters,
                               double pose[12])
{
    view_t v = {depth, NULL, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M, NULL, 0};
    return lm_refine(&v, I, nI, use_cov, iters, pose, pose + 9);
}

EXPORT void oracle_se3_exp(const double xi[6], double Rd[9], double td[3]) { se3_exp(xi, Rd, td); }

EXPORT double oracle_lm_linearise(const float* depth, int w, int h, const float K[4],
                                  const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                                  int T, int D, int M, const int32_t* I, int nI, int use_cov,
                                  const double pose[12], double N[36], double g[6])
{
    view_t v = {depth, NULL, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M, NULL, 0};
    return lm_linearise(&v, I, nI, use_cov, pose, pose + 9, N, g);
}

/*
 * Preemptive RANSAC (Sec. 3.2.3).  Hypotheses = the valid slots in slot order.  Every round draws eta pixels
 * from the eligible list (with replacement; round r, pixel k uses draw k%4
 * of the Philox block with counter (SCORE, r, k/4, 0) under the stream key of
 * (seed, request_seed)) and appends them to the
 * cumulative set I; each surviving hypothesis adds its Eq. 5 terms over the
 * new pixels to its energy.  If n_cull < #hypotheses the first round is the
 * initial cull to the n_cull lowest energies; every later round keeps the
 * ceil(n/2) lowest.  Rounds repeat while more than n_out hypotheses remain
 * (at least one round is always scored).  Order is (energy, slot) ascending.
 * With pose_update, every round after the first (the initial scoring or cull)
 * refines each survivor by lm_refine over the whole cumulative I, starting
 * from its pose so far (FP64, the float32 pose at first), and its energy
 * becomes E over the cumulative I at the refined pose; pose64_out (may be
 * NULL) receives every slot's final pose.
 * Outputs: survivors in final order (k = min(n, n_out) of them) with
 * energies; trace arrays (optional): I list, per-round survivor count.
 * Returns the number of rounds run (0 if there is no valid hypothesis).
 * Parity: energies 1e-4 relative; survivor sets equal up to near-ties.
 */
typedef struct { double e; int slot; } es_t;

static int es_cmp(const void* a, const void* b)
{
    const es_t* x = (const es_t*)a;
    const es_t* y = (const es_t*)b;
    if (x->e < y->e) return -1;
    if (x->e > y->e) return 1;
    return (x->slot > y->slot) - (x->slot < y->slot);
}

EXPORT int oracle_ransac(const float* depth, int w, int h, const float K[4],
                         const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                         int T, int D, int M, const int32_t* eligible, int n_elig,
                         const uint8_t* valid, const float* poses, int n_slots,
                         int eta, int n_cull, int n_out, int use_cov,
                         uint64_t seed, uint64_t request_seed,
                         int32_t* out_slots, double* out_energy, int32_t* out_count,
                         int32_t* I_out, int I_cap, int32_t* round_n, int round_cap,
                         int32_t* round_slots, double* round_energy, int pose_update,
                         int lm_iterations, double* pose64_out)
{
    view_t v = {depth, NULL, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M,
                eligible, n_elig};
    es_t* hs = (es_t*)malloc((size_t)(n_slots > 0 ? n_slots : 1) * sizeof(es_t));
    double* P64 = (double*)malloc((size_t)(n_slots > 0 ? n_slots : 1) * 12 * sizeof(double));
    for (size_t i = 0; i < (size_t)n_slots * 12; ++i) P64[i] = (double)poses[i];
    int* Iall = NULL;
    int n = 0;
    for (int s = 0; s < n_slots; ++s)
        if (valid[s]) { hs[n].e = 0.0; hs[n].slot = s; ++n; }
    *out_count = 0;
    if (n == 0 || n_elig <= 0) {
        if (pose64_out) memcpy(pose64_out, P64, (size_t)n_slots * 12 * sizeof(double));
        free(hs);
        free(P64);
        return 0;
    }
    int round = 0, nI = 0;
    int first = 1;
    uint32_t key[2];
    stream_key(seed, request_seed, key);
    while (first || n > n_out) {
        int* newpix = (int*)malloc((size_t)eta * sizeof(int));
        for (int k = 0; k < eta; ++k) {
            uint32_t r[4];
            philox_block(TAG_SCORE, 0, (uint32_t)round, (uint32_t)(k / 4), 0, key, r);
            newpix[k] = eligible[uniform_below(r[k % 4], (uint32_t)n_elig)];
            if (I_out && nI < I_cap) I_out[nI] = newpix[k];
            Iall = (int*)realloc(Iall, (size_t)(nI + 1) * sizeof(int));
            Iall[nI] = newpix[k];
            ++nI;
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) {
            double* P = P64 + 12 * (size_t)hs[i].slot;
            if (pose_update && !first) {
                hs[i].e = lm_refine(&v, Iall, nI, use_cov, lm_iterations, P, P + 9);
                continue;
            }
            double acc = 0.0;
            for (int k = 0; k < eta; ++k) acc += pixel_energy(&v, P, P + 9, newpix[k], use_cov, NULL);
            hs[i].e += acc;
        }
        free(newpix);
        qsort(hs, (size_t)n, sizeof(es_t), es_cmp);
        int keep = n;
        if (first && n_cull < n) keep = n_cull;
        else if (n > n_out) keep = (n + 1) / 2;
        n = keep;
        if (round_n && round < round_cap) {
            round_n[round] = n;
            if (round_slots)
                for (int i = 0; i < n; ++i) {
                    round_slots[(size_t)round * n_slots + i] = hs[i].slot;
                    round_energy[(size_t)round * n_slots + i] = hs[i].e;
                }
        }
        ++round;
        first = 0;
    }
    int k = n < n_out ? n : n_out;
    for (int i = 0; i < k; ++i) { out_slots[i] = hs[i].slot; out_energy[i] = hs[i].e; }
    *out_count = k;
    if (pose64_out) memcpy(pose64_out, P64, (size_t)n_slots * 12 * sizeof(double));
    free(hs);
    free(P64);
    free(Iall);
    return round;
}

/*
 * Final refit over the inliers (a reading for the full-size workload's "final
 * pose refinement over the inliers"; the paper instead optimises with LM):
 * for every pixel of I (with multiplicity), the mode minimising the Eq. 5
 * distance under the winner's pose; the pixel is an inlier iff the Euclidean
 * residual to that mode is <= inlier_threshold.  With >= 3 inliers the pose
 * is replaced by the Kabsch fit over all inlier pairs (x^C, mu), unless that
 * fit is degenerate.  Returns the inlier count; pose_out (FP64 R row-major,
 * t) is the input pose when not refitted.
 * Parity: noise-free correspondences => refit equals the true pose.
 */
EXPORT int oracle_refine(const float* depth, int w, int h, const float K[4],
                         const uint16_t* leaves, const uint8_t* nmodes, const float* modes,
                         int T, int D, int M, const float pose_in[12], const int32_t* I, int nI,
                         double inlier_threshold, int use_cov, double pose_out[12], int* refitted)
{
    view_t v = {depth, NULL, w, h, {K[0], K[1], K[2], K[3]}, leaves, nmodes, modes, T, D, M, NULL, 0};
    double R[9], t[3];
    for (int a = 0; a < 9; ++a) R[a] = pose_in[a];
    for (int a = 0; a < 3; ++a) t[a] = pose_in[9 + a];
    double* xc = (double*)malloc((size_t)(nI > 0 ? nI : 1) * 3 * sizeof(double));
    double* xw = (double*)malloc((size_t)(nI > 0 ? nI : 1) * 3 * sizeof(double));
    int ni = 0;
    for (int k = 0; k < nI; ++k) {
        int pix = I[k], am = -1;
        pixel_energy(&v, R, t, pix, use_cov, &am);
        if (am < 0) continue;
        const float* row = mode_row(&v, pix, am);
        double x[3], y[3];
        backproject(depth[pix], pix % w, pix / w, K, x);
        for (int a = 0; a < 3; ++a)
            y[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2] + t[a];
        double d0 = y[0] - (double)row[0], d1 = y[1] - (double)row[1], d2 = y[2] - (double)row[2];
        if (sqrt(d0 * d0 + d1 * d1 + d2 * d2) <= inlier_threshold) {
            for (int a = 0; a < 3; ++a) { xc[3 * ni + a] = x[a]; xw[3 * ni + a] = (double)row[a]; }
            ++ni;
        }
    }
    for (int a = 0; a < 9; ++a) pose_out[a] = R[a];
    for (int a = 0; a < 3; ++a) pose_out[9 + a] = t[a];
    *refitted = 0;
    if (ni >= 3) {
        double R2[9], t2[3];
        if (oracle_kabsch(xc, xw, ni, R2, t2, NULL)) {
            for (int a = 0; a < 9; ++a) pose_out[a] = R2[a];
            for (int a = 0; a < 3; ++a) pose_out[9 + a] = t2[a];
            *refitted = 1;
        }
    }
    free(xc); free(xw);
    return ni;
}

/* ------------------------------------------------------------------------ */
/*
 * Model-based score of a pose (the analogue, on an analytic scene model, of
 * the paper's depth-raycast comparison used to rank the final hypotheses and
 * to decide cascade fallbacks, Sec. 3.2.4-3.2.5): the mean, over pixels with
 * valid depth, of the distance from H x^C(u) to the nearest scene surface.
 * Surface record (16 floats): point p0 (3), unit normal n (3), in-plane axes
 * e1, e2 (3 + 3), half-extents a, b (2; a <= 0 marks an infinite plane),
 * 0, 0.  Distance to an infinite plane: |n . (y - p0)|; to a rectangle:
 * sqrt(c^2 + max(|a'| - a, 0)^2 + max(|b'| - b, 0)^2) with (a', b', c) the
 * coordinates of y - p0 on (e1, e2, n).
 * Parity: noise-free frame at its true pose => score 0 (up to float32 depth).
 */
EXPORT void oracle_plane_scores(const float* depth, int w, int h, const float K[4], const float* poses,
                                int n_poses, const float* surfaces, int n_surf, double* scores)
{
    for (int k = 0; k < n_poses; ++k) {
        const float* P = poses + 12 * (size_t)k;
        double R[9], t[3];
        for (int a = 0; a < 9; ++a) R[a] = P[a];
        for (int a = 0; a < 3; ++a) t[a] = P[9 + a];
        double acc = 0.0;
        long cnt = 0;
        for (int p = 0; p < w * h; ++p) {
            float d = depth[p];
            if (!depth_valid(d)) continue;
            double x[3], y[3];
            backproject(d, p % w, p / w, K, x);
            for (int a = 0; a < 3; ++a)
                y[a] = R[3 * a] * x[0] + R[3 * a + 1] * x[1] + R[3 * a + 2] * x[2] + t[a];
            double best = INFINITY;
            for (int s = 0; s < n_surf; ++s) {
                const float* S = surfaces + 16 * (size_t)s;
                double r0 = y[0] - S[0], r1 = y[1] - S[1], r2 = y[2] - S[2];
                double c = r0 * S[3] + r1 * S[4] + r2 * S[5];
                double dist;
                if (S[12] <= 0.0f) {
                    dist = fabs(c);
                } else {
                    double a = r0 * S[6] + r1 * S[7] + r2 * S[8];
                    double b = r0 * S[9] + r1 * S[10] + r2 * S[11];
                    double da = fabs(a) - S[12], db = fabs(b) - S[13];
                    if (da < 0) da = 0;
                    if (db < 0) db = 0;
                    dist = sqrt(c * c + da * da + db * db);
                }
                if (dist < best) best = dist;
            }
            acc += best;
            ++cnt;
        }
        scores[k] = cnt > 0 ? acc / (double)cnt : INFINITY;
    }
}

/* ------------------------------------------------------------------------ */
/*
 * Model-based hypothesis score, Sec. 3.2.4, Eq. 6-7, with the scene model
 * given analytically (the surface records of oracle_plane_scores).
 *
 * Synthetic depth raycast D~_xi from pose xi = (R, t), camera -> world: pixel
 * u = (x, y) on integer coordinates casts the camera ray
 * d^C = ((x - cx) / fx, (y - cy) / fy, 1) from o = t along d^W = R d^C; a
 * surface is hit at ray parameter z = ((p0 - o) . n) / (n . d^W) when
 * n . d^W != 0, z > 0 and, for a rectangle, |e1 . q| <= a and |e2 . q| <= b
 * with q = o + z d^W - p0.  D~(u) is the smallest hit z, which is the
 * camera-space depth because d^C has unit z.  Readings: D~(u) is valid when
 * some surface is hit at min_depth <= z <= max_depth (max_depth <= 0: no
 * upper limit), the stand-in for the range the model is rendered over; a
 * live depth is valid when positive and finite.
 *
 * mu(xi) (Eq. 6) = sum over pixels valid in both of |D_l(u) - D~(u)|,
 * divided by their number; s(xi) (Eq. 7) = mu(xi) when the valid fraction of
 * the raycast is at least 0.1, taken exactly as 10 * |valid| >= w * h, and
 * +inf otherwise, and also +inf when no pixel is valid in both.
 * Outputs per pose: scores[k] = s, mu[k] (NaN when no pixel is valid in
 * both), counts[2k] = |valid raycast pixels|, counts[2k+1] = |both valid|.
 * All arithmetic FP64 from the float32 inputs.
 */
static double raycast_depth(double ox, double oy, double oz, double dx, double dy, double dz,
                            const float* surfaces, int n_surf)
{
    double best = INFINITY;
    for (int s = 0; s < n_surf; ++s) {
        const float* S = surfaces + 16 * (size_t)s;
        const double nx = S[3], ny = S[4], nz = S[5];
        const double den = dx * nx + dy * ny + dz * nz;
        if (den == 0.0) continue;
        const double num = ((double)S[0] - ox) * nx + ((double)S[1] - oy) * ny + ((double)S[2] - oz) * nz;
        const double z = num / den;
        if (!(z > 0.0)) continue;
        if (S[12] > 0.0f) {
            const double qx = (ox + z * dx) - (double)S[0];
            const double qy = (oy + z * dy) - (double)S[1];
            const double qz = (oz + z * dz) - (double)S[2];
            const double a = qx * (double)S[6] + qy * (double)S[7] + qz * (double)S[8];
            const double b = qx * (double)S[9] + qy * (double)S[10] + qz * (double)S[11];
            if (!(fabs(a) <= (double)S[12] && fabs(b) <= (double)S[13])) continue;
        }
        if (z < best) best = z;
    }
    return best;
}

EXPORT void oracle_depth_scores(const float* depth, int w, int h, const float K[4], const float* poses,
                                int n_poses, const float* surfaces, int n_surf, float min_depth,
                                float max_depth, double* scores, double* mu, long long* counts)
{
    for (int k = 0; k < n_poses; ++k) {
        const float* P = poses + 12 * (size_t)k;
        double acc = 0.0;
        long long n_model = 0, n_both = 0;
        for (int p = 0; p < w * h; ++p) {
            const int x = p % w, y = p / w;
            const double cx = ((double)x - (double)K[2]) / (double)K[0];
            const double cy = ((double)y - (double)K[3]) / (double)K[1];
            const double dx = (double)P[0] * cx + (double)P[1] * cy + (double)P[2];
            const double dy = (double)P[3] * cx + (double)P[4] * cy + (double)P[5];
            const double dz = (double)P[6] * cx + (double)P[7] * cy + (double)P[8];
            const double z = raycast_depth(P[9], P[10], P[11], dx, dy, dz, surfaces, n_surf);
            if (!(z >= (double)min_depth && (max_depth <= 0.0f || z <= (double)max_depth))) continue;
            ++n_model;
            const float d = depth[p];
            if (!depth_valid(d)) continue;
            acc += fabs((double)d - z);
            ++n_both;
        }
        counts[2 * k] = n_model;
        counts[2 * k + 1] = n_both;
        mu[k] = n_both > 0 ? acc / (double)n_both : NAN;
        scores[k] = (n_both > 0 && 10 * n_model >= (long long)w * h) ? mu[k] : INFINITY;
    }
}
