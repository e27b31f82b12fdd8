// rl_rank_kernels.hip -- model-based hypothesis ranking (Sec. 3.2.4, Eq. 6-8)
// on an analytic scene model (gfx950, wave64).
//
//   k_depth_partial  per (1024-pixel tile, pose): synthetic depth raycast of
//                    the surfaces from the pose, compared with the live
//                    depth; per-tile sum of |D_l - D~| and the two counts
//   k_depth_final    per pose (one block): tile sums -> mu (Eq. 6), s (Eq. 7)
//
// The raycast's hit tests decide the counts, so they are evaluated in FP64
// with no contraction, in a fixed operation order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "rl_internal.hpp"

namespace rl {

constexpr int kRankTile = 1024;        // pixels per block (4 per thread)

// Smallest positive ray parameter at which the ray o + z d meets a surface
// (an infinite plane, or a rectangle: |e1 . q| <= a, |e2 . q| <= b for
// q = o + z d - p0); +inf when none.  Surface records: 16 floats each.
__device__ __forceinline__ double raycast_depth(const float* __restrict__ S0, int n_surf, double ox, double oy,
                                                double oz, double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    double best = INFINITY;
    for (int s = 0; s < n_surf; ++s) {
        const float* S = S0 + 16 * s;
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
        best = z < best ? z : best;
    }
    return best;
}

// grid (tiles, poses), 256 threads; partial[tile * 64 + pose],
// cnt[(tile * 64 + pose) * 2 + {0: valid raycast, 1: valid in both}]
__global__ __launch_bounds__(256) void k_depth_partial(FrameView src, int w, int h, float fx,
                                                       float fy, float cx, float cy,
                                                       const float* __restrict__ surfaces, int n_surf,
                                                       const float* __restrict__ poses, float zmin, float zmax,
                                                       double* __restrict__ partial, int* __restrict__ cnt)
{
#pragma clang fp contract(off)
    __shared__ float s_surf[kMaxModelSurfaces * 16];
    __shared__ double s_acc[256];
    __shared__ int s_nm[256], s_nb[256];
    const int tile = blockIdx.x, pose = blockIdx.y;
    for (int i = threadIdx.x; i < n_surf * 16; i += 256) s_surf[i] = surfaces[i];
    const float* P = poses + 12 * pose;
    const double R0 = P[0], R1 = P[1], R2 = P[2], R3 = P[3], R4 = P[4], R5 = P[5], R6 = P[6], R7 = P[7],
                 R8 = P[8], ox = P[9], oy = P[10], oz = P[11];
    __syncthreads();
    const int np = w * h;
    double acc = 0.0;
    int nm = 0, nb = 0;
    for (int k = 0; k < kRankTile / 256; ++k) {
        const int p = tile * kRankTile + k * 256 + (int)threadIdx.x;
        if (p >= np) break;
        const int x = p % w, y = p / w;
        const double ux = ((double)x - (double)cx) / (double)fx;
        const double uy = ((double)y - (double)cy) / (double)fy;
        const double dx = R0 * ux + R1 * uy + R2;
        const double dy = R3 * ux + R4 * uy + R5;
        const double dz = R6 * ux + R7 * uy + R8;
        const double z = raycast_depth(s_surf, n_surf, ox, oy, oz, dx, dy, dz);
        if (!(z >= (double)zmin && (zmax <= 0.0f || z <= (double)zmax))) continue;
        ++nm;
        const float d = src.d(x, y);
        if (!depth_ok(d)) continue;
        acc += fabs((double)d - z);
        ++nb;
    }
    s_acc[threadIdx.x] = acc;
    s_nm[threadIdx.x] = nm;
    s_nb[threadIdx.x] = nb;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if ((int)threadIdx.x < stride) {
            s_acc[threadIdx.x] += s_acc[threadIdx.x + stride];
            s_nm[threadIdx.x] += s_nm[threadIdx.x + stride];
            s_nb[threadIdx.x] += s_nb[threadIdx.x + stride];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const size_t o = (size_t)tile * kMaxModelPoses + pose;
        partial[o] = s_acc[0];
        cnt[2 * o] = s_nm[0];
        cnt[2 * o + 1] = s_nb[0];
    }
}

// one block per pose: thread i adds tiles i, i + 256, ... in order, then a
// fixed tree over the threads (every tile's partial is read by a single
// load, not by a pose's chain of dependent batches).  out[2 * pose] = s,
// out[2 * pose + 1] = mu (NaN when no pixel is valid in both);
// counts[2 * pose + {0, 1}]
__global__ __launch_bounds__(256) void k_depth_final(const double* __restrict__ partial,
                                                     const int* __restrict__ cnt, int ntiles, long long np,
                                                     double* __restrict__ out, long long* __restrict__ counts)
{
    __shared__ double s_acc[256];
    __shared__ long long s_nm[256], s_nb[256];
    const int pose = blockIdx.x, i = threadIdx.x;
    double acc = 0.0;
    long long nm = 0, nb = 0;
    for (int t = i; t < ntiles; t += 256) {
        const size_t o = (size_t)t * kMaxModelPoses + pose;
        acc += partial[o];
        nm += cnt[2 * o];
        nb += cnt[2 * o + 1];
    }
    s_acc[i] = acc;
    s_nm[i] = nm;
    s_nb[i] = nb;
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (i < stride) {
            s_acc[i] += s_acc[i + stride];
            s_nm[i] += s_nm[i + stride];
            s_nb[i] += s_nb[i + stride];
        }
        __syncthreads();
    }
    if (i == 0) {
        const double mu = s_nb[0] > 0 ? s_acc[0] / (double)s_nb[0] : NAN;
        out[2 * pose] = (s_nb[0] > 0 && 10 * s_nm[0] >= np) ? mu : INFINITY;
        out[2 * pose + 1] = mu;
        counts[2 * pose] = s_nm[0];
        counts[2 * pose + 1] = s_nb[0];
    }
}

hipError_t launch_depth_scores(const FrameView& src, int w, int h, float fx, float fy, float cx, float cy,
                               const float* surfaces, int n_surf, const float* poses, int n_poses, float zmin,
                               float zmax, double* partial, int* cnt, double* out, long long* counts,
                               hipStream_t st)
{
    if (n_surf < 1 || n_surf > kMaxModelSurfaces || n_poses < 1 || n_poses > kMaxModelPoses)
        return hipErrorInvalidValue;
    const int ntiles = (w * h + kRankTile - 1) / kRankTile;
    k_depth_partial<<<dim3(ntiles, n_poses), dim3(256), 0, st>>>(src, w, h, fx, fy, cx, cy, surfaces, n_surf,
                                                                  poses, zmin, zmax, partial, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_depth_final<<<dim3(n_poses), dim3(256), 0, st>>>(partial, cnt, ntiles, (long long)w * h, out, counts);
    return hipGetLastError();
}

}  // namespace rl
