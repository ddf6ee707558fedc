// Differentiable form of the tracking energy over keyframes.
//
// Loss of keyframe i (Sec. 4.1 Eq. (5) with the Huber penalty of Sec. 5.1):
//   L_i = sum_k rho_delta(r_ik),  r = psi_j + gh_j . (q - v_j),
//   q = T_i x_k,  T_i = exp(xi_i^) T0_i,  j = nearest voxel of q (Eq. (14)),
// gh_j = g_j / |g_j|.  Per-voxel parameters are {psi_j, g_j} (float4 in the
// map's slot order, voxel c of a block at its Morton index); the map's W
// only marks a voxel as observed.
//
// The adjoint recomputes every residual from the depth and the pose (no
// per-pixel Jacobian is stored):
//   dL/dpsi_j += sum_k s rho'(r_k),
//   dL/dg_j   += (I - gh gh^T) / |g_j| sum_k s rho'(r_k) (q_k - v_j),
//   dL/dxi_i   = Jl(xi_i)^T sum_k s rho'(r_ik) [gh; q x gh],
// with s the upstream gradient of L_i and k over the pixels whose voxel is j
// (the projection (I - gh gh^T) / |g_j| is the same for every pixel of a
// voxel, so it is applied once to the voxel's sum).
//
// The loss is a pixel-parallel pass.  The adjoint gathers instead of
// scattering: one work-group owns a map block, finds for every keyframe the
// pixels whose point can fall in one of the block's voxel cells (the
// block's box projected into the keyframe, and its depth range) and adds
// their terms into the block's 512 voxel sums in LDS, then writes each
// voxel once.  No two work-groups write the same voxel, so nothing is added
// to global memory atomically, and the voxel sums are 64-bit fixed point
// (an integer sum does not depend on the order of its terms), so the
// gradients are the same bits on every run.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "gsdf.h"
#include "gsdf_common.hpp"
#include "gsdf_fixed.hpp"
#include "gsdf_host.hpp"
#include "gsdf_se3.hpp"

namespace gsdf {

constexpr int kAdjBlock = 256;
constexpr int kAdjPart = 8;         // doubles per work-group partial: loss, 6 pose sums, count
constexpr int kAdjMaxGroups = 512;  // work-groups per keyframe of the loss pass
constexpr int kAdjTile = 32;        // the loss pass takes 32x32 pixel tiles, four pixels a thread
constexpr int kBackGroups = 8192;   // work-groups of the adjoint (each owns every 8192th block)
constexpr int kAdjBatch = 4;        // pixels a thread of the adjoint takes at a time

struct AdjArgs {
    int32_t W, H, groups, freeze;
    double fx, fy, ifx, ify, cx, cy;
    float zmin, zmax, delta, pad;
    double vs, inv_vs;
    int64_t param_blocks;   // rows of the parameter buffer (slots beyond are unobserved)
};

// Scratch of the keyframe calls: per-work-group partials, the keyframe
// poses exp(xi^) T0, and (frozen association) how far each keyframe's
// points lie outside their frozen voxels' cells.
struct AdjScratch {
    size_t partials, poses, reach, slots, total;
};

inline AdjScratch adj_scratch(int32_t K, int64_t npx) {
    AdjScratch L;
    size_t o = 0;
    const int g = kAdjMaxGroups > kBackGroups ? kAdjMaxGroups : kBackGroups;
    L.partials = o; o = align256(o + (size_t)K * g * kAdjPart * sizeof(double));
    L.poses = o;    o = align256(o + (size_t)K * 12 * sizeof(double));
    L.reach = o;    o = align256(o + (size_t)K * sizeof(double));
    L.slots = o;    o = align256(o + (size_t)K * npx * sizeof(int32_t));
    L.total = o;
    return L;
}

// World point q = R x + t of pixel (u, v) with depth D, x = D [(u-cx)/fx,
// (v-cy)/fy, 1], in float64 with every multiply-add written out, so that
// the loss pass and the adjoint form the same bits.
__device__ inline void pixel_point(const AdjArgs& a, const double R[9], const double t[3], float D, int u, int v,
                                   double q[3]) {
    const double Dd = (double)D;
    const double x0 = Dd * (((double)u - a.cx) * a.ifx);
    const double x1 = Dd * (((double)v - a.cy) * a.ify);
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = fma(R[3 * r], x0, fma(R[3 * r + 1], x1, fma(R[3 * r + 2], Dd, t[r])));
}

__device__ inline void nearest_voxel(const AdjArgs& a, const double q[3], int m[3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r) m[r] = (int)floor(q[r] * a.inv_vs + 0.5);
}

// Voxel, offset and parameters of one pixel; false when it has no usable
// voxel (invalid depth, block absent, W = 0 or g = 0).
struct PixelTerm {
    int64_t vi;
    float psi, gh[3], inv_ng, dq[3], q[3];
};

// The parameters of voxel vi and the pixel's offsets from voxel m (false
// when the voxel is unobserved or has g = 0).
__device__ inline bool param_term(const float4 p, const AdjArgs& a, int64_t vi, const double q[3], const int m[3],
                                  PixelTerm* P) {
    const float n2 = p.y * p.y + p.z * p.z + p.w * p.w;
    if (!(n2 > 0.0f)) return false;
    P->vi = vi;
    P->inv_ng = 1.0f / sqrtf(n2);
    P->psi = p.x;
    P->gh[0] = p.y * P->inv_ng;
    P->gh[1] = p.z * P->inv_ng;
    P->gh[2] = p.w * P->inv_ng;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        P->dq[r] = (float)(q[r] - a.vs * (double)m[r]);
        P->q[r] = (float)q[r];
    }
    return true;
}

__device__ inline bool voxel_term(const MapView& M, const AdjArgs& a, const float4* __restrict__ params, int64_t vi,
                                  const double q[3], const int m[3], PixelTerm* P) {
    if (!(M.weight[vi] > 0.0f)) return false;
    return param_term(params[vi], a, vi, q, m, P);
}

__device__ inline bool pixel_term(const MapView& M, const AdjArgs& a, const double R[9], const double t[3],
                                  const float4* __restrict__ params, float D, int u, int v,
                                  int32_t* __restrict__ as, PixelTerm* P) {
    if (!depth_ok(D, a.zmin, a.zmax)) {
        if (as && !a.freeze) as[0] = as[1] = as[2] = INT_MIN;
        return false;
    }
    double q[3];
    int m[3];
    pixel_point(a, R, t, D, u, v, q);
    nearest_voxel(a, q, m);
    if (as && a.freeze) {
        if (as[0] == INT_MIN) return false;
        m[0] = as[0];
        m[1] = as[1];
        m[2] = as[2];
    }
    bool ok = false;
    const int32_t slot = hash_find(M, block_of(m[0]), block_of(m[1]), block_of(m[2]));
    if (slot >= 0 && (int64_t)slot < a.param_blocks)
        ok = voxel_term(M, a, params, (int64_t)slot * kBlockVoxels + morton9(m[0] & 7, m[1] & 7, m[2] & 7), q, m, P);
    if (as && !a.freeze) {
        as[0] = ok ? m[0] : INT_MIN;
        as[1] = ok ? m[1] : INT_MIN;
        as[2] = ok ? m[2] : INT_MIN;
    }
    return ok;
}

// Residual terms of one pixel: Huber loss, s rho'(r) and the Jacobian row
// [gh; q x gh] of a left increment of the keyframe pose.
struct ResidualTerms {
    float rho, rp, J[6];
};

__device__ inline ResidualTerms residual_terms(const PixelTerm& P, float delta, float s) {
    ResidualTerms o;
    const float r = P.psi + P.gh[0] * P.dq[0] + P.gh[1] * P.dq[1] + P.gh[2] * P.dq[2];
    const float ar = fabsf(r);
    const bool quad = ar <= delta;
    o.rho = quad ? 0.5f * r * r : delta * (ar - 0.5f * delta);
    o.rp = s * (quad ? r : copysignf(delta, r));   // s rho'(r)
    o.J[0] = P.gh[0];
    o.J[1] = P.gh[1];
    o.J[2] = P.gh[2];
    o.J[3] = P.q[1] * P.gh[2] - P.q[2] * P.gh[1];
    o.J[4] = P.q[2] * P.gh[0] - P.q[0] * P.gh[2];
    o.J[5] = P.q[0] * P.gh[1] - P.q[1] * P.gh[0];
    return o;
}

// Work-group sum of kAdjPart float values per thread, in float64 (wave
// shuffles, then one value per wave in a fixed order); the totals land in
// out[] of threads 0 .. kAdjPart-1 (out[k] in thread k).
__device__ inline double block_sum_part(const float acc[kAdjPart], double (*s_red)[kAdjBlock / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) {
        double x = (double)acc[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) s_red[k][wave] = x;
    }
    __syncthreads();
    double x = 0.0;
    if (threadIdx.x < kAdjPart)
        for (int w = 0; w < kAdjBlock / 64; ++w) x += s_red[threadIdx.x][w];
    __syncthreads();
    return x;
}

// The loss pass.  Grid (groups, K): a work-group takes 32x32 pixel tiles of
// keyframe blockIdx.y and writes its partial sums (loss, the six pose sums
// unused here, the count of pixels used); with an association buffer and
// freeze = 0 it records each pixel's voxel.
__global__ __launch_bounds__(kAdjBlock) void k_keyframe_loss(MapView M, AdjArgs a, const float* __restrict__ depth,
                                                             const double* __restrict__ poses,
                                                             const float4* __restrict__ params,
                                                             int32_t* __restrict__ assoc,
                                                             double* __restrict__ partials) {
    __shared__ double s_red[kAdjPart][kAdjBlock / 64];
    const int kf = blockIdx.y;
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = poses[12 * kf + 4 * i + j];
        t[i] = poses[12 * kf + 4 * i + 3];
    }
    const int N = a.W * a.H;
    const float* dimg = depth + (size_t)kf * N;
    int32_t* aimg = assoc ? assoc + (size_t)kf * N * 3 : nullptr;
    float acc[kAdjPart];
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) acc[k] = 0.0f;
    const int tiles_x = (a.W + kAdjTile - 1) / kAdjTile;
    const int ntiles = tiles_x * ((a.H + kAdjTile - 1) / kAdjTile);
    for (int tile = blockIdx.x; tile < ntiles; tile += a.groups) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        for (int px = threadIdx.x; px < kAdjTile * kAdjTile; px += kAdjBlock) {
            const int u = tx * kAdjTile + (px % kAdjTile);
            const int v = ty * kAdjTile + px / kAdjTile;
            if (u >= a.W || v >= a.H) continue;
            const int i = v * a.W + u;
            PixelTerm P;
            if (pixel_term(M, a, R, t, params, dimg[i], u, v, aimg ? aimg + 3 * (size_t)i : nullptr, &P)) {
                acc[0] += residual_terms(P, a.delta, 0.0f).rho;
                acc[7] += 1.0f;
            }
        }
    }
    const double x = block_sum_part(acc, s_red);
    if (threadIdx.x < kAdjPart) partials[((size_t)kf * a.groups + blockIdx.x) * kAdjPart + threadIdx.x] = x;
}

// Keyframe poses exp(xi^) T0 (float64) and the cleared reach words.
__global__ void k_adj_setup(int32_t K, const double* __restrict__ T0, const double* __restrict__ xi,
                            double* __restrict__ poses, unsigned long long* __restrict__ reach) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double pose[12];
    for (int j = 0; j < 12; ++j) pose[j] = T0[12 * i + j];
    se3_apply_left(xi + 6 * i, pose);
    for (int j = 0; j < 12; ++j) poses[12 * i + j] = pose[j];
    reach[i] = 0ull;
}

// The block slot of every pixel's voxel (-1 for a pixel without a usable
// voxel: invalid depth, block absent or beyond param_blocks, W = 0 or
// g = 0), which the adjoint compares instead of recomputing every pixel of
// a block's rectangle.  With a frozen association it also finds, for each
// keyframe, how far (per axis, metres) its points lie outside the cells of
// their frozen voxels, as the bits of a non-negative float64 (whose integer
// order is its numeric order), so that the adjoint can widen each block's
// box by that much and still find every pixel frozen to one of its voxels.
// Grid (ceil(W H / 256), K).
template <bool FREEZE>
__global__ __launch_bounds__(kAdjBlock) void k_adj_slots(MapView M, AdjArgs a, const float* __restrict__ depth,
                                                         const double* __restrict__ poses,
                                                         const float4* __restrict__ params,
                                                         const int32_t* __restrict__ assoc,
                                                         int32_t* __restrict__ slots,
                                                         unsigned long long* __restrict__ reach) {
    __shared__ double s_max[kAdjBlock / 64];
    const int kf = blockIdx.y;
    const int N = a.W * a.H;
    const int i = blockIdx.x * kAdjBlock + threadIdx.x;
    double e = 0.0;
    if (i < N) {
        double R[9], t[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int c = 0; c < 3; ++c) R[3 * r + c] = poses[12 * kf + 4 * r + c];
            t[r] = poses[12 * kf + 4 * r + 3];
        }
        const size_t pi = (size_t)kf * N + i;
        const float D = depth[pi];
        int32_t slot = -1;
        if (depth_ok(D, a.zmin, a.zmax)) {
            double q[3];
            int m[3];
            pixel_point(a, R, t, D, i % a.W, i / a.W, q);
            nearest_voxel(a, q, m);
            bool ok = true;
            if (FREEZE) {
                const int32_t* as = assoc + pi * 3;
                ok = as[0] != INT_MIN;
                m[0] = as[0];
                m[1] = as[1];
                m[2] = as[2];
                if (ok)
#pragma unroll
                    for (int r = 0; r < 3; ++r) e = fmax(e, fabs(q[r] - a.vs * (double)m[r]) - 0.5 * a.vs);
            }
            if (ok) {
                const int32_t sl = hash_find(M, block_of(m[0]), block_of(m[1]), block_of(m[2]));
                if (sl >= 0 && (int64_t)sl < a.param_blocks) {
                    PixelTerm P;
                    if (voxel_term(M, a, params, (int64_t)sl * kBlockVoxels + morton9(m[0] & 7, m[1] & 7, m[2] & 7),
                                   q, m, &P))
                        slot = sl;
                }
            }
        }
        slots[pi] = slot;
    }
    if (!FREEZE) return;
    for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double x = 0.0;
        for (int w = 0; w < kAdjBlock / 64; ++w) x = fmax(x, s_max[w]);
        atomicMax(&reach[kf], (unsigned long long)__double_as_longlong(x));
    }
}

// The adjoint, one work-group per map block (every gridDim.x-th slot below
// min(param_blocks, blocks)).
//
// Which pixels can have their voxel in block b: for each keyframe the
// block's box of voxel cells, [v_s (8b - 1/2), v_s (8b + 15/2)) per axis
// (widened by a rounding margin, and for a frozen association by that
// keyframe's reach), projected into the image gives a rectangle, and its
// camera depth range bounds the depth of such a pixel.  The work-group
// takes up to kAdjChunk keyframes at a time: 8 threads per keyframe
// project the box's corners, and the rectangles are walked as one index
// space (thread t takes indices t, t + 256, ..., kAdjBatch of them per
// step with every load of a step issued before any is used), so no
// keyframe waits for another.  A pixel whose depth reaches the box, and
// whose nearest (or frozen) voxel lies in the block, adds s rho' and
// s rho' (q - v) into its voxel's sums, and its loss, pose terms and count
// into its keyframe's sums.  All sums are 64-bit fixed point (fixed_term):
// a thread keeps its keyframe sums in registers while its indices stay in
// one keyframe's rectangle and adds them to the work-group's LDS sums when
// they leave it.  Integer sums do not depend on the order of their terms,
// so every result is the same bits on every run.  At the end of a chunk
// each keyframe's sums (in float64) are added to this work-group's partial
// of that keyframe; at the end of a block each voxel's gradient is formed
// from its sums and added to dparams by the one thread that owns the voxel.
//
// Scales: with s_max = max_i |s_i| and N = K W H pixels at most per voxel,
// f_p keeps N s_max delta and f_q keeps N s_max delta (v_s / 2 + reach +
// margin) below 2^62 (the same in every work-group).  For a chunk's
// keyframe sums, with n the indices of the chunk, psi_max the largest
// |psi| of the block's voxels and q_max the largest coordinate of its box,
// the loss terms (at most delta (psi_max + sqrt(3) (v_s / 2 + reach)))
// and the pose terms (at most s_max delta max(1, sqrt(3) q_max)) get the
// scales that keep n times their bound below 2^62.
constexpr int kAdjChunk = kAdjBlock / 8;   // keyframes a work-group takes at a time

__device__ inline int fix_scale(double bound) {
    return (int)fmin(62.0, fmax(0.0, floor(62.0 - log2(fmax(bound, 1e-300)))));
}

template <bool FREEZE>
__global__ __launch_bounds__(kAdjBlock) void k_backward_blocks(MapView M, AdjArgs a, int32_t K,
                                                               const float* __restrict__ depth,
                                                               const double* __restrict__ poses,
                                                               const float4* __restrict__ params,
                                                               const float* __restrict__ gscale,
                                                               const int32_t* __restrict__ assoc,
                                                               const int32_t* __restrict__ slots,
                                                               const unsigned long long* __restrict__ reach,
                                                               float* __restrict__ dparams,
                                                               double* __restrict__ partials) {
    __shared__ unsigned long long sP[kBlockVoxels];
    __shared__ unsigned long long sQ[3][kBlockVoxels];
    __shared__ unsigned long long sK[kAdjChunk][kAdjPart];   // loss, 6 pose terms, count
    __shared__ double s_pose[kAdjChunk][12];
    __shared__ int s_rect[kAdjChunk][3];                      // u0, v0, width
    __shared__ int s_start[kAdjChunk + 1];                   // first index of each rectangle
    __shared__ float s_fmax[kAdjBlock / 64];
    __shared__ unsigned long long s_umax[kAdjBlock / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int N = a.W * a.H;

    // ---- voxel-sum scales (identical in every work-group)
    float smax = 0.0f;
    for (int k = threadIdx.x; k < K; k += kAdjBlock) smax = fmaxf(smax, fabsf(gscale[k]));
    for (int off = 32; off > 0; off >>= 1) smax = fmaxf(smax, __shfl_xor(smax, off));
    if (lane == 0) s_fmax[wave] = smax;
    // reach is a non-negative float64 stored as its bits: integer max = max
    unsigned long long rbits = 0ull;
    if (FREEZE)
        for (int k = threadIdx.x; k < K; k += kAdjBlock) rbits = reach[k] > rbits ? reach[k] : rbits;
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(rbits, off);
        rbits = o > rbits ? o : rbits;
    }
    if (lane == 0) s_umax[wave] = rbits;
    __syncthreads();
    smax = fmaxf(fmaxf(s_fmax[0], s_fmax[1]), fmaxf(s_fmax[2], s_fmax[3]));
    for (int w = 0; w < kAdjBlock / 64; ++w) rbits = s_umax[w] > rbits ? s_umax[w] : rbits;
    const double rmax = __longlong_as_double((long long)rbits);
    const double margin = 1e-6 * (1.0 + fabs(a.vs) * 1e3);
    const double base_p = (double)K * (double)N * (double)smax * (double)a.delta;
    const int fp = fix_scale(base_p), fq = fix_scale(base_p * (0.5 * a.vs + rmax + margin));
    const float wsp = ldexpf(1.0f, fp), whp = ldexpf(1.0f, fp - 32);
    const float wsq = ldexpf(1.0f, fq), whq = ldexpf(1.0f, fq - 32);

    // ---- this work-group's partials start at zero
    for (int k = threadIdx.x; k < K * kAdjPart; k += kAdjBlock)
        partials[((size_t)(k / kAdjPart) * gridDim.x + blockIdx.x) * kAdjPart + (k % kAdjPart)] = 0.0;

    int32_t nb = M.counters[kNumBlocks];
    nb = nb < M.max_blocks ? nb : M.max_blocks;
    const int64_t rows = a.param_blocks < (int64_t)nb ? a.param_blocks : (int64_t)nb;
    for (int64_t slot = blockIdx.x; slot < rows; slot += gridDim.x) {
        int b[3];
        unpack_key(M.block_keys[slot], &b[0], &b[1], &b[2]);
        // largest |psi| of the block's voxels (bounds the loss terms)
        float pmax = 0.0f;
        for (int c = threadIdx.x; c < kBlockVoxels; c += kAdjBlock) {
            sP[c] = 0ull;
            sQ[0][c] = sQ[1][c] = sQ[2][c] = 0ull;
            pmax = fmaxf(pmax, fabsf(params[slot * kBlockVoxels + c].x));
        }
        for (int off = 32; off > 0; off >>= 1) pmax = fmaxf(pmax, __shfl_xor(pmax, off));
        __syncthreads();   // s_fmax is free again
        if (lane == 0) s_fmax[wave] = pmax;
        __syncthreads();
        pmax = fmaxf(fmaxf(s_fmax[0], s_fmax[1]), fmaxf(s_fmax[2], s_fmax[3]));
        double qmax = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
            qmax = fmax(qmax, fmax(fabs(a.vs * (8.0 * b[i] - 0.5)), fabs(a.vs * (8.0 * b[i] + 7.5))));
        qmax += rmax + margin;

        for (int k0 = 0; k0 < K; k0 += kAdjChunk) {
            const int nk = K - k0 < kAdjChunk ? K - k0 : kAdjChunk;
            // ---- 8 threads per keyframe project the corners of the padded box
            {
                const int kl = threadIdx.x >> 3, c = threadIdx.x & 7;
                const int kf = k0 + (kl < nk ? kl : 0);
                const double* pose = poses + 12 * kf;
                double R[9], t[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
#pragma unroll
                    for (int j = 0; j < 3; ++j) R[3 * i + j] = pose[4 * i + j];
                    t[i] = pose[4 * i + 3];
                }
                const double pad = margin + (FREEZE ? __longlong_as_double((long long)reach[kf]) : 0.0);
                double X[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double lo = a.vs * (8.0 * b[i] - 0.5) - pad, hi = a.vs * (8.0 * b[i] + 7.5) + pad;
                    X[i] = ((c >> i) & 1) ? hi : lo;
                }
                double pc[3];
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    pc[j] = R[j] * (X[0] - t[0]) + R[3 + j] * (X[1] - t[1]) + R[6 + j] * (X[2] - t[2]);
                const bool front = pc[2] > 1e-6;
                const double iz = front ? 1.0 / pc[2] : 0.0;
                double umin = front ? a.fx * pc[0] * iz + a.cx : 1e300, umax = front ? umin : -1e300;
                double vmin = front ? a.fy * pc[1] * iz + a.cy : 1e300, vmax = front ? vmin : -1e300;
                int behind = front ? 0 : 1;
                for (int off = 1; off < 8; off <<= 1) {   // within the 8 lanes of this keyframe
                    umin = fmin(umin, __shfl_xor(umin, off));
                    umax = fmax(umax, __shfl_xor(umax, off));
                    vmin = fmin(vmin, __shfl_xor(vmin, off));
                    vmax = fmax(vmax, __shfl_xor(vmax, off));
                    behind |= __shfl_xor(behind, off);
                }
                if (kl < nk) {   // the keyframe's 8 threads store its pose: entries c and c + 8
                    s_pose[kl][c] = pose[c];
                    if (c + 8 < 12) s_pose[kl][c + 8] = pose[c + 8];
                }
                if (kl < nk && c == 0) {
                    int u0, u1, v0, v1;
                    if (behind) {   // the box reaches behind the image plane: every pixel
                        u0 = 0;
                        u1 = a.W - 1;
                        v0 = 0;
                        v1 = a.H - 1;
                    } else {
                        u0 = (int)fmin(fmax(0.0, floor(umin) - 1.0), (double)a.W);
                        u1 = (int)fmax(fmin((double)(a.W - 1), ceil(umax) + 1.0), -1.0);
                        v0 = (int)fmin(fmax(0.0, floor(vmin) - 1.0), (double)a.H);
                        v1 = (int)fmax(fmin((double)(a.H - 1), ceil(vmax) + 1.0), -1.0);
                    }
                    const bool empty = u1 < u0 || v1 < v0;
                    s_rect[kl][0] = u0;
                    s_rect[kl][1] = v0;
                    s_rect[kl][2] = empty ? 0 : u1 - u0 + 1;
                    s_start[kl + 1] = empty ? 0 : (u1 - u0 + 1) * (v1 - v0 + 1);   // area, summed below
                }
                if (threadIdx.x < kAdjChunk * kAdjPart) sK[threadIdx.x / kAdjPart][threadIdx.x % kAdjPart] = 0ull;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_start[0] = 0;
                for (int k = 1; k <= nk; ++k) s_start[k] += s_start[k - 1];
            }
            __syncthreads();
            const int total = s_start[nk];
            // chunk scales of the keyframe sums
            const double lossb = (double)a.delta * ((double)pmax + 1.7320508075688772 * (0.5 * a.vs + rmax + margin));
            const int fl = fix_scale((double)total * lossb);
            const int fj = fix_scale((double)total * (double)smax * (double)a.delta * fmax(1.0, 1.7320508075688772 * qmax));
            const float wsl = ldexpf(1.0f, fl), whl = ldexpf(1.0f, fl - 32);
            const float wsj = ldexpf(1.0f, fj), whj = ldexpf(1.0f, fj - 32);

            // ---- the rectangles' pixels
            int kcur = 0;                  // this thread's keyframe (its indices only grow)
            unsigned long long acc[kAdjPart];
#pragma unroll
            for (int k = 0; k < kAdjPart; ++k) acc[k] = 0ull;
            for (int base = threadIdx.x; base < total; base += kAdjBlock * kAdjBatch) {
                // stage 1: the slot of every index's pixel
                int uu[kAdjBatch], vv[kAdjBatch], kk[kAdjBatch];
                size_t pix[kAdjBatch];
                int32_t sl[kAdjBatch];
                int kw = kcur;
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j) {
                    const int p = base + j * kAdjBlock;
                    sl[j] = -1;
                    uu[j] = vv[j] = 0;
                    pix[j] = 0;
                    kk[j] = kw;
                    if (p >= total) continue;
                    while (p >= s_start[kw + 1]) ++kw;
                    kk[j] = kw;
                    const int bw = s_rect[kw][2];
                    const int q = p - s_start[kw];
                    // row and column without an integer division (q < 2^24 is exact)
                    int row = (int)(((float)q + 0.5f) * (1.0f / (float)bw));
                    int col = q - row * bw;
                    if (col < 0) {
                        --row;
                        col += bw;
                    } else if (col >= bw) {
                        ++row;
                        col -= bw;
                    }
                    uu[j] = s_rect[kw][0] + col;
                    vv[j] = s_rect[kw][1] + row;
                    pix[j] = (size_t)(k0 + kw) * N + (size_t)vv[j] * a.W + uu[j];
                    sl[j] = slots[pix[j]];
                }
                // stage 2: depth (and frozen voxel) of the pixels of this block
                bool live[kAdjBatch];
                float D[kAdjBatch];
                int m[kAdjBatch][3];
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j) {
                    live[j] = (int64_t)sl[j] == slot;
                    if (!live[j]) continue;
                    D[j] = depth[pix[j]];
                    if (FREEZE) {
                        const int32_t* as = assoc + pix[j] * 3;
                        m[j][0] = as[0];
                        m[j][1] = as[1];
                        m[j][2] = as[2];
                    }
                }
                // stage 3: point, voxel, the voxel's weight and parameters
                double q[kAdjBatch][3];
                int64_t vi[kAdjBatch];
                float Wv[kAdjBatch];
                float4 pr[kAdjBatch];
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j) {
                    if (!live[j]) continue;
                    const int kl = kk[j];
                    double R[9], t[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
#pragma unroll
                        for (int c = 0; c < 3; ++c) R[3 * i + c] = s_pose[kl][4 * i + c];
                        t[i] = s_pose[kl][4 * i + 3];
                    }
                    pixel_point(a, R, t, D[j], uu[j], vv[j], q[j]);
                    if (!FREEZE) nearest_voxel(a, q[j], m[j]);
                    vi[j] = slot * kBlockVoxels + morton9(m[j][0] & 7, m[j][1] & 7, m[j][2] & 7);
                    Wv[j] = M.weight[vi[j]];
                    pr[j] = params[vi[j]];
                }
                // stage 4: residuals and sums
#pragma unroll
                for (int j = 0; j < kAdjBatch; ++j) {
                    if (!live[j] || !(Wv[j] > 0.0f)) continue;
                    PixelTerm P;
                    if (!param_term(pr[j], a, vi[j], q[j], m[j], &P)) continue;
                    if (kk[j] != kcur) {   // this thread's indices left keyframe kcur
#pragma unroll
                        for (int k = 0; k < kAdjPart; ++k) {
                            if (acc[k]) atomicAdd(&sK[kcur][k], acc[k]);
                            acc[k] = 0ull;
                        }
                        kcur = kk[j];
                    }
                    const ResidualTerms rt = residual_terms(P, a.delta, gscale[k0 + kk[j]]);
                    acc[0] += fixed_term(wsl, whl, rt.rho);
#pragma unroll
                    for (int k = 0; k < 6; ++k) acc[1 + k] += fixed_term(wsj, whj, rt.rp * rt.J[k]);
                    acc[7] += 1ull;
                    const int c = (m[j][0] & 7) | ((m[j][1] & 7) << 3) | ((m[j][2] & 7) << 6);
                    atomicAdd(&sP[c], fixed_term(wsp, whp, rt.rp));
#pragma unroll
                    for (int k = 0; k < 3; ++k) atomicAdd(&sQ[k][c], fixed_term(wsq, whq, rt.rp * P.dq[k]));
                }
            }
#pragma unroll
            for (int k = 0; k < kAdjPart; ++k)
                if (acc[k]) atomicAdd(&sK[kcur][k], acc[k]);
            __syncthreads();
            // ---- the chunk's keyframe sums into this work-group's partials
            if (threadIdx.x < nk * kAdjPart) {
                const int kl = threadIdx.x / kAdjPart, k = threadIdx.x % kAdjPart;
                const long long v = (long long)sK[kl][k];
                const double x = k == 7 ? (double)v : (double)v * ldexp(1.0, k == 0 ? -fl : -fj);
                partials[((size_t)(k0 + kl) * gridDim.x + blockIdx.x) * kAdjPart + k] += x;
            }
            __syncthreads();
        }
        // ---- each voxel's gradient from its sums, added once by its owner
        const double ip = ldexp(1.0, -fp), iq = ldexp(1.0, -fq);
        for (int c = threadIdx.x; c < kBlockVoxels; c += kAdjBlock) {
            const unsigned long long p0 = sP[c], q0 = sQ[0][c], q1 = sQ[1][c], q2 = sQ[2][c];
            if ((p0 | q0 | q1 | q2) == 0ull) continue;
            const int64_t vi = slot * kBlockVoxels + morton9(c & 7, (c >> 3) & 7, c >> 6);
            const float4 p = params[vi];
            const float inv_ng = 1.0f / sqrtf(p.y * p.y + p.z * p.z + p.w * p.w);
            const float gh[3] = {p.y * inv_ng, p.z * inv_ng, p.w * inv_ng};
            const float S[3] = {(float)((double)(long long)q0 * iq), (float)((double)(long long)q1 * iq),
                                (float)((double)(long long)q2 * iq)};
            const float gS = gh[0] * S[0] + gh[1] * S[1] + gh[2] * S[2];
            float4 d = reinterpret_cast<float4*>(dparams)[vi];
            d.x += (float)((double)(long long)p0 * ip);
            d.y += inv_ng * (S[0] - gh[0] * gS);
            d.z += inv_ng * (S[1] - gh[1] * gS);
            d.w += inv_ng * (S[2] - gh[2] * gS);
            reinterpret_cast<float4*>(dparams)[vi] = d;
        }
        __syncthreads();
    }
}

// One work-group per keyframe: fixed-order sum of `groups` partials (256
// threads stride over the work-groups, then a tree in LDS), then
// loss_out[kf] and (when asked) dxi = Jl(xi)^T (pose sums).
__global__ __launch_bounds__(256) void k_keyframe_finish(int32_t groups, const double* __restrict__ xi,
                                                         const double* __restrict__ partials,
                                                         double* __restrict__ loss_out, double* __restrict__ dxi_out,
                                                         double* __restrict__ count_out) {
    __shared__ double s_part[kAdjPart][256];
    const int kf = blockIdx.x;
    double x[kAdjPart];
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) x[k] = 0.0;
    for (int g = threadIdx.x; g < groups; g += 256) {
        const double* p = partials + ((size_t)kf * groups + g) * kAdjPart;
#pragma unroll
        for (int k = 0; k < kAdjPart; ++k) x[k] += p[k];
    }
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) s_part[k][threadIdx.x] = x[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kAdjPart; ++k) s_part[k][threadIdx.x] += s_part[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    if (loss_out) loss_out[kf] = s_part[0][0];
    if (count_out) count_out[kf] = s_part[7][0];
    if (dxi_out) {
        double Jl[36];
        se3_left_jacobian(xi + 6 * kf, Jl);
        for (int c = 0; c < 6; ++c) {
            double v = 0.0;
            for (int r = 0; r < 6; ++r) v += Jl[6 * r + c] * s_part[1 + r][0];
            dxi_out[6 * kf + c] = v;
        }
    }
}

__global__ void k_export_params(MapView M, int storage, int64_t rows, float4* __restrict__ out) {
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    const int64_t n = (rows < (int64_t)nb ? rows : (int64_t)nb) * kBlockVoxels;
    for (int64_t vi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; vi < rows * kBlockVoxels;
         vi += (int64_t)gridDim.x * blockDim.x) {
        float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (vi < n) {
            const float Wv = M.weight[vi];
            if (storage == GSDF_FP32) {
                const float4 r = reinterpret_cast<const float4*>(M.vox)[vi];
                p = make_float4(Wv > 0.0f ? r.x / Wv : 0.0f, r.y, r.z, r.w);
            } else {
                const ushort4 r = reinterpret_cast<const ushort4*>(M.vox)[vi];
                p = make_float4(unpack16(r.x, storage) * M.truncation, unpack16(r.y, storage),
                                unpack16(r.z, storage), unpack16(r.w, storage));
            }
        }
        out[vi] = p;
    }
}

__global__ void k_import_params(MapView M, int storage, int64_t rows, const float4* __restrict__ in) {
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    const int64_t n = (rows < (int64_t)nb ? rows : (int64_t)nb) * kBlockVoxels;
    for (int64_t vi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; vi < n; vi += (int64_t)gridDim.x * blockDim.x) {
        const float Wv = M.weight[vi];
        if (!(Wv > 0.0f)) continue;   // unobserved voxels keep their (zero) record
        const float4 p = in[vi];
        if (storage == GSDF_FP32) {
            reinterpret_cast<float4*>(M.vox)[vi] = make_float4(p.x * Wv, p.y, p.z, p.w);
        } else {
            reinterpret_cast<ushort4*>(M.vox)[vi] =
                make_ushort4(pack16(p.x / M.truncation, storage), pack16(p.y, storage), pack16(p.z, storage),
                             pack16(p.w, storage));
        }
    }
}

__global__ void k_compose_poses(int32_t K, const double* __restrict__ T0, const double* __restrict__ xi,
                                double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double pose[12];
    for (int j = 0; j < 12; ++j) pose[j] = T0[12 * i + j];
    se3_apply_left(xi + 6 * i, pose);
    for (int j = 0; j < 12; ++j) out[12 * i + j] = pose[j];
}

inline int adj_groups(const gsdf_camera& cam) {
    const int n = ceil_div(cam.width, kAdjTile) * ceil_div(cam.height, kAdjTile);
    return n < kAdjMaxGroups ? n : kAdjMaxGroups;
}

inline AdjArgs adj_args(const gsdf_map& map, const gsdf_camera& cam, float delta, int32_t freeze,
                        int64_t param_blocks) {
    AdjArgs a;
    a.W = cam.width;
    a.H = cam.height;
    a.groups = adj_groups(cam);
    a.freeze = freeze;
    a.fx = cam.fx;
    a.fy = cam.fy;
    a.ifx = 1.0 / cam.fx;
    a.ify = 1.0 / cam.fy;
    a.cx = cam.cx;
    a.cy = cam.cy;
    a.zmin = cam.zmin;
    a.zmax = cam.zmax;
    a.delta = delta;
    a.pad = 0.0f;
    a.vs = map.desc.voxel_size;
    a.inv_vs = 1.0 / map.desc.voxel_size;
    a.param_blocks = param_blocks;
    return a;
}

}  // namespace gsdf

using namespace gsdf;

extern "C" {

size_t gsdf_keyframe_scratch_bytes(const gsdf_camera* cam, int32_t n_keyframes) {
    if (!valid_cam(cam) || n_keyframes <= 0) return 0;
    return adj_scratch(n_keyframes, (int64_t)cam->width * cam->height).total;
}

static int keyframe_common(const gsdf_map* map, const float* depth_dev, int32_t K, const gsdf_camera* cam,
                           const double* T0_dev, const double* xi_dev, const float* params_dev,
                           int64_t param_blocks, float huber_delta, void* scratch, size_t scratch_bytes) {
    if (!valid_map(map) || !valid_cam(cam) || K <= 0 || K > 65535 || !depth_dev || !T0_dev || !xi_dev ||
        !params_dev || param_blocks < 0 || param_blocks > map->desc.max_blocks || !(huber_delta > 0.0f) || !scratch)
        return GSDF_EINVAL;
    if (scratch_bytes < gsdf_keyframe_scratch_bytes(cam, K)) return GSDF_EINVAL;
    if (!has_gradients(map)) return GSDF_EINVAL;
    return GSDF_OK;
}

int gsdf_keyframe_loss(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes, const gsdf_camera* cam,
                       const double* T0_dev, const double* xi_dev, const float* params_dev, int64_t param_blocks,
                       float huber_delta, int32_t* assoc_dev, int32_t freeze, double* loss_dev, double* count_dev,
                       void* scratch, size_t scratch_bytes, void* stream) {
    int rc = keyframe_common(map, depth_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                             huber_delta, scratch, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!loss_dev || (freeze && !assoc_dev)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const AdjArgs a = adj_args(*map, *cam, huber_delta, freeze, param_blocks);
    const AdjScratch L = adj_scratch(n_keyframes, (int64_t)cam->width * cam->height);
    char* base = (char*)scratch;
    double* partials = (double*)(base + L.partials);
    double* poses = (double*)(base + L.poses);
    k_adj_setup<<<ceil_div(n_keyframes, 64), 64, 0, s>>>(n_keyframes, T0_dev, xi_dev, poses,
                                                        (unsigned long long*)(base + L.reach));
    {
        TimedLaunch tl(map->timer, GSDF_K_LOSS, s);
        k_keyframe_loss<<<dim3(a.groups, n_keyframes), kAdjBlock, 0, s>>>(
            make_view(*map), a, depth_dev, poses, reinterpret_cast<const float4*>(params_dev), assoc_dev, partials);
    }
    k_keyframe_finish<<<n_keyframes, 256, 0, s>>>(a.groups, xi_dev, partials, loss_dev, nullptr, count_dev);
    return launch_status();
}

int gsdf_backward(const gsdf_map* map, const float* depth_dev, int32_t n_keyframes,
                  const gsdf_camera* cam, const double* T0_dev, const double* xi_dev, const float* params_dev,
                  int64_t param_blocks, float huber_delta, int32_t* assoc_dev, int32_t freeze,
                  const float* grad_loss_dev, float* dparams_dev, double* dxi_dev, double* loss_dev, void* scratch,
                  size_t scratch_bytes, void* stream) {
    int rc = keyframe_common(map, depth_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                             huber_delta, scratch, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!grad_loss_dev || !dparams_dev || !dxi_dev || (freeze && !assoc_dev)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const AdjArgs a = adj_args(*map, *cam, huber_delta, freeze, param_blocks);
    const AdjScratch L = adj_scratch(n_keyframes, (int64_t)cam->width * cam->height);
    char* base = (char*)scratch;
    double* partials = (double*)(base + L.partials);
    double* poses = (double*)(base + L.poses);
    unsigned long long* reach = (unsigned long long*)(base + L.reach);
    const int groups = (int)(param_blocks < kBackGroups ? (param_blocks > 0 ? param_blocks : 1) : kBackGroups);
    k_adj_setup<<<ceil_div(n_keyframes, 64), 64, 0, s>>>(n_keyframes, T0_dev, xi_dev, poses, reach);
    const MapView M = make_view(*map);
    const float4* P = reinterpret_cast<const float4*>(params_dev);
    int32_t* slots = (int32_t*)(base + L.slots);
    const dim3 pgrid(ceil_div(cam->width * cam->height, kAdjBlock), n_keyframes);
    {
        TimedLaunch tl(map->timer, GSDF_K_BACKWARD, s);
        if (freeze) {
            k_adj_slots<true><<<pgrid, kAdjBlock, 0, s>>>(M, a, depth_dev, poses, P, assoc_dev, slots, reach);
            k_backward_blocks<true><<<groups, kAdjBlock, 0, s>>>(M, a, n_keyframes, depth_dev, poses, P,
                                                                grad_loss_dev, assoc_dev, slots, reach, dparams_dev,
                                                                partials);
        } else {
            k_adj_slots<false><<<pgrid, kAdjBlock, 0, s>>>(M, a, depth_dev, poses, P, nullptr, slots, reach);
            k_backward_blocks<false><<<groups, kAdjBlock, 0, s>>>(M, a, n_keyframes, depth_dev, poses, P,
                                                                 grad_loss_dev, nullptr, slots, reach, dparams_dev,
                                                                 partials);
        }
    }
    k_keyframe_finish<<<n_keyframes, 256, 0, s>>>(groups, xi_dev, partials, loss_dev, dxi_dev, nullptr);
    return launch_status();
}

int gsdf_export_params(const gsdf_map* map, float* params_dev, int64_t param_blocks, void* stream) {
    if (!valid_map(map) || !params_dev || param_blocks < 0 || param_blocks > map->desc.max_blocks ||
        !has_gradients(map))
        return GSDF_EINVAL;
    if (param_blocks == 0) return GSDF_OK;
    k_export_params<<<2048, 256, 0, (hipStream_t)stream>>>(make_view(*map), map->desc.storage, param_blocks,
                                                           reinterpret_cast<float4*>(params_dev));
    return launch_status();
}

int gsdf_import_params(gsdf_map* map, const float* params_dev, int64_t param_blocks, void* stream) {
    if (!valid_map(map) || !params_dev || param_blocks < 0 || param_blocks > map->desc.max_blocks ||
        !has_gradients(map))
        return GSDF_EINVAL;
    if (param_blocks == 0) return GSDF_OK;
    k_import_params<<<2048, 256, 0, (hipStream_t)stream>>>(make_view(*map), map->desc.storage, param_blocks,
                                                           reinterpret_cast<const float4*>(params_dev));
    return launch_status();
}

int gsdf_compose_poses(int32_t n, const double* T0_dev, const double* xi_dev, double* T_out_dev, void* stream) {
    if (n < 0 || (n > 0 && (!T0_dev || !xi_dev || !T_out_dev))) return GSDF_EINVAL;
    if (n == 0) return GSDF_OK;
    k_compose_poses<<<ceil_div(n, 64), 64, 0, (hipStream_t)stream>>>(n, T0_dev, xi_dev, T_out_dev);
    return launch_status();
}

int gsdf_voxel_order(int32_t order_out[512]) {
    if (!order_out) return GSDF_EINVAL;
    for (int c = 0; c < kBlockVoxels; ++c) order_out[c] = morton9(c & 7, (c >> 3) & 7, c >> 6);
    return GSDF_OK;
}

}  // extern "C"
