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
// scattering.  A pixel-parallel pass over 32x32 pixel tiles finds each
// pixel's voxel, adds the pixel's loss and pose terms into its keyframe's
// sums (fixed-order float64 reductions), and groups the tile's pixels by map
// block: each tile writes its pixels' ids block by block into its own part
// of a list and one record (block, count) per block it touches.  A scan of
// the per-block record counts and a scatter of the records give each block
// the runs of the list that hold its pixels.  Then one work-group owns a
// map block, walks its runs and adds the pixels' terms into the block's 512
// voxel sums in LDS, and writes each voxel once.  No two work-groups write
// the same voxel, so nothing is added to global memory atomically except
// integer counts, and the voxel sums are 64-bit fixed point (an integer sum
// does not depend on the order of its terms, and the order of the runs
// does vary), so the gradients are the same bits on every run.
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
constexpr int kAdjMaxGroups = 512;  // work-groups per keyframe of the pixel passes
constexpr int kAdjTile = 32;        // the pixel passes take 32x32 pixel tiles, four pixels a thread
constexpr int kBackGroups = 8192;   // work-groups of the per-block gather (each owns every 8192th block)
constexpr int kScanTile = 4096;     // block counts per work-group of the offset scan (16 a thread)
constexpr int kPoseLds = 64;        // the gather keeps the poses in LDS for up to this many keyframes
constexpr int kTilePx = kAdjTile * kAdjTile;
constexpr int kGatherBatch = 2;     // list entries a thread of the gather loads at a time
constexpr int kLookup = 2;          // pixels a thread of the pixel passes looks up together
constexpr int kRunBatch = 256;      // runs the gather holds in LDS at a time

struct AdjArgs {
    int32_t W, H, groups, freeze;
    double fx, fy, ifx, ify, cx, cy;
    float zmin, zmax, delta, pad;
    double vs, inv_vs;
    int64_t param_blocks;   // rows of the parameter buffer (slots beyond are unobserved)
};

// Scratch of the keyframe calls: per-work-group partials of the keyframe
// sums, the keyframe poses exp(xi^) T0, two words of bounds (the reach of a
// frozen association as float64 bits, max |s_i|), and the pixel lists:
// per tile (K x tiles of them) 1024 list entries (pixel id, depth) and up
// to 1024 records
// (block, count), the records' count per tile, the runs (start, count)
// sorted by block, and per block its pixel count, run count, first run and
// a cursor, with the per-tile sums of the scan.
struct AdjScratch {
    size_t partials, poses, bounds, list, recs, nrec, runs, pix_count, run_count, run_off, cursor, tiles, total;
};

inline int64_t adj_tiles(int32_t W, int32_t H) {
    return (int64_t)((W + kAdjTile - 1) / kAdjTile) * ((H + kAdjTile - 1) / kAdjTile);
}

inline AdjScratch adj_scratch(int32_t K, int64_t tiles, int64_t param_blocks) {
    AdjScratch L;
    size_t o = 0;
    const size_t regions = (size_t)K * (size_t)tiles;
    const size_t n = regions * kTilePx;
    const size_t nb = (size_t)(param_blocks > 0 ? param_blocks : 1);
    L.partials = o;  o = align256(o + (size_t)K * kAdjMaxGroups * kAdjPart * sizeof(double));
    L.poses = o;     o = align256(o + (size_t)K * 12 * sizeof(double));
    L.bounds = o;    o = align256(o + 2 * sizeof(double));
    L.list = o;      o = align256(o + n * sizeof(uint2));
    L.recs = o;      o = align256(o + n * sizeof(int2));
    L.nrec = o;      o = align256(o + regions * sizeof(int32_t));
    L.runs = o;      o = align256(o + n * sizeof(int2));
    L.pix_count = o; o = align256(o + nb * sizeof(int32_t));
    L.run_count = o; o = align256(o + nb * sizeof(int32_t));
    L.run_off = o;   o = align256(o + nb * sizeof(int32_t));
    L.cursor = o;    o = align256(o + nb * sizeof(int32_t));
    L.tiles = o;     o = align256(o + ((nb + kScanTile - 1) / kScanTile) * sizeof(int32_t));
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
    for (int r = 0; r < 3; ++r) m[r] = (int)floor(fma(q[r], a.inv_vs, 0.5));
}

// Voxel, offsets and parameters of one pixel.
struct PixelTerm {
    float D, psi, gh[3], inv_ng, dq[3], q[3];
};

// Pool slot of a block key whose first probe, at h, held neither the key
// nor the empty key: linear probing from h + 1 (an empty entry ends it).
__device__ inline int32_t hash_probe_rest(const MapView& M, uint64_t key, uint64_t h) {
    for (uint64_t probe = 1; probe <= M.mask; ++probe) {
        h = (h + 1) & M.mask;
        const uint4 e = *reinterpret_cast<const uint4*>(&M.hash[h]);
        const uint64_t k = (uint64_t)e.x | ((uint64_t)e.y << 32);
        if (k == key) return (int32_t)e.z;
        if (k == kEmptyKey) return -1;
    }
    return -1;
}

// The voxel terms of NP pixels of one thread, stage by stage, every load of
// a stage issued for all NP pixels before any is used: the depth (and the
// frozen voxel when READ_ASSOC), then the point q = T x and its nearest
// voxel (Eq. (14)) with the block's first hash probe, then the rest of the
// probe (rarely needed), then the voxel's weight and parameters.  ok[j]:
// the pixel has a usable voxel (valid depth, block present below
// param_blocks, W > 0, g != 0); then slot[j], m[j] (voxel coordinates) and
// P[j] hold it.  look[j]: the pixel reached the hash lookup (valid depth
// and, when READ_ASSOC, an associated voxel).  With READ_ASSOC, *reach
// takes the largest per-axis distance of a point outside its frozen
// voxel's cell.
template <int NP, bool READ_ASSOC>
__device__ inline void lookup_batch(const MapView& M, const AdjArgs& a, const double R[9], const double t[3],
                                    const float4* __restrict__ params, const float* __restrict__ dimg,
                                    const int32_t* __restrict__ aimg, const int (&u)[NP], const int (&v)[NP],
                                    const bool (&in)[NP], bool (&ok)[NP], bool (&look)[NP], int32_t (&slot)[NP],
                                    int (&m)[NP][3], PixelTerm (&P)[NP], double* reach) {
    float D[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        const size_t i = (size_t)v[j] * a.W + u[j];
        D[j] = in[j] ? dimg[i] : 0.0f;
        if (READ_ASSOC && in[j]) {
            m[j][0] = aimg[3 * i];
            m[j][1] = aimg[3 * i + 1];
            m[j][2] = aimg[3 * i + 2];
        }
    }
    uint64_t key[NP], h[NP];
    uint4 e[NP];
    bool probe[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        probe[j] = false;
        look[j] = in[j] && depth_ok(D[j], a.zmin, a.zmax);
        if (READ_ASSOC) look[j] = look[j] && m[j][0] != INT_MIN;
        if (!look[j]) continue;
        P[j].D = D[j];
        double q[3];
        pixel_point(a, R, t, D[j], u[j], v[j], q);
        if (READ_ASSOC) {
#pragma unroll
            for (int r = 0; r < 3; ++r) *reach = fmax(*reach, fabs(q[r] - a.vs * (double)m[j][r]) - 0.5 * a.vs);
        } else {
            nearest_voxel(a, q, m[j]);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            P[j].q[r] = (float)q[r];
            P[j].dq[r] = (float)(q[r] - a.vs * (double)m[j][r]);
        }
        const int bx = block_of(m[j][0]), by = block_of(m[j][1]), bz = block_of(m[j][2]);
        probe[j] = key_in_range(bx, by, bz);
        if (!probe[j]) continue;
        key[j] = pack_key(bx, by, bz);
        h[j] = mix64(key[j]) & M.mask;
        e[j] = *reinterpret_cast<const uint4*>(&M.hash[h[j]]);
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        slot[j] = -1;
        if (!look[j] || !probe[j]) continue;
        const uint64_t k = (uint64_t)e[j].x | ((uint64_t)e[j].y << 32);
        if (k == key[j])
            slot[j] = (int32_t)e[j].z;
        else if (k != kEmptyKey)
            slot[j] = hash_probe_rest(M, key[j], h[j]);
    }
    float Wv[NP];
    float4 pr[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        ok[j] = slot[j] >= 0 && (int64_t)slot[j] < a.param_blocks;
        if (!ok[j]) continue;
        const int64_t vi = (int64_t)slot[j] * kBlockVoxels + morton9(m[j][0] & 7, m[j][1] & 7, m[j][2] & 7);
        Wv[j] = M.weight[vi];
        pr[j] = params[vi];
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        if (!ok[j]) continue;
        const float n2 = pr[j].y * pr[j].y + pr[j].z * pr[j].z + pr[j].w * pr[j].w;
        ok[j] = Wv[j] > 0.0f && n2 > 0.0f;
        if (!ok[j]) continue;
        P[j].inv_ng = 1.0f / sqrtf(n2);
        P[j].psi = pr[j].x;
        P[j].gh[0] = pr[j].y * P[j].inv_ng;
        P[j].gh[1] = pr[j].z * P[j].inv_ng;
        P[j].gh[2] = pr[j].w * P[j].inv_ng;
    }
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

// Work-group sum of kAdjPart values per thread, in float64 (wave shuffles,
// then one value per wave in a fixed order); the totals land in out[] of
// threads 0 .. kAdjPart-1 (out[k] in thread k).
template <typename T>
__device__ inline double block_sum_part(const T acc[kAdjPart], double (*s_red)[kAdjBlock / 64]) {
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
// keyframe blockIdx.y (four pixels a thread, looked up together) and
// writes its partial sums (loss, the six pose sums unused here, the count
// of pixels used); FREEZE reads each pixel's voxel from the association
// buffer, else with an association buffer it records each pixel's voxel
// (INT32_MIN for a pixel without a usable voxel).
template <bool FREEZE>
__global__ __launch_bounds__(kAdjBlock) void k_keyframe_loss(MapView M, AdjArgs a, const float* __restrict__ depth,
                                                             const double* __restrict__ poses,
                                                             const float4* __restrict__ params,
                                                             int32_t* __restrict__ assoc,
                                                             double* __restrict__ partials) {
    __shared__ double s_red[kAdjPart][kAdjBlock / 64];
    constexpr int kPer = kTilePx / kAdjBlock;
    // work-group (x, k) in XCD-aware order: neighbouring tiles share an L2
    const int lin = band_rank(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int kf = lin / gridDim.x, grp = lin - kf * gridDim.x;
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
    double reach = 0.0;
    const int tiles_x = (a.W + kAdjTile - 1) / kAdjTile;
    const int ntiles = tiles_x * ((a.H + kAdjTile - 1) / kAdjTile);
    for (int tile = grp; tile < ntiles; tile += a.groups) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
#pragma unroll
        for (int g = 0; g < kPer; g += kLookup) {
            int u[kLookup], v[kLookup];
            bool in[kLookup], ok[kLookup], look[kLookup];
            int32_t slot[kLookup];
            int m[kLookup][3];
            PixelTerm P[kLookup];
#pragma unroll
            for (int j = 0; j < kLookup; ++j) {
                const int px = threadIdx.x + (g + j) * kAdjBlock;
                u[j] = tx * kAdjTile + (px % kAdjTile);
                v[j] = ty * kAdjTile + px / kAdjTile;
                in[j] = u[j] < a.W && v[j] < a.H;
            }
            lookup_batch<kLookup, FREEZE>(M, a, R, t, params, dimg, aimg, u, v, in, ok, look, slot, m, P, &reach);
#pragma unroll
            for (int j = 0; j < kLookup; ++j) {
                if (ok[j]) {
                    acc[0] += residual_terms(P[j], a.delta, 0.0f).rho;
                    acc[7] += 1.0f;
                }
                if (!FREEZE && aimg && in[j]) {
                    int32_t* as = aimg + 3 * ((size_t)v[j] * a.W + u[j]);
                    as[0] = ok[j] ? m[j][0] : INT_MIN;
                    as[1] = ok[j] ? m[j][1] : INT_MIN;
                    as[2] = ok[j] ? m[j][2] : INT_MIN;
                }
            }
        }
    }
    const double x = block_sum_part(acc, s_red);
    if (threadIdx.x < kAdjPart) partials[((size_t)kf * a.groups + grp) * kAdjPart + threadIdx.x] = x;
}

// Keyframe poses exp(xi^) T0 (float64), and for the adjoint the cleared
// per-block counters and reach word.  One thread per keyframe and per block.
__global__ void k_adj_setup(int32_t K, const double* __restrict__ T0, const double* __restrict__ xi,
                            double* __restrict__ poses, int64_t nb, int32_t* __restrict__ pix_count,
                            int32_t* __restrict__ run_count, int32_t* __restrict__ cursor,
                            unsigned long long* __restrict__ reach) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < K) {
        double pose[12];
        for (int j = 0; j < 12; ++j) pose[j] = T0[12 * i + j];
        se3_apply_left(xi + 6 * i, pose);
        for (int j = 0; j < 12; ++j) poses[12 * i + j] = pose[j];
    }
    if (i < nb) {
        pix_count[i] = 0;
        run_count[i] = 0;
        cursor[i] = 0;
    }
    if (i == 0 && reach) *reach = 0ull;
}

// Exclusive work-group prefix sums of two int32 per thread (all 256
// threads): a wave scan, the wave totals in LDS (s_w: 8 words).  The
// totals land in *tot_a, *tot_b.
__device__ inline void block_scan2(int32_t a, int32_t b, int32_t* ex_a, int32_t* ex_b, int32_t* tot_a,
                                   int32_t* tot_b, int32_t* s_w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t ia = a, ib = b;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t ya = __shfl_up(ia, d), yb = __shfl_up(ib, d);
        if (lane >= d) {
            ia += ya;
            ib += yb;
        }
    }
    __syncthreads();   // s_w may still be read by a previous call
    if (lane == 63) {
        s_w[wave] = ia;
        s_w[4 + wave] = ib;
    }
    __syncthreads();
    int32_t pa = 0, pb = 0, ta = 0, tb = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        if (w < wave) {
            pa += s_w[w];
            pb += s_w[4 + w];
        }
        ta += s_w[w];
        tb += s_w[4 + w];
    }
    *ex_a = pa + ia - a;
    *ex_b = pb + ib - b;
    *tot_a = ta;
    *tot_b = tb;
}

// The adjoint's pixel pass.  Grid (groups, K), 32x32 tiles as the loss
// pass; tile t of keyframe k is region r = k tiles + t.  Per pixel: its
// voxel (nearest, or frozen), and when the voxel is usable (block present
// below param_blocks, W > 0, g != 0) its loss, pose terms s rho' [g^; q x g^]
// and count into this work-group's partial of its keyframe.  The tile's
// usable pixels are grouped by block in LDS (an open-addressing table of
// 1024 entries, so it never fills; one LDS atomic add gives a pixel its
// rank in its block); a scan of the entries' counts places each block's
// pixels (id and depth) in a run of the region's 1024 list entries, and the region gets
// one record (block, count) per block, in run order, and nrec[r] records.
// The per-block pixel and record counts are integer atomics.  With a
// frozen association the pass also finds how far (per axis, metres) the
// points lie outside the cells of their frozen voxels, as the bits of a
// non-negative float64 (whose integer order is its numeric order); that
// bounds the offsets q - v of the voxel sums.
template <bool FREEZE>
__global__ __launch_bounds__(kAdjBlock) void k_adj_pixels(MapView M, AdjArgs a, const float* __restrict__ depth,
                                                          const double* __restrict__ poses,
                                                          const float4* __restrict__ params,
                                                          const float* __restrict__ gscale,
                                                          const int32_t* __restrict__ assoc,
                                                          uint2* __restrict__ list, int2* __restrict__ recs,
                                                          int32_t* __restrict__ nrec, int32_t* __restrict__ pix_count,
                                                          int32_t* __restrict__ run_count,
                                                          unsigned long long* __restrict__ reach,
                                                          double* __restrict__ partials) {
    __shared__ double s_red[kAdjPart][kAdjBlock / 64];
    __shared__ double s_max[kAdjBlock / 64];
    __shared__ int32_t s_key[kTilePx];
    __shared__ int32_t s_cnt[kTilePx];
    __shared__ int32_t s_w[8];
    constexpr int kPer = kTilePx / kAdjBlock;   // pixels (and table entries) a thread takes: 4
    // work-group (x, k) in XCD-aware order: neighbouring tiles share an L2
    const int lin = band_rank(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int kf = lin / gridDim.x, grp = lin - kf * gridDim.x;
    double R[9], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) R[3 * r + c] = poses[12 * kf + 4 * r + c];
        t[r] = poses[12 * kf + 4 * r + 3];
    }
    const float s = gscale[kf];
    const int N = a.W * a.H;
    const float* dimg = depth + (size_t)kf * N;
    const int32_t* aimg = FREEZE ? assoc + (size_t)kf * N * 3 : nullptr;
    float acc[kAdjPart];   // a thread's (at most four pixels per tile) sums; float64 across threads
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) acc[k] = 0.0f;
    double e = 0.0;
    const int tiles_x = (a.W + kAdjTile - 1) / kAdjTile;
    const int ntiles = tiles_x * ((a.H + kAdjTile - 1) / kAdjTile);
    for (int tile = grp; tile < ntiles; tile += a.groups) {
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        const int64_t region = (int64_t)kf * ntiles + tile;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            s_key[threadIdx.x + k * kAdjBlock] = -1;
            s_cnt[threadIdx.x + k * kAdjBlock] = 0;
        }
        __syncthreads();
        int32_t ent[kPer], rank[kPer];
        uint32_t pid[kPer];
        float dep[kPer];
#pragma unroll
        for (int g = 0; g < kPer; g += kLookup) {
            int u[kLookup], v[kLookup];
            bool in[kLookup], ok[kLookup], look[kLookup];
            int32_t slot[kLookup];
            int m[kLookup][3];
            PixelTerm P[kLookup];
#pragma unroll
            for (int j = 0; j < kLookup; ++j) {
                const int px = threadIdx.x + (g + j) * kAdjBlock;
                u[j] = tx * kAdjTile + (px % kAdjTile);
                v[j] = ty * kAdjTile + px / kAdjTile;
                in[j] = u[j] < a.W && v[j] < a.H;
            }
            lookup_batch<kLookup, FREEZE>(M, a, R, t, params, dimg, aimg, u, v, in, ok, look, slot, m, P, &e);
#pragma unroll
            for (int j = 0; j < kLookup; ++j) {
                ent[g + j] = -1;
                rank[g + j] = 0;
                pid[g + j] = (uint32_t)((size_t)kf * N + (size_t)v[j] * a.W + u[j]);
                dep[g + j] = P[j].D;
                if (!ok[j]) continue;
                const ResidualTerms rt = residual_terms(P[j], a.delta, s);
                acc[0] += rt.rho;
#pragma unroll
                for (int k = 0; k < 6; ++k) acc[1 + k] += rt.rp * rt.J[k];
                acc[7] += 1.0f;
                // the block's entry in the tile's table (at most 1024 keys: a
                // free or matching entry is always found)
                const int32_t sl = slot[j];
                uint32_t h = ((uint32_t)sl * 2654435761u) >> 22;
                for (;;) {
                    const int32_t old = atomicCAS(&s_key[h], -1, sl);
                    if (old == -1 || old == sl) break;
                    h = (h + 1) & (kTilePx - 1);
                }
                ent[g + j] = (int32_t)h;
                rank[g + j] = atomicAdd(&s_cnt[h], 1);
            }
        }
        __syncthreads();
        // runs: exclusive scan of the entries' counts (thread t owns entries
        // kPer t .. kPer t + kPer - 1), records in the same order
        int32_t c[kPer], own = 0, used = 0;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            c[k] = s_cnt[kPer * threadIdx.x + k];
            own += c[k];
            used += c[k] > 0 ? 1 : 0;
        }
        int32_t run, rec, tot_px, tot_rec;
        block_scan2(own, used, &run, &rec, &tot_px, &tot_rec, s_w);
        __syncthreads();   // every count is read before s_cnt turns into offsets
        const int64_t base = region * kTilePx;
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            s_cnt[kPer * threadIdx.x + k] = run;
            if (c[k] > 0) {
                const int32_t sl = s_key[kPer * threadIdx.x + k];
                recs[base + rec] = make_int2(sl, c[k]);
                atomicAdd(&pix_count[sl], c[k]);
                atomicAdd(&run_count[sl], 1);
                ++rec;
            }
            run += c[k];
        }
        if (threadIdx.x == 0) nrec[region] = tot_rec;
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kPer; ++j)
            if (ent[j] >= 0)
                list[base + s_cnt[ent[j]] + rank[j]] = make_uint2(pid[j], __float_as_uint(dep[j]));
        __syncthreads();   // the table is cleared for the next tile
    }
    const double x = block_sum_part(acc, s_red);
    if (threadIdx.x < kAdjPart) partials[((size_t)kf * a.groups + grp) * kAdjPart + threadIdx.x] = x;
    if (!FREEZE) return;
    for (int off = 32; off > 0; off >>= 1) e = fmax(e, __shfl_xor(e, off));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double y = 0.0;
        for (int w = 0; w < kAdjBlock / 64; ++w) y = fmax(y, s_max[w]);
        atomicMax(reach, (unsigned long long)__double_as_longlong(y));
    }
}

// Work-group sum of one int32 per thread (all 256 threads), in every thread.
__device__ inline int32_t block_sum_i32(int32_t x, int32_t* s_w) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = x;
    __syncthreads();
    return s_w[0] + s_w[1] + s_w[2] + s_w[3];
}

// Sum of the per-block run counts of each tile of kScanTile blocks.
__global__ __launch_bounds__(256) void k_adj_tile_sums(int64_t nb, const int32_t* __restrict__ counts,
                                                       int32_t* __restrict__ tiles) {
    __shared__ int32_t s_w[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t x = 0;
    for (int k = threadIdx.x; k < kScanTile; k += 256)
        if (base + k < nb) x += counts[base + k];
    x = block_sum_i32(x, s_w);
    if (threadIdx.x == 0) tiles[blockIdx.x] = x;
}

// First run of each block (exclusive prefix sums of the run counts), one
// work-group per tile: the sum of the earlier tiles, then a scan of the
// tile (16 consecutive counts a thread).  Work-group 0 also writes
// max_i |s_i|.
__global__ __launch_bounds__(256) void k_adj_offsets(int64_t nb, const int32_t* __restrict__ counts,
                                                     const int32_t* __restrict__ tiles,
                                                     int32_t* __restrict__ offsets, int32_t K,
                                                     const float* __restrict__ gscale, double* __restrict__ bounds) {
    __shared__ int32_t s_w[8];
    int32_t before = 0;
    if (tiles) {   // null for a single tile
        for (int g = threadIdx.x; g < (int)blockIdx.x; g += 256) before += tiles[g];
        before = block_sum_i32(before, s_w);
    }
    const int64_t i0 = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * 16;
    int32_t c[16];
    int32_t own = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        c[k] = i0 + k < nb ? counts[i0 + k] : 0;
        own += c[k];
    }
    int32_t run, unused, tot, tot2;
    block_scan2(own, 0, &run, &unused, &tot, &tot2, s_w);
    run += before;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (i0 + k < nb) offsets[i0 + k] = run;
        run += c[k];
    }
    if (blockIdx.x != 0) return;
    float smax = 0.0f;
    for (int k = threadIdx.x; k < K; k += 256) smax = fmaxf(smax, fabsf(gscale[k]));
    for (int off = 32; off > 0; off >>= 1) smax = fmaxf(smax, __shfl_xor(smax, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = __float_as_int(smax);   // non-negative: integer order
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t b = s_w[0];
        for (int w = 1; w < 4; ++w) b = s_w[w] > b ? s_w[w] : b;
        bounds[1] = (double)__int_as_float(b);
    }
}

// Each region's records into their blocks' run lists: one wave per region
// (four a work-group); a record's run starts in the region's list at the
// sum of the counts of the records before it; its place among its block's
// runs comes from the block's cursor.
__global__ __launch_bounds__(256) void k_adj_runs(int64_t regions, const int32_t* __restrict__ nrec,
                                                  const int2* __restrict__ recs, const int32_t* __restrict__ run_off,
                                                  int32_t* __restrict__ cursor, int2* __restrict__ runs) {
    const int64_t region = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (region >= regions) return;   // the whole wave
    const int32_t n = nrec[region];
    int32_t start = 0;
    for (int k0 = 0; k0 < n; k0 += 64) {   // uniform over the wave
        const int k = k0 + lane;
        const int2 r = k < n ? recs[region * kTilePx + k] : make_int2(0, 0);
        int32_t incl = r.y;
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t y = __shfl_up(incl, d);
            if (lane >= d) incl += y;
        }
        if (k < n) {
            const int32_t pos = run_off[r.x] + atomicAdd(&cursor[r.x], 1);
            runs[pos] = make_int2((int32_t)(region * kTilePx) + start + incl - r.y, r.y);
        }
        start += __shfl(incl, 63);
    }
}

// The adjoint's voxel sums, one work-group per map block (every
// gridDim.x-th slot below param_blocks): the work-group walks the block's
// runs of the list (up to kRunBatch runs at a time in LDS, thread t taking
// entries t, t + 256, ..., kGatherBatch of them per step with each load of
// a step issued before any is used), recomputes each pixel's point, voxel
// and residual, and adds s rho' and s rho' (q - v) into its voxel's sums in
// LDS; then each voxel's gradient is formed from its sums and added to
// dparams by the one thread that owns the voxel.
//
// The sums are 64-bit fixed point (fixed_term).  With n the pixels of the
// block and s_max = max_i |s_i|, the scale f_p keeps n s_max delta below
// 2^62 and f_q keeps n s_max delta (v_s / 2 + reach + margin) below 2^62
// (|q - v| per axis is at most v_s / 2 for the nearest voxel, plus the
// reach of a frozen association).
// Largest f in [0, 62] with bound 2^f < 2^62 (bound = m 2^e, 1 <= m < 2:
// f = 61 - e).
__device__ inline int fix_scale(double bound) {
    if (!(bound > 0.0)) return 62;
    const int f = 61 - ilogb(bound);
    return f < 0 ? 0 : (f > 62 ? 62 : f);
}

template <bool FREEZE>
__global__ __launch_bounds__(kAdjBlock) void k_backward_gather(MapView M, AdjArgs a, int32_t K,
                                                               const float* __restrict__ depth,
                                                               const double* __restrict__ poses,
                                                               const float4* __restrict__ params,
                                                               const float* __restrict__ gscale,
                                                               const int32_t* __restrict__ assoc,
                                                               const uint2* __restrict__ list,
                                                               const int2* __restrict__ runs,
                                                               const int32_t* __restrict__ pix_count,
                                                               const int32_t* __restrict__ run_count,
                                                               const int32_t* __restrict__ run_off,
                                                               const double* __restrict__ bounds,
                                                               float* __restrict__ dparams) {
    __shared__ unsigned long long sP[kBlockVoxels];
    __shared__ unsigned long long sQ[3][kBlockVoxels];
    __shared__ double s_pose[kPoseLds][12];
    __shared__ float s_s[kPoseLds];
    __shared__ int32_t s_rstart[kRunBatch];
    __shared__ int32_t s_rpre[kRunBatch + 1];
    __shared__ int32_t s_w[8];
    const bool lds_pose = K <= kPoseLds;
    if (lds_pose) {
        for (int k = threadIdx.x; k < K * 12; k += kAdjBlock) s_pose[k / 12][k % 12] = poses[k];
        for (int k = threadIdx.x; k < K; k += kAdjBlock) s_s[k] = gscale[k];
    }
    const double rmax =
        FREEZE ? __longlong_as_double((long long)reinterpret_cast<const unsigned long long*>(bounds)[0]) : 0.0;
    const double smax = bounds[1];
    const double margin = 1e-6 * (1.0 + fabs(a.vs) * 1e3);
    const uint32_t N = (uint32_t)a.W * (uint32_t)a.H;
    const double invN = 1.0 / (double)N, invW = 1.0 / (double)a.W;
    int64_t slot = blockIdx.x;
    int32_t n = slot < a.param_blocks ? pix_count[slot] : 0;
    __syncthreads();

    for (; slot < a.param_blocks; slot += gridDim.x, n = slot < a.param_blocks ? pix_count[slot] : 0) {
        if (n == 0) continue;
        const int32_t nruns = run_count[slot], roff = run_off[slot];
        for (int c = threadIdx.x; c < kBlockVoxels; c += kAdjBlock) {
            sP[c] = 0ull;
            sQ[0][c] = sQ[1][c] = sQ[2][c] = 0ull;
        }
        const double base_p = (double)n * smax * (double)a.delta;
        const int fp = fix_scale(base_p), fq = fix_scale(base_p * (0.5 * a.vs + rmax + margin));
        const float wsp = ldexpf(1.0f, fp), whp = ldexpf(1.0f, fp - 32);
        const float wsq = ldexpf(1.0f, fq), whq = ldexpf(1.0f, fq - 32);
        for (int r0 = 0; r0 < nruns; r0 += kRunBatch) {
            // ---- up to kRunBatch runs: starts and prefix counts in LDS
            const int nr = nruns - r0 < kRunBatch ? nruns - r0 : kRunBatch;
            const int2 run = threadIdx.x < nr ? runs[roff + r0 + threadIdx.x] : make_int2(0, 0);
            int32_t ex, unused, total, tot2;
            block_scan2(run.y, 0, &ex, &unused, &total, &tot2, s_w);   // its barriers order the clears above
            s_rstart[threadIdx.x] = run.x;
            s_rpre[threadIdx.x] = ex;
            if (threadIdx.x == 0) s_rpre[kRunBatch] = total;
            __syncthreads();
            int rc = 0;   // this thread's run (its entries only grow)
            for (int j0 = threadIdx.x; j0 < total; j0 += kAdjBlock * kGatherBatch) {
                uint2 le[kGatherBatch];
                bool live[kGatherBatch];
#pragma unroll
                for (int b = 0; b < kGatherBatch; ++b) {
                    const int j = j0 + b * kAdjBlock;
                    live[b] = j < total;
                    le[b] = make_uint2(0u, 0u);
                    if (!live[b]) continue;
                    while (rc + 1 < nr && j >= s_rpre[rc + 1]) ++rc;
                    le[b] = list[s_rstart[rc] + (j - s_rpre[rc])];
                }
                int m[kGatherBatch][3];
                uint32_t kk[kGatherBatch];
                int uu[kGatherBatch], vv[kGatherBatch];
#pragma unroll
                for (int b = 0; b < kGatherBatch; ++b) {
                    if (!live[b]) continue;
                    // keyframe, row and column of the pixel id (the float64
                    // quotients are within 1 of the integer ones)
                    const uint32_t p = le[b].x;
                    int32_t kf = (int32_t)((double)p * invN);
                    int32_t i = (int32_t)(p - (uint32_t)kf * N);
                    if (i < 0) {
                        --kf;
                        i += (int32_t)N;
                    } else if (i >= (int32_t)N) {
                        ++kf;
                        i -= (int32_t)N;
                    }
                    int32_t v = (int32_t)((double)i * invW);
                    int32_t u = i - v * a.W;
                    if (u < 0) {
                        --v;
                        u += a.W;
                    } else if (u >= a.W) {
                        ++v;
                        u -= a.W;
                    }
                    kk[b] = (uint32_t)kf;
                    uu[b] = u;
                    vv[b] = v;
                    if (FREEZE) {
                        const int32_t* as = assoc + (size_t)p * 3;
                        m[b][0] = as[0];
                        m[b][1] = as[1];
                        m[b][2] = as[2];
                    }
                }
                float4 pr[kGatherBatch];
                float qf[kGatherBatch][3], dq[kGatherBatch][3];
                float sv[kGatherBatch];
#pragma unroll
                for (int b = 0; b < kGatherBatch; ++b) {
                    if (!live[b]) continue;
                    const uint32_t kf = kk[b];
                    double R[9], t[3];
                    if (lds_pose) {
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) R[3 * r + c] = s_pose[kf][4 * r + c];
                            t[r] = s_pose[kf][4 * r + 3];
                        }
                        sv[b] = s_s[kf];
                    } else {
#pragma unroll
                        for (int r = 0; r < 3; ++r) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) R[3 * r + c] = poses[12 * kf + 4 * r + c];
                            t[r] = poses[12 * kf + 4 * r + 3];
                        }
                        sv[b] = gscale[kf];
                    }
                    double q[3];
                    pixel_point(a, R, t, __uint_as_float(le[b].y), uu[b], vv[b], q);
                    if (!FREEZE) nearest_voxel(a, q, m[b]);
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        qf[b][r] = (float)q[r];
                        dq[b][r] = (float)(q[r] - a.vs * (double)m[b][r]);
                    }
                    pr[b] = params[slot * kBlockVoxels + morton9(m[b][0] & 7, m[b][1] & 7, m[b][2] & 7)];
                }
#pragma unroll
                for (int b = 0; b < kGatherBatch; ++b) {
                    if (!live[b]) continue;
                    const float4 pv = pr[b];
                    const float n2 = pv.y * pv.y + pv.z * pv.z + pv.w * pv.w;
                    if (!(n2 > 0.0f)) continue;   // not taken: the pixel pass checked it
                    PixelTerm P;
                    P.inv_ng = 1.0f / sqrtf(n2);
                    P.psi = pv.x;
                    P.gh[0] = pv.y * P.inv_ng;
                    P.gh[1] = pv.z * P.inv_ng;
                    P.gh[2] = pv.w * P.inv_ng;
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        P.q[r] = qf[b][r];
                        P.dq[r] = dq[b][r];
                    }
                    const ResidualTerms rt = residual_terms(P, a.delta, sv[b]);
                    const int c = (m[b][0] & 7) | ((m[b][1] & 7) << 3) | ((m[b][2] & 7) << 6);
                    atomicAdd(&sP[c], fixed_term(wsp, whp, rt.rp));
#pragma unroll
                    for (int k = 0; k < 3; ++k) atomicAdd(&sQ[k][c], fixed_term(wsq, whq, rt.rp * P.dq[k]));
                }
            }
            __syncthreads();   // the run table is rewritten by the next batch
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

size_t gsdf_keyframe_scratch_bytes(const gsdf_camera* cam, int32_t n_keyframes, int64_t param_blocks) {
    if (!valid_cam(cam) || n_keyframes <= 0 || n_keyframes > 65535 || param_blocks < 0) return 0;
    const int64_t tiles = adj_tiles(cam->width, cam->height);
    if ((int64_t)n_keyframes * tiles * kTilePx > (int64_t)INT32_MAX) return 0;   // list entries are int32
    return adj_scratch(n_keyframes, tiles, param_blocks).total;
}

static int keyframe_common(const gsdf_map* map, const float* depth_dev, int32_t K, const gsdf_camera* cam,
                           const double* T0_dev, const double* xi_dev, const float* params_dev,
                           int64_t param_blocks, float huber_delta, void* scratch, size_t scratch_bytes) {
    if (!valid_map(map) || !valid_cam(cam) || K <= 0 || K > 65535 || !depth_dev || !T0_dev || !xi_dev ||
        !params_dev || param_blocks < 0 || param_blocks > map->desc.max_blocks || !(huber_delta > 0.0f) || !scratch)
        return GSDF_EINVAL;
    const size_t need = gsdf_keyframe_scratch_bytes(cam, K, param_blocks);
    if (need == 0 || scratch_bytes < need) return GSDF_EINVAL;
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
    const AdjScratch L = adj_scratch(n_keyframes, adj_tiles(cam->width, cam->height), param_blocks);
    char* base = (char*)scratch;
    double* partials = (double*)(base + L.partials);
    double* poses = (double*)(base + L.poses);
    k_adj_setup<<<ceil_div(n_keyframes, 64), 64, 0, s>>>(n_keyframes, T0_dev, xi_dev, poses, 0, nullptr, nullptr,
                                                        nullptr, nullptr);
    {
        TimedLaunch tl(map->timer, GSDF_K_LOSS, s);
        const dim3 grid(a.groups, n_keyframes);
        const float4* P = reinterpret_cast<const float4*>(params_dev);
        if (freeze)
            k_keyframe_loss<true><<<grid, kAdjBlock, 0, s>>>(make_view(*map), a, depth_dev, poses, P, assoc_dev,
                                                             partials);
        else
            k_keyframe_loss<false><<<grid, kAdjBlock, 0, s>>>(make_view(*map), a, depth_dev, poses, P, assoc_dev,
                                                              partials);
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
    const int K = n_keyframes;
    const int64_t ntiles = adj_tiles(cam->width, cam->height);
    const AdjArgs a = adj_args(*map, *cam, huber_delta, freeze, param_blocks);
    const AdjScratch L = adj_scratch(K, ntiles, param_blocks);
    char* base = (char*)scratch;
    double* partials = (double*)(base + L.partials);
    double* poses = (double*)(base + L.poses);
    double* bounds = (double*)(base + L.bounds);
    unsigned long long* reach = (unsigned long long*)bounds;
    uint2* list = (uint2*)(base + L.list);
    int2* recs = (int2*)(base + L.recs);
    int32_t* nrec = (int32_t*)(base + L.nrec);
    int2* runs = (int2*)(base + L.runs);
    int32_t* pix_count = (int32_t*)(base + L.pix_count);
    int32_t* run_count = (int32_t*)(base + L.run_count);
    int32_t* run_off = (int32_t*)(base + L.run_off);
    int32_t* cursor = (int32_t*)(base + L.cursor);
    int32_t* tiles = (int32_t*)(base + L.tiles);
    const MapView M = make_view(*map);
    const float4* P = reinterpret_cast<const float4*>(params_dev);
    const int64_t nb = param_blocks;
    const int nscan = (int)ceil_div(nb, (int64_t)kScanTile);
    const int groups = (int)(nb < kBackGroups ? nb : kBackGroups);
    const int64_t setup_n = nb > K ? nb : K;
    const dim3 pgrid(a.groups, K);
    {
        TimedLaunch tl(map->timer, GSDF_K_BACKWARD, s);
        k_adj_setup<<<(unsigned)ceil_div(setup_n, (int64_t)256), 256, 0, s>>>(K, T0_dev, xi_dev, poses, nb, pix_count,
                                                                           run_count, cursor, reach);
        if (freeze)
            k_adj_pixels<true><<<pgrid, kAdjBlock, 0, s>>>(M, a, depth_dev, poses, P, grad_loss_dev, assoc_dev, list,
                                                           recs, nrec, pix_count, run_count, reach, partials);
        else
            k_adj_pixels<false><<<pgrid, kAdjBlock, 0, s>>>(M, a, depth_dev, poses, P, grad_loss_dev, nullptr, list,
                                                            recs, nrec, pix_count, run_count, reach, partials);
        if (nb > 0) {
            if (nscan > 1) k_adj_tile_sums<<<nscan, 256, 0, s>>>(nb, run_count, tiles);
            k_adj_offsets<<<nscan, 256, 0, s>>>(nb, run_count, nscan > 1 ? tiles : nullptr, run_off, K,
                                                grad_loss_dev, bounds);
            const int64_t regions = (int64_t)K * ntiles;
            k_adj_runs<<<(unsigned)ceil_div(regions, (int64_t)4), 256, 0, s>>>(regions, nrec, recs, run_off, cursor,
                                                                               runs);
            if (freeze)
                k_backward_gather<true><<<groups, kAdjBlock, 0, s>>>(M, a, K, depth_dev, poses, P, grad_loss_dev,
                                                                     assoc_dev, list, runs, pix_count, run_count,
                                                                     run_off, bounds, dparams_dev);
            else
                k_backward_gather<false><<<groups, kAdjBlock, 0, s>>>(M, a, K, depth_dev, poses, P, grad_loss_dev,
                                                                      nullptr, list, runs, pix_count, run_count,
                                                                      run_off, bounds, dparams_dev);
        }
        k_keyframe_finish<<<K, 256, 0, s>>>(a.groups, xi_dev, partials, loss_dev, dxi_dev, nullptr);
    }
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
