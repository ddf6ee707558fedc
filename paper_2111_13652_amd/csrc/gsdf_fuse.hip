// integrate_frame: normals from a 5x5 plane fit, the viewing-angle filter,
// and the running weighted average of SDF and gradient, Eq. (1)-(3) of
// Gradient-SDF (Sec. 3.1, 3.2), driven by depth pixels as in the Sec. 5.3
// setup.
//
// Two kernels (the frame path runs the first together with allocation, as
// k_alloc_normals).
//  1. k_pixel_normals: one work-group per 16x16 pixel tile with its 2-pixel
//     halo staged in LDS; every pixel gets its world-frame normal and depth
//     (float4), or zeros when it fails the window or the angle test.
//  2. k_fuse_blocks: one work-group per block touched by the frame (the
//     allocation step flags them).  It projects the block's box into the
//     image, walks the pixels of that rectangle, clips each pixel's ray to
//     the box to find the few band samples that can land inside, evaluates
//     exactly those samples with the binary32 band rule, and adds w d, w n_w
//     and w into a 512-voxel accumulator in LDS.  The block then writes each
//     voxel it changed once.  Each block is owned by one work-group per
//     frame, so no global atomics are needed and every touched voxel costs
//     one read and one write of its record.
//
// FP32 storage keeps, per voxel, float4 {sum w d, g_x, g_y, g_z} and W:
// psi = (sum w d) / W is Eq. (1)-(2) unrolled over all observations and g
// is Eq. (3) exactly, so the write is an addition.  16-bit storage keeps
// {psi/T, gbar} (gbar = g / W, bounded) and applies Eq. (1)-(3) with the
// frame's sums before rounding once.  The gradient-free storage keeps
// {sum w d} and W only: the same distance sums as FP32 storage, without
// the three gradient sums (Eq. (3)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include <climits>

#include "gsdf_alloc.hpp"
#include "gsdf_common.hpp"
#include "gsdf_fixed.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

constexpr int kTile = 16;
constexpr int kHalo = 2;
constexpr int kTileH = kTile + 2 * kHalo;
constexpr int kFuseBlock = 256;
constexpr int kFuseChunk = 2048;   // box pixels scanned per pass (LDS queue capacity)
constexpr int kFuseGroups = 4096;
constexpr int kShortRun = 8;       // queue entries with at most this many band samples count as short
constexpr float kBoxMargin = 1e-4f;  // metres; far above binary32 rounding of coordinates

struct FuseConsts {
    BandConsts band;
    float fxf, fyf, rcx, rcy;     // float32 intrinsics for the normal fit
    double fx_d, fy_d, ifx_d, ify_d, cx_d, cy_d;
    float zmin, zmax;
    float eps, cos_min;
    float inv_span;   // 1 / (T - eps), the slope of the linear weight
    double inv_vs_d, vs_d;
    float vs_f, T_f;
    float inv_df;   // 1 / band sample spacing
    int W, H;
    float fix_scale;     // 2^f: fixed-point scale of the per-frame voxel sums
    double fix_inv;      // 2^-f
};

// w(d) = 1 for d <= eps, (T - d) / (T - eps) for eps < d < T, 0 for d >= T,
// written as the clamp of the middle piece (the same function, no branches)
__device__ inline float linear_weight(float d, float T, float inv_span) {
    return fminf(1.0f, fmaxf(0.0f, (T - d) * inv_span));
}

// ---------------------------------------------------------------------------
// 1. Normals
// ---------------------------------------------------------------------------
// Tile (tu, tv) of 16x16 pixels; every thread of the 256-thread work-group
// must call it (it synchronises); tile and itile are kTileH x (kTileH + 1)
// floats of LDS (depths and their reciprocals, each computed once per tile).
__device__ inline void normals_tile(const float* __restrict__ depth, const FuseConsts& fc,
                                    const double* __restrict__ Twc, float4* __restrict__ pix, int tu, int tv,
                                    float (*tile)[kTileH + 1], float (*itile)[kTileH + 1]) {
    const int tx = threadIdx.x & (kTile - 1);
    const int ty = threadIdx.x / kTile;
    const int u0 = tu * kTile - kHalo;
    const int v0 = tv * kTile - kHalo;
    for (int i = threadIdx.x; i < kTileH * kTileH; i += blockDim.x) {
        const int ly = i / kTileH, lx = i % kTileH;
        const int uu = u0 + lx, vv = v0 + ly;
        float d = 0.0f;
        if (uu >= 0 && uu < fc.W && vv >= 0 && vv < fc.H) d = depth[(size_t)vv * fc.W + uu];
        tile[ly][lx] = d;
        itile[ly][lx] = d > 0.0f ? 1.0f / d : 0.0f;
    }
    __syncthreads();

    const int u = tu * kTile + tx;
    const int v = tv * kTile + ty;
    if (u >= fc.W || v >= fc.H) return;  // no barrier follows
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    const float Dc = tile[ty + kHalo][tx + kHalo];
    if (u >= kHalo && v >= kHalo && u < fc.W - kHalo && v < fc.H - kHalo &&
        depth_ok(Dc, fc.zmin, fc.zmax)) {
        // least-squares plane 1/z = a . [x/z, y/z, 1] on the 5x5 window.
        // Over the symmetric window the design (1, du, dv) is orthogonal, so
        // the fit has a closed form in the centred inverse depths
        // 1/D_i - 1/D_c = (D_c - D_i) (1/D_c) (1/D_i), whose numerators are
        // exact (no cancellation; the reciprocals come from the tile).
        const float iDc = itile[ty + kHalo][tx + kHalo];
        float s0 = 0.0f, sa = 0.0f, sb = 0.0f;
        bool ok = true;
#pragma unroll
        for (int dv = -kHalo; dv <= kHalo; ++dv) {
#pragma unroll
            for (int du = -kHalo; du <= kHalo; ++du) {
                const float Di = tile[ty + kHalo + dv][tx + kHalo + du];
                ok = ok && depth_ok(Di, fc.zmin, fc.zmax) && (fabsf(Di - Dc) <= fc.band.Tf);
                const float dy = (Dc - Di) * iDc * itile[ty + kHalo + dv][tx + kHalo + du];
                s0 += dy;
                sa += (float)du * dy;
                sb += (float)dv * dy;
            }
        }
        if (ok) {
            const float h = iDc + s0 * (1.0f / 25.0f);
            const float alpha = sa * (1.0f / 50.0f);   // sum du^2 = 50 over the window
            const float beta = sb * (1.0f / 50.0f);
            const float ax = alpha * fc.fxf;
            const float ay = beta * fc.fyf;
            const float az = h - alpha * ((float)u - fc.rcx) - beta * ((float)v - fc.rcy);
            const float na = sqrtf(ax * ax + ay * ay + az * az);
            const float rx = ((float)u - fc.rcx) * fc.band.ifx;
            const float ry = ((float)v - fc.rcy) * fc.band.ify;
            const float ina = 1.0f / na;
            const float cosang = h * ina * __frsqrt_rn(rx * rx + ry * ry + 1.0f);
            if (cosang >= fc.cos_min) {
                // a . ray = h > 0: the normal faces away from the camera
                const float n0 = ax * ina, n1 = ay * ina, n2 = az * ina;
                float nw[3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    nw[i] = (float)Twc[4 * i] * n0 + (float)Twc[4 * i + 1] * n1 + (float)Twc[4 * i + 2] * n2;
                out = make_float4(nw[0], nw[1], nw[2], Dc);
            }
        }
    }
    pix[(size_t)v * fc.W + u] = out;
}

__global__ __launch_bounds__(256) void k_pixel_normals(const float* __restrict__ depth, FuseConsts fc,
                                                       const double* __restrict__ Twc,
                                                       float4* __restrict__ pix) {
    __shared__ float tile[kTileH][kTileH + 1];
    __shared__ float itile[kTileH][kTileH + 1];
    normals_tile(depth, fc, Twc, pix, blockIdx.x, blockIdx.y, tile, itile);
}

// The frame path's allocation and normals in one launch: both work on the
// same 16x16 tiles of the same depth image and pose and are independent of
// each other (allocation never reads a normal), so each work-group runs the
// tile's allocation and then its normals.
__global__ __launch_bounds__(256) void k_alloc_normals(MapView M, const float* __restrict__ depth, FuseConsts fc,
                                                       const double* __restrict__ Twc, float4* __restrict__ pix,
                                                       int32_t* status) {
    __shared__ unsigned long long s_keys[kAllocSet];
    __shared__ unsigned long long red[4];
    __shared__ float tile[kTileH][kTileH + 1];
    __shared__ float itile[kTileH][kTileH + 1];
    allocate_tile(M, depth, fc.W, fc.H, fc.zmin, fc.zmax, fc.band, Twc, status, blockIdx.x, blockIdx.y, s_keys,
                  red);
    normals_tile(depth, fc, Twc, pix, blockIdx.x, blockIdx.y, tile, itile);
}

// ---------------------------------------------------------------------------
// 2. Per-block gather
// ---------------------------------------------------------------------------
struct BlockBox {
    int u0, u1, v0, v1;       // inclusive pixel rectangle (u1 < u0: empty)
    float lo[3], hi[3];       // box relative to the camera centre, with margin
    float zmin, zmax;         // camera-frame depth range of the box corners
    float inv_bw;             // 1 / rectangle width
};

// Called by lanes 0..7 of wave 0 together, one box corner each (on one
// lane the eight projections are a long dependent float64 chain); lane 0
// writes the result.
__device__ inline void block_box(const FuseConsts& fc, const double* R, const double* t, int bx,
                                 int by, int bz, BlockBox* B) {
    const int b[3] = {bx, by, bz};
    double lo[3], hi[3], mag = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lo[i] = fc.vs_d * (8.0 * b[i] - 0.5);
        hi[i] = fc.vs_d * (8.0 * b[i] + 7.5);
        mag = fmax(mag, fmax(fabs(lo[i]), fabs(hi[i])) + fabs(t[i]));
    }
    // the margin stays far above the binary32 rounding of sample positions
    // (a few ulps of the coordinate magnitude)
    const double margin = kBoxMargin + 4e-6 * mag;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lo[i] -= margin;
        hi[i] += margin;
    }
    // corner c of the box: its camera-frame point and pixel; the extremes
    // over the 8 corners by shuffles within the 8 lanes
    double umin, umax, vmin, vmax, zlo, zhi;
    bool behind;
    {
        const int c = threadIdx.x & 7;
        const double X[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
        double pc[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            pc[j] = R[j] * (X[0] - t[0]) + R[3 + j] * (X[1] - t[1]) + R[6 + j] * (X[2] - t[2]);
        // reciprocal (hardware estimate and one Newton step) instead of two
        // divisions: the rectangle is widened by a pixel on each side anyway
        // (a corner behind the camera gives a meaningless value here, and
        // the whole image is used then)
        double iz = __builtin_amdgcn_rcp(pc[2]);
        iz = fma(iz, fma(-pc[2], iz, 1.0), iz);
        const double u = fc.fx_d * pc[0] * iz + fc.cx_d;
        const double v = fc.fy_d * pc[1] * iz + fc.cy_d;
        umin = umax = u;
        vmin = vmax = v;
        zlo = zhi = pc[2];
        behind = pc[2] <= 1e-6;
#pragma unroll
        for (int m = 1; m < 8; m <<= 1) {
            umin = fmin(umin, __shfl_xor(umin, m, 8));
            umax = fmax(umax, __shfl_xor(umax, m, 8));
            vmin = fmin(vmin, __shfl_xor(vmin, m, 8));
            vmax = fmax(vmax, __shfl_xor(vmax, m, 8));
            zlo = fmin(zlo, __shfl_xor(zlo, m, 8));
            zhi = fmax(zhi, __shfl_xor(zhi, m, 8));
            behind = behind || __shfl_xor((int)behind, m, 8);
        }
    }
    if (threadIdx.x != 0) return;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        B->lo[i] = (float)(lo[i] - t[i]);
        B->hi[i] = (float)(hi[i] - t[i]);
    }
    B->zmin = (float)zlo;
    B->zmax = (float)zhi;
    if (behind) {
        B->u0 = 0;
        B->u1 = fc.W - 1;
        B->v0 = 0;
        B->v1 = fc.H - 1;
        B->inv_bw = 1.0f / (float)fc.W;
        return;
    }
    // clamp in double before converting: far-off projections stay in range
    B->u0 = (int)fmin(fmax(0.0, floor(umin) - 1.0), (double)fc.W);
    B->u1 = (int)fmax(fmin((double)(fc.W - 1), ceil(umax) + 1.0), -1.0);
    B->v0 = (int)fmin(fmax(0.0, floor(vmin) - 1.0), (double)fc.H);
    B->v1 = (int)fmax(fmin((double)(fc.H - 1), ceil(vmax) + 1.0), -1.0);
    B->inv_bw = B->u1 >= B->u0 ? 1.0f / (float)(B->u1 - B->u0 + 1) : 0.0f;
}

// Per-frame voxel sums are fixed point with f fraction bits (fixed_term,
// gsdf_fixed.hpp); f is chosen on the host so that the largest possible sum
// fits (see fix_bits).

template <int STORAGE>
__global__ __launch_bounds__(kFuseBlock) void k_fuse_blocks(MapView M, const float4* __restrict__ pix,
                                                           FuseConsts fc, const double* __restrict__ Twc,
                                                           int32_t* status) {
    // per-voxel sums of the frame in fixed point (see fixed_term), indexed
    // lx + 8 ly + 64 lz (the pool's Morton order is applied at the write):
    // integer additions are associative, so the sums (and the map) do not
    // depend on the order in which the work-group's threads add their updates
    constexpr bool kGrad = STORAGE != GSDF_NOGRAD_FP32;
    __shared__ unsigned long long aS[kBlockVoxels];
    __shared__ unsigned long long aG[kGrad ? 3 : 1][kGrad ? kBlockVoxels : 1];
    __shared__ unsigned long long aW[kBlockVoxels];
    __shared__ BlockBox box;
    __shared__ uint32_t q_pix[kFuseChunk];
    __shared__ uint32_t q_k[kFuseChunk];
    __shared__ int q_count[2];   // short entries from the front, long ones from the back

    if (!pose_finite(Twc)) {   // nothing is fused at a non-finite pose
        if (blockIdx.x == 0 && threadIdx.x == 0) raise_status(status, GSDF_EINVAL);
        return;
    }
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = Twc[4 * i + j];
        t[i] = Twc[4 * i + 3];
    }
    const float Rf[9] = {(float)R[0], (float)R[1], (float)R[2], (float)R[3], (float)R[4],
                         (float)R[5], (float)R[6], (float)R[7], (float)R[8]};
    // camera-relative float32 pose for 16-bit storage: voxel nearest the
    // camera centre and the remainder of the translation
    int mc[3];
    float trf[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        mc[i] = (int)floor(t[i] * fc.inv_vs_d + 0.5);
        trf[i] = (float)(t[i] - fc.vs_d * (double)mc[i]);
    }
    const float ivsf = (float)fc.inv_vs_d;
    const BandRule br = make_band_rule(Twc, fc.band.ifx, fc.band.ify, fc.band.cxf, fc.band.cyf,
                                       fc.band.invvs, fc.band.Tf, fc.band.Df, fc.band.nsamples);
    int n_blocks = M.counters[kNumBlocks];
    n_blocks = n_blocks < M.max_blocks ? n_blocks : M.max_blocks;
    unsigned long long my_updates = 0, my_visits = 0, my_voxels = 0, my_blocks = 0;
    // The newest blocks (highest slots: usually nearest the camera, with
    // the largest boxes) are taken first, so the longest work-groups do not
    // start last.
    for (int item = blockIdx.x; item < n_blocks; item += gridDim.x) {
        const int slot = n_blocks - 1 - item;
        if (M.touched_flag[slot] == 0) continue;   // uniform across the work-group
        ++my_blocks;
        int bx, by, bz;
        unpack_key(M.block_keys[slot], &bx, &by, &bz);
        for (int c = threadIdx.x; c < kBlockVoxels; c += kFuseBlock) {
            aS[c] = 0ull;
            if constexpr (kGrad) {
                aG[0][c] = 0ull;
                aG[1][c] = 0ull;
                aG[2][c] = 0ull;
            }
            aW[c] = 0ull;
        }
        if (threadIdx.x < 8) block_box(fc, R, t, bx, by, bz, &box);
        __syncthreads();

        const int bw = box.u1 - box.u0 + 1;
        const int bh = box.v1 - box.v0 + 1;
        const int npx = (bw > 0 && bh > 0) ? bw * bh : 0;
        const float inv_bw = box.inv_bw;
        // the depth band [D - T, D + T] must reach the box's depth range
        const float zreach_lo = box.zmin - fc.band.Tf - fc.band.Df;
        const float zreach_hi = box.zmax + fc.band.Tf + fc.band.Df;
        const float last = (float)(fc.band.nsamples - 1);
        const float inv_df = fc.inv_df;

        // The box is gathered in chunks of kFuseChunk pixels, each in two
        // phases.  Scan: every thread tests pixels of the chunk against the
        // block (depth reach, ray/box slab, band samples inside) and the
        // survivors go to an LDS queue with their sample range.  Fuse: the
        // queue is worked densely, so the sample loop and the LDS atomics run
        // with most lanes busy (a thread-per-pixel loop over the box leaves
        // three lanes in four idle).
        for (int c0 = 0; c0 < npx; c0 += kFuseChunk) {
            const int cn = min(kFuseChunk, npx - c0);
            if (threadIdx.x < 2) q_count[threadIdx.x] = 0;
            __syncthreads();
            for (int p = threadIdx.x; p < cn; p += kFuseBlock) {
                const int q = c0 + p;
                // row and column without an integer division (q < 2^24 is exact)
                int row = (int)(((float)q + 0.5f) * inv_bw);
                int col = q - row * bw;
                if (col < 0) {
                    --row;
                    col += bw;
                } else if (col >= bw) {
                    ++row;
                    col -= bw;
                }
                const int u = box.u0 + col;
                const int v = box.v0 + row;
                const float D = pix[(size_t)v * fc.W + u].w;
                bool keep = D > 0.0f && D >= zreach_lo && D <= zreach_hi;
                int k0 = 0, k1 = -1;
                if (keep) {
                    ++my_visits;
                    // clip the pixel's ray z * (R ray) to the block's box (the
                    // box's margin absorbs the approximate reciprocals)
                    const float xr = pixel_xr(br, u);
                    const float yr = pixel_yr(br, v);
                    float zin = 0.0f, zout = 3.0e38f;
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const float dir = Rf[3 * i] * xr + Rf[3 * i + 1] * yr + Rf[3 * i + 2];
                        if (fabsf(dir) < 1e-20f) {
                            if (box.lo[i] > 0.0f || box.hi[i] < 0.0f) zout = -1.0f;
                        } else {
                            const float id = __builtin_amdgcn_rcpf(dir);
                            const float a = box.lo[i] * id, b = box.hi[i] * id;
                            zin = fmaxf(zin, fminf(a, b));
                            zout = fminf(zout, fmaxf(a, b));
                        }
                    }
                    // samples inside the box widened by kBoxMargin: no other
                    // sample can land in a voxel of this block (binary32
                    // rounding of a sample's position is far below the
                    // margin), so the run structure of the consecutive-repeat
                    // rule inside the block is the same as over the whole band
                    const float zb0 = D - fc.band.Tf;  // first band sample
                    keep = zin <= zout;
                    if (keep) {
                        k0 = (int)fmaxf(0.0f, ceilf(fminf((zin - zb0) * inv_df, last + 1.0f)));
                        k1 = (int)fminf(last, floorf(fmaxf((zout - zb0) * inv_df, -1.0f)));
                        keep = k0 <= k1;
                    }
                }
                // wave-level compaction into the queue: entries with at most
                // kShortRun samples fill it from the front, longer ones from
                // the back, so a wave of the fuse phase takes entries of one
                // kind and its sample loop leaves fewer lanes idle
                const bool is_long = k1 - k0 >= kShortRun;
                const int lane = threadIdx.x & 63;
#pragma unroll
                for (int kind = 0; kind < 2; ++kind) {
                    const bool mine = keep && (is_long == (kind == 1));
                    const unsigned long long ballot = __ballot(mine);
                    if (!ballot) continue;
                    const int leader = __ffsll((long long)ballot) - 1;
                    int base = 0;
                    if (lane == leader) base = atomicAdd(&q_count[kind], __popcll(ballot));
                    base = __shfl(base, leader);
                    if (mine) {
                        const int r = base + __popcll(ballot & ((1ull << lane) - 1ull));
                        const int slot_q = kind == 0 ? r : kFuseChunk - 1 - r;
                        q_pix[slot_q] = ((uint32_t)v << 16) | (uint32_t)u;   // u, v < 2^16
                        q_k[slot_q] = (uint32_t)(k0 | (k1 << 16));
                    }
                }
            }
            __syncthreads();
            const int nq0 = q_count[0], nq1 = q_count[1];
            // lane-major order within each kind: the lanes of a wave take
            // entries n/64 apart (different rows of the box), so the LDS
            // atomics of one instruction rarely hit the same voxel; a wave's
            // row of 64 entries lies within one kind
            const int ls0 = (nq0 + 63) / 64, ls1 = (nq1 + 63) / 64;
            for (int p = threadIdx.x; p < (ls0 + ls1) * 64; p += kFuseBlock) {
                const int row = p >> 6;
                int e;
                if (row < ls0) {
                    e = (p & 63) * ls0 + row;
                    if (e >= nq0) continue;
                } else {
                    e = (p & 63) * ls1 + (row - ls0);
                    if (e >= nq1) continue;
                    e = kFuseChunk - 1 - e;
                }
                const uint32_t uv = q_pix[e];
                const int k0 = (int)(q_k[e] & 0xffffu), k1 = (int)(q_k[e] >> 16);
                const int v = (int)(uv >> 16);
                const int u = (int)(uv & 0xffffu);
                const float4 px = pix[(size_t)v * fc.W + u];
                const float D = px.w;
                const float xr = pixel_xr(br, u);
                const float yr = pixel_yr(br, v);
                // observed point as an offset from a nearby voxel: formed in
                // float64 for FP32 storage; camera-relative float32 for 16-bit
                // storage (q - v_s m_c = R x + t_r, |t_r| < v_s)
                int mref[3];
                float prel[3];
                if (STORAGE == GSDF_FP32 || STORAGE == GSDF_NOGRAD_FP32) {
                    const double Dd = (double)D;
                    const double x0 = Dd * (((double)u - fc.cx_d) * fc.ifx_d);
                    const double x1 = Dd * (((double)v - fc.cy_d) * fc.ify_d);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const double q = R[3 * i] * x0 + R[3 * i + 1] * x1 + R[3 * i + 2] * Dd + t[i];
                        mref[i] = (int)floor(q * fc.inv_vs_d + 0.5);
                        prel[i] = (float)(q - fc.vs_d * (double)mref[i]);
                    }
                } else {
                    const float x0 = D * (((float)u - fc.rcx) / fc.fxf);
                    const float x1 = D * (((float)v - fc.rcy) / fc.fyf);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const float qc = Rf[3 * i] * x0 + Rf[3 * i + 1] * x1 + Rf[3 * i + 2] * D + trf[i];
                        const int dm = (int)floorf(qc * ivsf + 0.5f);
                        mref[i] = mc[i] + dm;
                        prel[i] = qc - fc.vs_f * (float)dm;
                    }
                }
                int pm[3] = {INT_MIN, INT_MIN, INT_MIN};
                for (int k = k0; k <= k1; ++k) {
                    int m[3];
                    if (!band_sample(br, xr, yr, D, k, m)) continue;
                    if (m[0] == pm[0] && m[1] == pm[1] && m[2] == pm[2]) continue;
                    pm[0] = m[0];
                    pm[1] = m[1];
                    pm[2] = m[2];
                    if (block_of(m[0]) != bx || block_of(m[1]) != by || block_of(m[2]) != bz) continue;
                    float off[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) off[i] = fc.vs_f * (float)(m[i] - mref[i]) - prel[i];
                    float d = px.x * off[0] + px.y * off[1] + px.z * off[2];
                    d = fminf(fc.T_f, fmaxf(-fc.T_f, d));
                    const float w = linear_weight(d, fc.T_f, fc.inv_span);
                    if (!(w > 0.0f)) continue;
                    const int c = (m[0] & 7) | ((m[1] & 7) << 3) | ((m[2] & 7) << 6);  // lx + 8 ly + 64 lz
                    const float ws = w * fc.fix_scale, wh = ws * 2.3283064365386963e-10f;
                    atomicAdd(&aS[c], fixed_term(ws, wh, d));
                    if constexpr (kGrad) {
                        atomicAdd(&aG[0][c], fixed_term(ws, wh, px.x));
                        atomicAdd(&aG[1][c], fixed_term(ws, wh, px.y));
                        atomicAdd(&aG[2][c], fixed_term(ws, wh, px.z));
                    }
                    atomicAdd(&aW[c], fixed_term(ws, wh, 1.0f));
                    ++my_updates;
                }
            }
            __syncthreads();
        }

        // write the voxels this frame changed: this work-group owns the block.
        // A thread reads all of its voxels before it writes any, so their
        // loads are in flight together.
        constexpr int kPerThread = kBlockVoxels / kFuseBlock;
        static_assert(kBlockVoxels % kFuseBlock == 0, "every thread writes the same number of voxels");
        float sw[kPerThread], sS[kPerThread], sG[kPerThread][3], Wold[kPerThread], d1[kPerThread];
        int64_t vi[kPerThread];
        bool on[kPerThread];
        float4 r32[kPerThread];
        ushort4 r16[kPerThread];
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int c = threadIdx.x + j * kFuseBlock;
            sw[j] = from_fixed(aW[c], fc.fix_inv);
            on[j] = sw[j] > 0.0f;
            if (!on[j]) continue;
            sS[j] = from_fixed(aS[c], fc.fix_inv);
            vi[j] = (int64_t)slot * kBlockVoxels + morton9(c & 7, (c >> 3) & 7, c >> 6);
            if constexpr (kGrad) {
#pragma unroll
                for (int i = 0; i < 3; ++i) sG[j][i] = from_fixed(aG[i][c], fc.fix_inv);
            }
            if constexpr (!kGrad)
                d1[j] = reinterpret_cast<const float*>(M.vox)[vi[j]];
            else if (STORAGE == GSDF_FP32)
                r32[j] = reinterpret_cast<const float4*>(M.vox)[vi[j]];
            else
                r16[j] = reinterpret_cast<const ushort4*>(M.vox)[vi[j]];
            Wold[j] = M.weight[vi[j]];
        }
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            if (!on[j]) continue;
            ++my_voxels;
            if constexpr (!kGrad) {
                reinterpret_cast<float*>(M.vox)[vi[j]] = d1[j] + sS[j];
                M.weight[vi[j]] = Wold[j] + sw[j];
                continue;
            }
            if (STORAGE == GSDF_FP32) {
                float4 r = r32[j];
                r.x += sS[j];
                r.y += sG[j][0];
                r.z += sG[j][1];
                r.w += sG[j][2];
                reinterpret_cast<float4*>(M.vox)[vi[j]] = r;
                M.weight[vi[j]] = Wold[j] + sw[j];
            } else {
                const ushort4 p = r16[j];
                const float Wn = Wold[j] + sw[j];
                const float psi = (Wold[j] * unpack16(p.x, STORAGE) * M.truncation + sS[j]) / Wn;
                const float g0 = (Wold[j] * unpack16(p.y, STORAGE) + sG[j][0]) / Wn;
                const float g1 = (Wold[j] * unpack16(p.z, STORAGE) + sG[j][1]) / Wn;
                const float g2 = (Wold[j] * unpack16(p.w, STORAGE) + sG[j][2]) / Wn;
                reinterpret_cast<ushort4*>(M.vox)[vi[j]] =
                    make_ushort4(pack16(psi / M.truncation, STORAGE), pack16(g0, STORAGE), pack16(g1, STORAGE),
                                 pack16(g2, STORAGE));
                M.weight[vi[j]] = Wn;
            }
        }
        if (threadIdx.x == 0) M.touched_flag[slot] = 0;
        __syncthreads();
    }

    // work counters: one striped atomic per work-group and counter
    __shared__ unsigned long long red[kFuseBlock / 64];
    const unsigned long long u_s = block_sum_u64(my_updates, red);
    const unsigned long long v_s = block_sum_u64(my_visits, red);
    const unsigned long long x_s = block_sum_u64(my_voxels, red);
    if (threadIdx.x == 0) {
        add_stat(M, kStatUpdates, u_s);
        add_stat(M, kStatPixelVisits, v_s);
        add_stat(M, kStatFusedVoxels, x_s);
        add_stat(M, kStatFusedBlocks, my_blocks);
    }
}

// Fraction bits of the fixed-point voxel sums.  A pixel's band meets a voxel
// at most once and contributes |w d| <= T, |w n| <= 1, w <= 1, so a frame's
// sum is bounded by max(1, T) times the pixels whose rays can cross the
// voxel: its footprint, at most (f v_s sqrt(3) / z + 2)^2 pixels at the
// nearest depth z = max(zmin - T, v_s) a voxel of the band can have.  The
// bits are chosen to keep that bound below 2^62.
inline int fix_bits(const gsdf_camera& cam, double vs, double T) {
    const double z = std::max((double)cam.zmin - T, vs);
    const double side = std::max(cam.fx, cam.fy) * vs * std::sqrt(3.0) / z + 2.0;
    const double bound = side * side * std::max(1.0, T);
    const int f = (int)std::floor(62.0 - std::log2(bound));
    return std::min(56, std::max(24, f));
}

inline FuseConsts fuse_consts(const gsdf_map& map, const gsdf_camera& cam, const gsdf_fuse_params& p) {
    FuseConsts fc;
    fc.band = band_consts(cam, map.desc.voxel_size, map.desc.truncation);
    fc.fxf = (float)cam.fx;
    fc.fyf = (float)cam.fy;
    fc.rcx = (float)cam.cx;
    fc.rcy = (float)cam.cy;
    fc.fx_d = cam.fx;
    fc.fy_d = cam.fy;
    fc.ifx_d = 1.0 / cam.fx;
    fc.ify_d = 1.0 / cam.fy;
    fc.cx_d = cam.cx;
    fc.cy_d = cam.cy;
    fc.zmin = cam.zmin;
    fc.zmax = cam.zmax;
    fc.eps = p.eps_weight;
    fc.inv_span = (float)(1.0 / (map.desc.truncation - (double)p.eps_weight));
    fc.cos_min = p.cos_max_angle;
    fc.inv_vs_d = 1.0 / map.desc.voxel_size;
    fc.vs_d = map.desc.voxel_size;
    fc.vs_f = (float)map.desc.voxel_size;
    fc.T_f = (float)map.desc.truncation;
    fc.inv_df = (float)(2.0 / map.desc.voxel_size);
    fc.W = cam.width;
    fc.H = cam.height;
    const int f = fix_bits(cam, map.desc.voxel_size, map.desc.truncation);
    fc.fix_scale = std::ldexp(1.0f, f);
    fc.fix_inv = std::ldexp(1.0, -f);
    return fc;
}

inline void launch_fuse_blocks(int storage, hipStream_t s, const MapView& M, const float4* pix, const FuseConsts& fc,
                               const double* Twc, int32_t* status) {
    switch (storage) {
        case GSDF_FP32: k_fuse_blocks<GSDF_FP32><<<kFuseGroups, kFuseBlock, 0, s>>>(M, pix, fc, Twc, status); break;
        case GSDF_BF16: k_fuse_blocks<GSDF_BF16><<<kFuseGroups, kFuseBlock, 0, s>>>(M, pix, fc, Twc, status); break;
        case GSDF_FP16: k_fuse_blocks<GSDF_FP16><<<kFuseGroups, kFuseBlock, 0, s>>>(M, pix, fc, Twc, status); break;
        default: k_fuse_blocks<GSDF_NOGRAD_FP32><<<kFuseGroups, kFuseBlock, 0, s>>>(M, pix, fc, Twc, status); break;
    }
}

}  // namespace gsdf

using namespace gsdf;

extern "C" size_t gsdf_integrate_scratch_bytes(const gsdf_camera* cam) {
    if (!valid_cam(cam)) return 0;
    return align256((size_t)cam->width * cam->height * sizeof(float4));
}

extern "C" int gsdf_integrate_frame(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                                    const double* T_wc_dev, const gsdf_fuse_params* params,
                                    void* scratch_dev, size_t scratch_bytes, int32_t* status_dev,
                                    void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev || !params || !scratch_dev)
        return GSDF_EINVAL;
    if (!(params->eps_weight < map->desc.truncation)) return GSDF_EINVAL;
    if (scratch_bytes < gsdf_integrate_scratch_bytes(cam)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const FuseConsts fc = fuse_consts(*map, *cam, *params);
    const MapView M = make_view(*map);
    float4* pix = (float4*)scratch_dev;
    {
        TimedLaunch t(map->timer, GSDF_K_NORMALS, s);
        dim3 grid(ceil_div(cam->width, kTile), ceil_div(cam->height, kTile));
        k_pixel_normals<<<grid, 256, 0, s>>>(depth_dev, fc, T_wc_dev, pix);
    }
    {
        TimedLaunch t(map->timer, GSDF_K_INTEGRATE, s);
        launch_fuse_blocks(map->desc.storage, s, M, pix, fc, T_wc_dev, status_dev);
    }
    return launch_status();
}

extern "C" int gsdf_fuse_frame(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                               const double* T_wc_dev, const gsdf_fuse_params* params, void* scratch_dev,
                               size_t scratch_bytes, int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev || !params || !scratch_dev)
        return GSDF_EINVAL;
    if (!(params->eps_weight < map->desc.truncation)) return GSDF_EINVAL;
    if (scratch_bytes < gsdf_integrate_scratch_bytes(cam)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const FuseConsts fc = fuse_consts(*map, *cam, *params);
    const MapView M = make_view(*map);
    float4* pix = (float4*)scratch_dev;
    {
        TimedLaunch t(map->timer, GSDF_K_ALLOC_NORMALS, s);
        dim3 grid(ceil_div(cam->width, kTile), ceil_div(cam->height, kTile));
        k_alloc_normals<<<grid, 256, 0, s>>>(M, depth_dev, fc, T_wc_dev, pix, status_dev);
    }
    {
        TimedLaunch t(map->timer, GSDF_K_INTEGRATE, s);
        launch_fuse_blocks(map->desc.storage, s, M, pix, fc, T_wc_dev, status_dev);
    }
    return launch_status();
}
