// integrate_frame: normals from a 5x5 plane fit, the viewing-angle filter,
// and the running weighted average of SDF and gradient, Eq. (1)-(3) of
// Gradient-SDF (Sec. 3.1, 3.2), driven pixel by pixel as in the Sec. 5.3
// setup.
//
// One work-group covers a 16x16 pixel tile; its depths plus a 2-pixel halo
// are staged in LDS once, so the 25-tap normal fit reads LDS only.  Every
// pixel then walks its ray band (the binary32 rule shared with allocation)
// and adds w d, w n_w and w into the voxels it crosses.
//
// FP32 storage keeps, per voxel, float4 {sum w d, g_x, g_y, g_z} and W:
// psi = (sum w d) / W is Eq. (1)-(2) unrolled over all observations and g
// is Eq. (3) exactly, so the update is pure addition (hardware float
// atomics, no second pass).  Reduced-precision storage keeps normalised
// values that must be averaged: the pixel pass adds into per-voxel float32
// accumulators and a second pass over the touched blocks applies Eq. (1)-(3)
// and rounds once per frame.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <climits>

#include "gsdf_common.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

constexpr int kTile = 16;
constexpr int kHalo = 2;
constexpr int kTileH = kTile + 2 * kHalo;

struct FuseConsts {
    BandConsts band;
    float fxf, fyf, cxf, cyf;     // float32 intrinsics for the normal fit
    float rcx, rcy;               // (float) cx, cy
    double ifx_d, ify_d, cx_d, cy_d;
    float zmin, zmax;
    float eps, cos_min;
    double inv_vs_d, vs_d;
    float vs_f, T_f;
    int W, H;
};

__device__ inline float linear_weight(float d, float eps, float T) {
    if (d <= eps) return 1.0f;
    if (d >= T) return 0.0f;
    return (T - d) / (T - eps);
}

template <int STORAGE>
__global__ __launch_bounds__(256) void k_integrate(MapView M, const float* __restrict__ depth,
                                                   FuseConsts fc, const double* __restrict__ Twc,
                                                   int32_t* status) {
    __shared__ float tile[kTileH][kTileH + 1];
    const int tx = threadIdx.x & (kTile - 1);
    const int ty = threadIdx.x / kTile;
    const int u0 = blockIdx.x * kTile - kHalo;
    const int v0 = blockIdx.y * kTile - kHalo;
    for (int i = threadIdx.x; i < kTileH * kTileH; i += blockDim.x) {
        const int ly = i / kTileH, lx = i % kTileH;
        const int uu = u0 + lx, vv = v0 + ly;
        float d = 0.0f;
        if (uu >= 0 && uu < fc.W && vv >= 0 && vv < fc.H) d = depth[(size_t)vv * fc.W + uu];
        tile[ly][lx] = d;
    }
    __syncthreads();

    const int u = blockIdx.x * kTile + tx;
    const int v = blockIdx.y * kTile + ty;
    if (u < kHalo || v < kHalo || u >= fc.W - kHalo || v >= fc.H - kHalo) return;
    const float Dc = tile[ty + kHalo][tx + kHalo];
    if (!depth_ok(Dc, fc.zmin, fc.zmax)) return;

    // ---- normal: least-squares plane 1/z = a . [x/z, y/z, 1] on the 5x5
    // window.  Over the symmetric window the design (1, du, dv) is
    // orthogonal, so the fit has a closed form in the centred inverse depths
    // 1/D_i - 1/D_c = (D_c - D_i) / (D_i D_c), whose numerators are exact.
    float s0 = 0.0f, sa = 0.0f, sb = 0.0f;
    bool ok = true;
#pragma unroll
    for (int dv = -kHalo; dv <= kHalo; ++dv) {
#pragma unroll
        for (int du = -kHalo; du <= kHalo; ++du) {
            const float Di = tile[ty + kHalo + dv][tx + kHalo + du];
            ok = ok && depth_ok(Di, fc.zmin, fc.zmax) && (fabsf(Di - Dc) <= fc.band.Tf);
            const float dy = (Dc - Di) / (Di * Dc);
            s0 += dy;
            sa += (float)du * dy;
            sb += (float)dv * dy;
        }
    }
    if (!ok) return;
    const float h = 1.0f / Dc + s0 * (1.0f / 25.0f);
    const float alpha = sa * (1.0f / 50.0f);   // sum du^2 = 50 over the window
    const float beta = sb * (1.0f / 50.0f);
    const float ax = alpha * fc.fxf;
    const float ay = beta * fc.fyf;
    const float az = h - alpha * ((float)u - fc.rcx) - beta * ((float)v - fc.rcy);
    const float na = sqrtf(ax * ax + ay * ay + az * az);
    const float rx = ((float)u - fc.rcx) / fc.fxf;
    const float ry = ((float)v - fc.rcy) / fc.fyf;
    const float cosang = h / (na * sqrtf(rx * rx + ry * ry + 1.0f));
    if (!(cosang >= fc.cos_min)) return;
    const float nc[3] = {ax / na, ay / na, az / na};   // a . ray = h > 0: faces away

    // ---- pose: rotate the normal; observed point in float64, kept as an
    // offset from a nearby voxel so voxel-to-point vectors stay small.
    double Rd[9], td[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) Rd[3 * i + j] = Twc[4 * i + j];
        td[i] = Twc[4 * i + 3];
    }
    float nw[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        nw[i] = (float)Rd[3 * i] * nc[0] + (float)Rd[3 * i + 1] * nc[1] + (float)Rd[3 * i + 2] * nc[2];
    const double Dd = (double)Dc;
    const double x[3] = {Dd * (((double)u - fc.cx_d) * fc.ifx_d), Dd * (((double)v - fc.cy_d) * fc.ify_d), Dd};
    int mref[3];
    float prel[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double p = Rd[3 * i] * x[0] + Rd[3 * i + 1] * x[1] + Rd[3 * i + 2] * x[2] + td[i];
        mref[i] = (int)floor(p * fc.inv_vs_d + 0.5);
        prel[i] = (float)(p - fc.vs_d * (double)mref[i]);
    }

    // ---- walk the ray band
    const BandRule br = make_band_rule(Twc, fc.band.ifx, fc.band.ify, fc.band.cxf, fc.band.cyf,
                                       fc.band.invvs, fc.band.Tf, fc.band.Df, fc.band.nsamples);
    const float xr = pixel_xr(br, u);
    const float yr = pixel_yr(br, v);
    int pm[3] = {INT_MIN, INT_MIN, INT_MIN};
    int cb[3] = {INT_MIN, INT_MIN, INT_MIN};
    int32_t slot = -1;
    for (int k = 0; k < br.nsamples; ++k) {
        int m[3];
        if (!band_sample(br, xr, yr, Dc, k, m)) continue;
        if (m[0] == pm[0] && m[1] == pm[1] && m[2] == pm[2]) continue;
        pm[0] = m[0];
        pm[1] = m[1];
        pm[2] = m[2];
        const int bx = block_of(m[0]), by = block_of(m[1]), bz = block_of(m[2]);
        if (bx != cb[0] || by != cb[1] || bz != cb[2]) {
            cb[0] = bx;
            cb[1] = by;
            cb[2] = bz;
            slot = hash_find(M, bx, by, bz);
            if (STORAGE != GSDF_FP32 && slot >= 0) {
                if (__hip_atomic_load(&M.touched_flag[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
                    atomicCAS(&M.touched_flag[slot], 0, 1) == 0) {
                    const int32_t pos = atomicAdd(&M.counters[kNumTouched], 1);
                    M.touched_list[pos] = slot;
                }
            }
        }
        if (slot < 0) continue;
        float off[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) off[i] = fc.vs_f * (float)(m[i] - mref[i]) - prel[i];
        float d = nw[0] * off[0] + nw[1] * off[1] + nw[2] * off[2];
        d = fminf(fc.T_f, fmaxf(-fc.T_f, d));
        const float w = linear_weight(d, fc.eps, fc.T_f);
        if (!(w > 0.0f)) continue;
        const int64_t vi = (int64_t)slot * kBlockVoxels + morton9(m[0] & 7, m[1] & 7, m[2] & 7);
        if (STORAGE == GSDF_FP32) {
            float* rec = reinterpret_cast<float*>(M.vox) + 4 * vi;
            unsafeAtomicAdd(rec + 0, w * d);
            unsafeAtomicAdd(rec + 1, w * nw[0]);
            unsafeAtomicAdd(rec + 2, w * nw[1]);
            unsafeAtomicAdd(rec + 3, w * nw[2]);
            unsafeAtomicAdd(M.weight + vi, w);
        } else {
            float* acc = M.accum + 5 * vi;
            unsafeAtomicAdd(acc + 0, w * d);
            unsafeAtomicAdd(acc + 1, w * nw[0]);
            unsafeAtomicAdd(acc + 2, w * nw[1]);
            unsafeAtomicAdd(acc + 3, w * nw[2]);
            unsafeAtomicAdd(acc + 4, w);
        }
    }
}

// ---- reduced-precision storage: apply the frame's sums to touched blocks ----
__global__ __launch_bounds__(256) void k_finalize(MapView M, int storage) {
    const int n = M.counters[kNumTouched];
    for (int b = blockIdx.x; b < n; b += gridDim.x) {
        const int slot = M.touched_list[b];
        for (int c = threadIdx.x; c < kBlockVoxels; c += blockDim.x) {
            const int64_t vi = (int64_t)slot * kBlockVoxels + c;
            float* acc = M.accum + 5 * vi;
            const float sw = acc[4];
            if (!(sw > 0.0f)) continue;
            const float Wold = M.weight[vi];
            const ushort4 p = reinterpret_cast<const ushort4*>(M.vox)[vi];
            const float psi_old = unpack16(p.x, storage) * M.truncation;
            const float Wn = Wold + sw;
            const float psi = (Wold * psi_old + acc[0]) / Wn;
            const float g0 = (Wold * unpack16(p.y, storage) + acc[1]) / Wn;
            const float g1 = (Wold * unpack16(p.z, storage) + acc[2]) / Wn;
            const float g2 = (Wold * unpack16(p.w, storage) + acc[3]) / Wn;
            reinterpret_cast<ushort4*>(M.vox)[vi] =
                make_ushort4(pack16(psi / M.truncation, storage), pack16(g0, storage),
                             pack16(g1, storage), pack16(g2, storage));
            M.weight[vi] = Wn;
            acc[0] = 0.0f;
            acc[1] = 0.0f;
            acc[2] = 0.0f;
            acc[3] = 0.0f;
            acc[4] = 0.0f;
        }
        __syncthreads();
        if (threadIdx.x == 0) M.touched_flag[slot] = 0;
    }
}

__global__ void k_finalize_done(MapView M) {
    if (threadIdx.x == 0 && blockIdx.x == 0) M.counters[kNumTouched] = 0;
}

}  // namespace gsdf

using namespace gsdf;

extern "C" int gsdf_integrate_frame(gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                                    const double* T_wc_dev, const gsdf_fuse_params* params,
                                    int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev || !params) return GSDF_EINVAL;
    if (!(params->eps_weight < map->desc.truncation)) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    FuseConsts fc;
    fc.band = band_consts(*cam, map->desc.voxel_size, map->desc.truncation);
    fc.fxf = (float)cam->fx;
    fc.fyf = (float)cam->fy;
    fc.cxf = (float)cam->cx;
    fc.cyf = (float)cam->cy;
    fc.rcx = (float)cam->cx;
    fc.rcy = (float)cam->cy;
    fc.ifx_d = 1.0 / cam->fx;
    fc.ify_d = 1.0 / cam->fy;
    fc.cx_d = cam->cx;
    fc.cy_d = cam->cy;
    fc.zmin = cam->zmin;
    fc.zmax = cam->zmax;
    fc.eps = params->eps_weight;
    fc.cos_min = params->cos_max_angle;
    fc.inv_vs_d = 1.0 / map->desc.voxel_size;
    fc.vs_d = map->desc.voxel_size;
    fc.vs_f = (float)map->desc.voxel_size;
    fc.T_f = (float)map->desc.truncation;
    fc.W = cam->width;
    fc.H = cam->height;
    const MapView M = make_view(*map);
    dim3 grid(ceil_div(cam->width, kTile), ceil_div(cam->height, kTile));
    {
        TimedLaunch t(GSDF_K_INTEGRATE, s);
        switch (map->desc.storage) {
            case GSDF_FP32: k_integrate<GSDF_FP32><<<grid, 256, 0, s>>>(M, depth_dev, fc, T_wc_dev, status_dev); break;
            case GSDF_BF16: k_integrate<GSDF_BF16><<<grid, 256, 0, s>>>(M, depth_dev, fc, T_wc_dev, status_dev); break;
            default: k_integrate<GSDF_FP16><<<grid, 256, 0, s>>>(M, depth_dev, fc, T_wc_dev, status_dev); break;
        }
    }
    if (map->desc.storage != GSDF_FP32) {
        TimedLaunch t(GSDF_K_FINALIZE, s);
        k_finalize<<<2048, 256, 0, s>>>(M, map->desc.storage);
        k_finalize_done<<<1, 64, 0, s>>>(M);
    }
    return launch_status();
}
