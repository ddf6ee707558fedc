// Photometric term over keyframes for joint refinement with colour.
//
// Surface point of voxel j (Sec. 4.2 Eq. (18)): p_j = v_j - psi_j gh_j with
// gh_j held fixed while psi_j changes.  Voxels take part when observed
// (W > 0, g != 0) and their cell contains the surface point:
// max_k |psi_j gh_jk| <= v_s / 2.  Keyframe i sees voxel j when
// x = R_i^T (p_j - t_i) has z >= zmin, projects to (u, v) inside
// [0, width-1) x [0, height-1), the nearest pixel's depth D is valid with
// |z - D| <= T, and gh_j . (p_j - t_i) > 0.  With the voxel's stored colour
// rho_j (3 floats) and bilinear samples I_i^c(u, v):
//   L_i = lambda sum_{j seen by i} sum_c huber_delta(I_i^c(u, v) - rho_j^c).
// Gradients: d/drho_j^c = -lambda rho'(r_c); with e = sum_c lambda rho'(r_c)
// dI^c/d(u, v) and a = R_i (e . dpi/dx): d/dpsi_j = -a . gh_j, and for a
// left increment of T_i [-a ; a x p_j], mapped through Jl(xi_i)^T.
// The mean colour of Sec. 4.2 Eq. (21) uses the same visibility.
//
// Work layout: one work-group per map block, looping over the keyframes, so
// each voxel's psi and colour gradients are summed in registers and written
// once, without atomics; per keyframe the work-group's pose sums go to a
// partial that a second kernel reduces in a fixed order.  Few of a block's
// 512 voxels take part (those holding the surface: about 5 % on a room
// map), so the work-group first lists them in voxel order and hands the
// r-th to thread r mod 256 (two per thread at most): the projection and
// sampling then run on dense lanes, and waves with nothing to do skip the
// keyframe loop's work.  Projection and visibility are decided in float64 (they are
// discrete decisions), samples and gradients are float32.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gsdf.h"
#include "gsdf_common.hpp"
#include "gsdf_host.hpp"
#include "gsdf_se3.hpp"

namespace gsdf {

constexpr int kPhotoBlock = 256;
constexpr int kPhotoPart = 8;   // loss, 6 pose sums, visible count
constexpr int kPhotoMaxKeyframes = 1024;

struct PhotoArgs {
    int32_t W, H, K, pad0;
    double fx, fy, cx, cy;
    double zmin, zmax_f, trunc;
    double vs;
    float delta, lambda;
    int64_t param_blocks;
};

struct PhotoVoxel {
    bool ok;
    double p[3], gh[3];
    float ghf[3], rho[3];
};

__device__ inline void photo_voxel(const MapView& M, const PhotoArgs& a, const float4* __restrict__ params,
                                   const float* __restrict__ colors, int64_t slot, int c, PhotoVoxel* V) {
    V->ok = false;
    const int64_t vi = slot * kBlockVoxels + c;
    if (!(M.weight[vi] > 0.0f)) return;
    const float4 q = params[vi];
    const double g0 = q.y, g1 = q.z, g2 = q.w;
    const double ng = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    if (!(ng > 0.0)) return;
    V->gh[0] = g0 / ng;
    V->gh[1] = g1 / ng;
    V->gh[2] = g2 / ng;
    const double psi = q.x;
    for (int k = 0; k < 3; ++k)
        if (fabs(psi * V->gh[k]) > 0.5 * a.vs) return;
    const uint64_t key = M.block_keys[slot];
    int bx, by, bz;
    unpack_key(key, &bx, &by, &bz);
    int lx, ly, lz;
    demorton9(c, &lx, &ly, &lz);
    const int m[3] = {8 * bx + lx, 8 * by + ly, 8 * bz + lz};
    for (int k = 0; k < 3; ++k) {
        V->p[k] = a.vs * (double)m[k] - psi * V->gh[k];
        V->ghf[k] = (float)V->gh[k];
        V->rho[k] = colors ? colors[3 * vi + k] : 0.0f;
    }
    V->ok = true;
}

// Projection of p into keyframe i (pose row-major 3x4); false when not seen.
struct PhotoProj {
    double x[3], z, u, v;
};

__device__ inline bool photo_project(const PhotoArgs& a, const double* T, const float* __restrict__ depth_i,
                                     const PhotoVoxel& V, PhotoProj* P) {
    const double d[3] = {V.p[0] - T[3], V.p[1] - T[7], V.p[2] - T[11]};
    for (int r = 0; r < 3; ++r) P->x[r] = T[r] * d[0] + T[4 + r] * d[1] + T[8 + r] * d[2];
    P->z = P->x[2];
    if (!(P->z >= a.zmin)) return false;
    P->u = a.fx * P->x[0] / P->z + a.cx;
    P->v = a.fy * P->x[1] / P->z + a.cy;
    if (!(P->u >= 0.0 && P->u < (double)(a.W - 1) && P->v >= 0.0 && P->v < (double)(a.H - 1))) return false;
    const int iu = (int)floor(P->u + 0.5), iv = (int)floor(P->v + 0.5);
    const float D = depth_i[(size_t)iv * a.W + iu];
    if (!depth_ok(D, (float)a.zmin, (float)a.zmax_f)) return false;
    if (!(fabs(P->z - (double)D) <= a.trunc)) return false;
    return V.gh[0] * d[0] + V.gh[1] * d[1] + V.gh[2] * d[2] > 0.0;
}

__device__ inline void bilinear3(const float* __restrict__ img, int W, double u, double v, float I[3],
                                 float dIu[3], float dIv[3]) {
    const int u0 = (int)floor(u), v0 = (int)floor(v);
    const float fa = (float)(u - (double)u0), fb = (float)(v - (double)v0);
    const float* p00 = img + 3 * ((size_t)v0 * W + u0);
    const float* p01 = p00 + 3 * (size_t)W;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float i00 = p00[c], i10 = p00[3 + c], i01 = p01[c], i11 = p01[3 + c];
        I[c] = (1.0f - fa) * (1.0f - fb) * i00 + fa * (1.0f - fb) * i10 + (1.0f - fa) * fb * i01 + fa * fb * i11;
        dIu[c] = (1.0f - fb) * (i10 - i00) + fb * (i11 - i01);
        dIv[c] = (1.0f - fa) * (i01 - i00) + fa * (i11 - i10);
    }
}

// MODE 0: loss only; 1: loss and gradients; 2: mean colour (Eq. (21));
// 3: adjoint of the mean colour: with the upstream gradient G_j (in
// `colors`) and the view counts N_j (in `counts`), each sample adds
// (G_j / N_j) . dI_ij to the psi and pose gradients (g^ held fixed).
template <int MODE>
__global__ __launch_bounds__(kPhotoBlock) void k_photometric(MapView M, PhotoArgs a, const float* __restrict__ depth,
                                                            const float* __restrict__ rgb,
                                                            const double* __restrict__ poses,
                                                            const float4* __restrict__ params,
                                                            const float* __restrict__ colors,
                                                            const float* __restrict__ gscale,
                                                            float* __restrict__ dparams, float* __restrict__ dcolors,
                                                            float* __restrict__ out_colors,
                                                            float* __restrict__ out_count,
                                                            const float* __restrict__ counts,
                                                            double* __restrict__ partials) {
    constexpr int kWaves = kPhotoBlock / 64;
    __shared__ double s_red[kPhotoPart][kWaves];
    __shared__ int s_wcount[2][kWaves];
    __shared__ short s_list[kBlockVoxels];
    const int64_t slot = blockIdx.x;
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // 1. the voxels that take part, listed in voxel order (c = t, then 256 + t)
    bool take[2];
    unsigned long long bal[2];
    for (int h = 0; h < 2; ++h) {
        const int c = threadIdx.x + h * kPhotoBlock;
        PhotoVoxel Q;
        Q.ok = false;
        if (slot < nb) photo_voxel(M, a, params, nullptr, slot, c, &Q);
        if (MODE == 3 && Q.ok && !(counts[slot * kBlockVoxels + c] > 0.0f)) Q.ok = false;
        take[h] = Q.ok;
        if (MODE == 2 && !Q.ok) {
            // not seen by construction: zero mean and count
            const int64_t vi = slot * kBlockVoxels + c;
#pragma unroll
            for (int k = 0; k < 3; ++k) out_colors[3 * vi + k] = 0.0f;
            if (out_count) out_count[vi] = 0.0f;
        }
        bal[h] = __ballot(take[h]);
        if (lane == 0) s_wcount[h][wave] = __popcll(bal[h]);
    }
    __syncthreads();
    // rank of a listed voxel: the voxels of the earlier (h, wave) groups,
    // then those of the earlier lanes of its own
    int base[2] = {0, 0}, n_act = 0;
    for (int h = 0; h < 2; ++h)
        for (int w = 0; w < kWaves; ++w) {
            if (w == wave) base[h] = n_act;
            n_act += s_wcount[h][w];
        }
    for (int h = 0; h < 2; ++h)
        if (take[h])
            s_list[base[h] + __popcll(bal[h] & ((1ull << lane) - 1ull))] = (short)(threadIdx.x + h * kPhotoBlock);
    __syncthreads();
    if (n_act == 0) {
        // nothing in this block is seen: zero pose partials
        if (MODE != 2)
            for (int i = threadIdx.x; i < a.K * kPhotoPart; i += kPhotoBlock)
                partials[((size_t)(i / kPhotoPart) * a.param_blocks + slot) * kPhotoPart + i % kPhotoPart] = 0.0;
        return;
    }
    // 2. thread t takes the listed voxels t and t + 256
    PhotoVoxel V[2];
    int vc[2];
    for (int h = 0; h < 2; ++h) {
        const int r = threadIdx.x + h * kPhotoBlock;
        V[h].ok = false;
        vc[h] = 0;
        if (r >= n_act) continue;
        vc[h] = s_list[r];
        photo_voxel(M, a, params, MODE == 2 ? nullptr : colors, slot, vc[h], &V[h]);
        if (MODE == 3) {
            // upstream gradient per sample of the mean: G_j / N_j
            const float n = counts[slot * kBlockVoxels + vc[h]];
#pragma unroll
            for (int c = 0; c < 3; ++c) V[h].rho[c] /= n;
        }
    }
    // waves holding a listed voxel (uniform per wave)
    const bool any = wave * 64 < n_act;
    const size_t npx = (size_t)a.W * a.H;
    float gpsi[2] = {0.0f, 0.0f}, grho[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}};
    float csum[2][3] = {{0.0f, 0.0f, 0.0f}, {0.0f, 0.0f, 0.0f}}, cnt[2] = {0.0f, 0.0f};

    for (int kf = 0; kf < a.K; ++kf) {
        float acc[kPhotoPart];
#pragma unroll
        for (int k = 0; k < kPhotoPart; ++k) acc[k] = 0.0f;
        if (any) {
            double T[12];
            for (int i = 0; i < 12; ++i) T[i] = poses[12 * kf + i];
            const float s = MODE == 1 ? gscale[kf] : 1.0f;
            for (int h = 0; h < 2; ++h) {
                if (!V[h].ok) continue;
                PhotoProj P;
                if (!photo_project(a, T, depth + kf * npx, V[h], &P)) continue;
                float I[3], dIu[3], dIv[3];
                bilinear3(rgb + 3 * kf * npx, a.W, P.u, P.v, I, dIu, dIv);
                acc[7] += 1.0f;
                if (MODE == 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) csum[h][c] += I[c];
                    cnt[h] += 1.0f;
                    continue;
                }
                float eu = 0.0f, ev = 0.0f;
                if (MODE == 3) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        eu += V[h].rho[c] * dIu[c];
                        ev += V[h].rho[c] * dIv[c];
                    }
                }
#pragma unroll
                for (int c = 0; c < 3 && MODE != 3; ++c) {
                    const float r = I[c] - V[h].rho[c];
                    const float ar = fabsf(r);
                    const bool quad = ar <= a.delta;
                    acc[0] += a.lambda * (quad ? 0.5f * r * r : a.delta * (ar - 0.5f * a.delta));
                    if (MODE == 1) {
                        const float rp = s * a.lambda * (quad ? r : copysignf(a.delta, r));
                        grho[h][c] -= rp;
                        eu += rp * dIu[c];
                        ev += rp * dIv[c];
                    }
                }
                if (MODE == 1 || MODE == 3) {
                    const float iz = (float)(1.0 / P.z);
                    const float fx = (float)a.fx, fy = (float)a.fy;
                    const float x0 = (float)P.x[0], x1 = (float)P.x[1];
                    const float gx[3] = {eu * fx * iz, ev * fy * iz, -(eu * fx * x0 + ev * fy * x1) * iz * iz};
                    float aw[3];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        aw[r] = (float)T[4 * r] * gx[0] + (float)T[4 * r + 1] * gx[1] + (float)T[4 * r + 2] * gx[2];
                    gpsi[h] -= aw[0] * V[h].ghf[0] + aw[1] * V[h].ghf[1] + aw[2] * V[h].ghf[2];
                    const float p0 = (float)V[h].p[0], p1 = (float)V[h].p[1], p2 = (float)V[h].p[2];
                    acc[1] -= aw[0];
                    acc[2] -= aw[1];
                    acc[3] -= aw[2];
                    acc[4] += aw[1] * p2 - aw[2] * p1;
                    acc[5] += aw[2] * p0 - aw[0] * p2;
                    acc[6] += aw[0] * p1 - aw[1] * p0;
                }
            }
        }
        if (MODE == 2) continue;
        // work-group sums for this keyframe (float64 across lanes)
#pragma unroll
        for (int k = 0; k < kPhotoPart; ++k) {
            double x = (double)acc[k];
            if (any)
                for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
            if (lane == 0) s_red[k][wave] = x;
        }
        __syncthreads();
        if (threadIdx.x < kPhotoPart) {
            double x = 0.0;
            for (int w = 0; w < kPhotoBlock / 64; ++w) x += s_red[threadIdx.x][w];
            partials[((size_t)kf * a.param_blocks + slot) * kPhotoPart + threadIdx.x] = x;
        }
        __syncthreads();
    }
    for (int h = 0; h < 2; ++h) {
        if (!V[h].ok) continue;
        const int64_t vi = slot * kBlockVoxels + vc[h];
        if (MODE == 2) {
            const float n = cnt[h];
#pragma unroll
            for (int c = 0; c < 3; ++c) out_colors[3 * vi + c] = n > 0.0f ? csum[h][c] / n : 0.0f;
            if (out_count) out_count[vi] = n;
        } else if (MODE == 1) {
            dparams[4 * vi] += gpsi[h];
#pragma unroll
            for (int c = 0; c < 3; ++c) dcolors[3 * vi + c] += grho[h][c];
        } else if (MODE == 3) {
            dparams[4 * vi] += gpsi[h];
        }
    }
}

// One work-group per keyframe: fixed-order sum over the map blocks' partials.
__global__ __launch_bounds__(256) void k_photometric_finish(PhotoArgs a, const double* __restrict__ xi,
                                                            const double* __restrict__ partials,
                                                            double* __restrict__ loss_out,
                                                            double* __restrict__ count_out,
                                                            double* __restrict__ dxi_out) {
    __shared__ double s_part[kPhotoPart][256];
    const int kf = blockIdx.x;
    double x[kPhotoPart];
    for (int k = 0; k < kPhotoPart; ++k) x[k] = 0.0;
    for (int64_t b = threadIdx.x; b < a.param_blocks; b += 256)
        for (int k = 0; k < kPhotoPart; ++k) x[k] += partials[((size_t)kf * a.param_blocks + b) * kPhotoPart + k];
    for (int k = 0; k < kPhotoPart; ++k) s_part[k][threadIdx.x] = x[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < kPhotoPart; ++k) s_part[k][threadIdx.x] += s_part[k][threadIdx.x + w];
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

__global__ void k_photo_poses(int32_t K, const double* __restrict__ T0, const double* __restrict__ xi,
                              double* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= K) return;
    double pose[12];
    for (int j = 0; j < 12; ++j) pose[j] = T0[12 * i + j];
    se3_apply_left(xi + 6 * i, pose);
    for (int j = 0; j < 12; ++j) out[12 * i + j] = pose[j];
}

inline PhotoArgs photo_args(const gsdf_map& map, const gsdf_camera& cam, int32_t K, int64_t param_blocks,
                            float delta, float lambda) {
    PhotoArgs a;
    a.W = cam.width;
    a.H = cam.height;
    a.K = K;
    a.pad0 = 0;
    a.fx = cam.fx;
    a.fy = cam.fy;
    a.cx = cam.cx;
    a.cy = cam.cy;
    a.zmin = cam.zmin;
    a.zmax_f = cam.zmax;
    a.trunc = map.desc.truncation;
    a.vs = map.desc.voxel_size;
    a.delta = delta;
    a.lambda = lambda;
    a.param_blocks = param_blocks;
    return a;
}

struct PhotoScratch {
    size_t poses, partials, total;
};

inline PhotoScratch photo_scratch(int64_t param_blocks, int32_t K) {
    PhotoScratch s;
    s.poses = 0;
    s.partials = align256((size_t)K * 12 * sizeof(double));
    s.total = s.partials + (size_t)K * param_blocks * kPhotoPart * sizeof(double);
    return s;
}

}  // namespace gsdf

using namespace gsdf;

extern "C" {

size_t gsdf_photometric_scratch_bytes(int64_t param_blocks, int32_t n_keyframes) {
    if (param_blocks < 0 || n_keyframes <= 0 || n_keyframes > kPhotoMaxKeyframes) return 0;
    return photo_scratch(param_blocks, n_keyframes).total;
}

static int photo_check(const gsdf_map* map, const float* depth_dev, const float* rgb_dev, int32_t K,
                       const gsdf_camera* cam, const double* T0_dev, const double* xi_dev, const float* params_dev,
                       int64_t param_blocks, void* scratch, size_t scratch_bytes) {
    if (!valid_map(map) || !valid_cam(cam) || K <= 0 || K > kPhotoMaxKeyframes || !depth_dev || !rgb_dev ||
        !T0_dev || !xi_dev || !params_dev || param_blocks < 0 || param_blocks > map->desc.max_blocks || !scratch)
        return GSDF_EINVAL;
    if (scratch_bytes < photo_scratch(param_blocks, K).total) return GSDF_EINVAL;
    if (!has_gradients(map)) return GSDF_EINVAL;
    return GSDF_OK;
}

static void photo_launch(int mode, const gsdf_map* map, const float* depth, const float* rgb, int32_t K,
                         const gsdf_camera* cam, const double* T0, const double* xi, const float* params,
                         const float* colors, int64_t param_blocks, float delta, float lambda, const float* gscale,
                         float* dparams, float* dcolors, float* out_colors, float* out_count, double* loss_out,
                         double* count_out, double* dxi_out, void* scratch, hipStream_t s,
                         const float* counts = nullptr) {
    const PhotoArgs a = photo_args(*map, *cam, K, param_blocks, delta, lambda);
    const PhotoScratch L = photo_scratch(param_blocks, K);
    double* poses = (double*)((char*)scratch + L.poses);
    double* partials = (double*)((char*)scratch + L.partials);
    k_photo_poses<<<ceil_div(K, 64), 64, 0, s>>>(K, T0, xi, poses);
    if (param_blocks > 0) {
        const MapView M = make_view(*map);
        const float4* P = reinterpret_cast<const float4*>(params);
        TimedLaunch tl(map->timer, GSDF_K_PHOTOMETRIC, s);
        if (mode == 0)
            k_photometric<0><<<(unsigned)param_blocks, kPhotoBlock, 0, s>>>(
                M, a, depth, rgb, poses, P, colors, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, partials);
        else if (mode == 1)
            k_photometric<1><<<(unsigned)param_blocks, kPhotoBlock, 0, s>>>(
                M, a, depth, rgb, poses, P, colors, gscale, dparams, dcolors, nullptr, nullptr, nullptr, partials);
        else if (mode == 2)
            k_photometric<2><<<(unsigned)param_blocks, kPhotoBlock, 0, s>>>(
                M, a, depth, rgb, poses, P, nullptr, nullptr, nullptr, nullptr, out_colors, out_count, nullptr,
                partials);
        else
            k_photometric<3><<<(unsigned)param_blocks, kPhotoBlock, 0, s>>>(
                M, a, depth, rgb, poses, P, colors, nullptr, dparams, nullptr, nullptr, nullptr, counts, partials);
    }
    if (mode != 2)
        k_photometric_finish<<<K, 256, 0, s>>>(a, xi, partials, loss_out, count_out, dxi_out);
}

// Quadratic regulariser of the distances towards reference values
// (lambda sum_j (psi_j - psi0_j)^2 over observed voxels), used with the
// bundle-adjustment energy; one work-group per map block.
__global__ __launch_bounds__(256) void k_psi_regulariser(MapView M, int64_t param_blocks, const float4* __restrict__ params,
                                                         const float4* __restrict__ params0, float lambda,
                                                         float* __restrict__ dparams, double* __restrict__ partials) {
    __shared__ double s_red[4];
    const int64_t slot = blockIdx.x;
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    double e = 0.0;
    for (int c = threadIdx.x; c < kBlockVoxels; c += 256) {
        const int64_t vi = slot * kBlockVoxels + c;
        if (slot >= nb || !(M.weight[vi] > 0.0f)) continue;
        const float d = params[vi].x - params0[vi].x;
        e += (double)(lambda * d * d);
        if (dparams) dparams[4 * vi] += 2.0f * lambda * d;
    }
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) partials[slot] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ partials, int64_t n,
                                                      double* __restrict__ out) {
    __shared__ double s[256];
    double x = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) x += partials[i];
    s[threadIdx.x] = x;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

int gsdf_photometric_loss(const gsdf_map* map, const float* depth_dev, const float* rgb_dev, int32_t n_keyframes,
                          const gsdf_camera* cam, const double* T0_dev, const double* xi_dev,
                          const float* params_dev, const float* colors_dev, int64_t param_blocks,
                          float huber_delta, float weight, double* loss_dev, double* count_dev, void* scratch_dev,
                          size_t scratch_bytes, void* stream) {
    int rc = photo_check(map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                         scratch_dev, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!colors_dev || !loss_dev || !(huber_delta > 0.0f) || !(weight >= 0.0f)) return GSDF_EINVAL;
    photo_launch(0, map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, colors_dev,
                 param_blocks, huber_delta, weight, nullptr, nullptr, nullptr, nullptr, nullptr, loss_dev, count_dev,
                 nullptr, scratch_dev, (hipStream_t)stream);
    return launch_status();
}

int gsdf_photometric_backward(const gsdf_map* map, const float* depth_dev, const float* rgb_dev,
                              int32_t n_keyframes, const gsdf_camera* cam, const double* T0_dev,
                              const double* xi_dev, const float* params_dev, const float* colors_dev,
                              int64_t param_blocks, float huber_delta, float weight, const float* grad_loss_dev,
                              float* dparams_dev, float* dcolors_dev, double* dxi_dev, double* loss_dev,
                              void* scratch_dev, size_t scratch_bytes, void* stream) {
    int rc = photo_check(map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                         scratch_dev, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!colors_dev || !grad_loss_dev || !dparams_dev || !dcolors_dev || !dxi_dev || !(huber_delta > 0.0f) ||
        !(weight >= 0.0f))
        return GSDF_EINVAL;
    photo_launch(1, map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, colors_dev,
                 param_blocks, huber_delta, weight, grad_loss_dev, dparams_dev, dcolors_dev, nullptr, nullptr,
                 loss_dev, nullptr, dxi_dev, scratch_dev, (hipStream_t)stream);
    return launch_status();
}

int gsdf_mean_color_backward(const gsdf_map* map, const float* depth_dev, const float* rgb_dev,
                             int32_t n_keyframes, const gsdf_camera* cam, const double* T0_dev,
                             const double* xi_dev, const float* params_dev, int64_t param_blocks,
                             const float* grad_colors_dev, const float* counts_dev, float* dparams_dev,
                             double* dxi_dev, void* scratch_dev, size_t scratch_bytes, void* stream) {
    int rc = photo_check(map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                         scratch_dev, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!grad_colors_dev || !counts_dev || !dparams_dev || !dxi_dev) return GSDF_EINVAL;
    photo_launch(3, map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, grad_colors_dev,
                 param_blocks, 1.0f, 1.0f, nullptr, dparams_dev, nullptr, nullptr, nullptr, nullptr, nullptr,
                 dxi_dev, scratch_dev, (hipStream_t)stream, counts_dev);
    return launch_status();
}

int gsdf_psi_regulariser(const gsdf_map* map, const float* params_dev, const float* params0_dev,
                         int64_t param_blocks, float weight, double* loss_dev, float* dparams_dev,
                         void* scratch_dev, size_t scratch_bytes, void* stream) {
    if (!valid_map(map) || !params_dev || !params0_dev || !loss_dev || param_blocks < 0 ||
        param_blocks > map->desc.max_blocks || !(weight >= 0.0f) || !scratch_dev ||
        scratch_bytes < (size_t)(param_blocks > 0 ? param_blocks : 1) * sizeof(double))
        return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    double* partials = (double*)scratch_dev;
    if (param_blocks > 0)
        k_psi_regulariser<<<(unsigned)param_blocks, 256, 0, s>>>(make_view(*map), param_blocks,
                                                                 reinterpret_cast<const float4*>(params_dev),
                                                                 reinterpret_cast<const float4*>(params0_dev),
                                                                 weight, dparams_dev, partials);
    k_sum_partials<<<1, 256, 0, s>>>(partials, param_blocks, loss_dev);
    return launch_status();
}

int gsdf_mean_color(const gsdf_map* map, const float* depth_dev, const float* rgb_dev, int32_t n_keyframes,
                    const gsdf_camera* cam, const double* T0_dev, const double* xi_dev, const float* params_dev,
                    int64_t param_blocks, float* colors_out_dev, float* count_out_dev, void* scratch_dev,
                    size_t scratch_bytes, void* stream) {
    int rc = photo_check(map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, param_blocks,
                         scratch_dev, scratch_bytes);
    if (rc != GSDF_OK) return rc;
    if (!colors_out_dev) return GSDF_EINVAL;
    photo_launch(2, map, depth_dev, rgb_dev, n_keyframes, cam, T0_dev, xi_dev, params_dev, nullptr, param_blocks,
                 1.0f, 1.0f, nullptr, nullptr, nullptr, colors_out_dev, count_out_dev, nullptr, nullptr, nullptr,
                 scratch_dev, (hipStream_t)stream);
    return launch_status();
}

}  // extern "C"
