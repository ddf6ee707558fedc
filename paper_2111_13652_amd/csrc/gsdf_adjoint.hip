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
// per-pixel Jacobian is stored) and scatters
//   dL/dpsi_j += s rho'(r),
//   dL/dg_j   += s rho'(r) (I - gh gh^T)(q - v_j) / |g_j|,
// into the parameter-gradient buffer at the voxel's slot, where s is the
// upstream gradient of L_i, and sums s rho'(r) [gh; q x gh] (the derivative
// with respect to a left increment of T_i) per keyframe; a second kernel
// maps it through the SE(3) left Jacobian of xi_i:
//   dL/dxi_i = Jl(xi_i)^T sum_k s rho'(r_ik) [gh; q x gh].
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "gsdf.h"
#include "gsdf_common.hpp"
#include "gsdf_host.hpp"
#include "gsdf_se3.hpp"

namespace gsdf {

constexpr int kAdjBlock = 256;
constexpr int kAdjPart = 8;         // doubles per work-group partial: loss, 6 pose sums, count
constexpr int kAdjMaxGroups = 512;  // work-groups per keyframe
constexpr int kAdjTile = 32;        // a work-group takes 32x32 pixel tiles, four pixels a thread
constexpr int kAdjSetBits = 10;
constexpr int kAdjSet = 1 << kAdjSetBits;   // LDS table of a tile's voxels (entries)
constexpr long long kAdjEmpty = -1;

struct AdjArgs {
    int32_t W, H, groups, freeze;
    double ifx, ify, cx, cy;
    float zmin, zmax, delta, pad;
    double vs, inv_vs;
    int64_t param_blocks;   // rows of the parameter buffer (slots beyond are unobserved)
};

// Voxel, offset and parameters of one pixel; false when it has no usable
// voxel (invalid depth, block absent, W = 0 or g = 0).
struct PixelTerm {
    int64_t vi;
    float psi, gh[3], inv_ng, dq[3], q[3];
};

__device__ inline bool pixel_term(const MapView& M, const AdjArgs& a, const double R[9], const double t[3],
                                  const float4* __restrict__ params, float D, int u, int v,
                                  int32_t* __restrict__ as, PixelTerm* P) {
    if (!depth_ok(D, a.zmin, a.zmax)) {
        if (as && !a.freeze) as[0] = as[1] = as[2] = INT_MIN;
        return false;
    }
    const double Dd = (double)D;
    const double x0 = Dd * (((double)u - a.cx) * a.ifx);
    const double x1 = Dd * (((double)v - a.cy) * a.ify);
    double q[3];
    int m[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        q[r] = R[3 * r] * x0 + R[3 * r + 1] * x1 + R[3 * r + 2] * Dd + t[r];
        m[r] = (int)floor(q[r] * a.inv_vs + 0.5);
    }
    if (as && a.freeze) {
        if (as[0] == INT_MIN) return false;
        m[0] = as[0];
        m[1] = as[1];
        m[2] = as[2];
    }
    bool ok = false;
    const int32_t slot = hash_find(M, block_of(m[0]), block_of(m[1]), block_of(m[2]));
    if (slot >= 0 && (int64_t)slot < a.param_blocks) {
        P->vi = (int64_t)slot * kBlockVoxels + morton9(m[0] & 7, m[1] & 7, m[2] & 7);
        if (M.weight[P->vi] > 0.0f) {
            const float4 p = params[P->vi];
            const float n2 = p.y * p.y + p.z * p.z + p.w * p.w;
            if (n2 > 0.0f) {
                ok = true;
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
            }
        }
    }
    if (as && !a.freeze) {
        as[0] = ok ? m[0] : INT_MIN;
        as[1] = ok ? m[1] : INT_MIN;
        as[2] = ok ? m[2] : INT_MIN;
    }
    return ok;
}

// Grid (groups, K).  GRAD = false: loss only.  GRAD = true: loss, the
// scatter into dparams and the per-keyframe pose sums.
template <bool GRAD>
__global__ __launch_bounds__(kAdjBlock) void k_keyframe_loss(MapView M, AdjArgs a, const float* __restrict__ depth,
                                                             const double* __restrict__ T0,
                                                             const double* __restrict__ xi,
                                                             const float4* __restrict__ params,
                                                             const float* __restrict__ gscale,
                                                             int32_t* __restrict__ assoc, float* __restrict__ dparams,
                                                             double* __restrict__ partials) {
    __shared__ double s_pose[12];
    __shared__ double s_red[kAdjPart][kAdjBlock / 64];
    const int kf = blockIdx.y;
    if (threadIdx.x == 0) {
        double pose[12];
        for (int i = 0; i < 12; ++i) pose[i] = T0[12 * kf + i];
        se3_apply_left(xi + 6 * kf, pose);
        for (int i = 0; i < 12; ++i) s_pose[i] = pose[i];
    }
    __syncthreads();
    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = s_pose[4 * i + j];
        t[i] = s_pose[4 * i + 3];
    }
    const float s = GRAD ? gscale[kf] : 0.0f;
    const int N = a.W * a.H;
    const float* dimg = depth + (size_t)kf * N;
    int32_t* aimg = assoc ? assoc + (size_t)kf * N * 3 : nullptr;
    float acc[kAdjPart];
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) acc[k] = 0.0f;

    // A work-group takes 32x32 pixel tiles; a tile's pixels share a few
    // hundred voxels, so the gradient pass first adds each pixel's terms into
    // an LDS table keyed by voxel and then issues one set of global atomic
    // adds per distinct voxel of the tile (device-scope float atomics are
    // the costly part of the scatter).  A full table sends the pixel's terms
    // to global memory directly.  The larger the tile, the fewer of its
    // voxels it shares with its neighbours, which flush them again.
    __shared__ long long s_key[kAdjSet];
    __shared__ float s_val[4][kAdjSet];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tiles_x = (a.W + kAdjTile - 1) / kAdjTile;
    const int ntiles = tiles_x * ((a.H + kAdjTile - 1) / kAdjTile);
    for (int tile = blockIdx.x; tile < ntiles; tile += a.groups) {
        if (GRAD) {
            for (int e = threadIdx.x; e < kAdjSet; e += kAdjBlock) {
                s_key[e] = kAdjEmpty;
                s_val[0][e] = s_val[1][e] = s_val[2][e] = s_val[3][e] = 0.0f;
            }
            __syncthreads();
        }
        const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
        for (int px = threadIdx.x; px < kAdjTile * kAdjTile; px += kAdjBlock) {
            const int u = tx * kAdjTile + (px % kAdjTile);
            const int v = ty * kAdjTile + px / kAdjTile;
            const int i = v * a.W + u;
            PixelTerm P;
            bool ok = false;
            if (u < a.W && v < a.H)
                ok = pixel_term(M, a, R, t, params, dimg[i], u, v, aimg ? aimg + 3 * (size_t)i : nullptr, &P);
            if (ok) {
                const float r = P.psi + P.gh[0] * P.dq[0] + P.gh[1] * P.dq[1] + P.gh[2] * P.dq[2];
                const float ar = fabsf(r);
                const bool quad = ar <= a.delta;
                acc[0] += quad ? 0.5f * r * r : a.delta * (ar - 0.5f * a.delta);
                acc[7] += 1.0f;
                if (GRAD) {
                    const float rp = s * (quad ? r : copysignf(a.delta, r));   // s rho'(r)
                    const float J[6] = {P.gh[0], P.gh[1], P.gh[2], P.q[1] * P.gh[2] - P.q[2] * P.gh[1],
                                        P.q[2] * P.gh[0] - P.q[0] * P.gh[2], P.q[0] * P.gh[1] - P.q[1] * P.gh[0]};
#pragma unroll
                    for (int k = 0; k < 6; ++k) acc[1 + k] += rp * J[k];
                    const float gd = P.gh[0] * P.dq[0] + P.gh[1] * P.dq[1] + P.gh[2] * P.dq[2];
                    const float c = rp * P.inv_ng;
                    const float g4[4] = {rp, c * (P.dq[0] - P.gh[0] * gd), c * (P.dq[1] - P.gh[1] * gd),
                                         c * (P.dq[2] - P.gh[2] * gd)};
                    const long long key = (long long)P.vi;
                    unsigned h = (unsigned)(((unsigned long long)key * 0x9E3779B97F4A7C15ull) >> (64 - kAdjSetBits));
                    bool placed = false;
                    for (int probe = 0; probe < 32; ++probe) {
                        const long long old = (long long)atomicCAS(reinterpret_cast<unsigned long long*>(&s_key[h]),
                                                                   (unsigned long long)kAdjEmpty,
                                                                   (unsigned long long)key);
                        if (old == kAdjEmpty || old == key) {
#pragma unroll
                            for (int k = 0; k < 4; ++k) atomicAdd(&s_val[k][h], g4[k]);
                            placed = true;
                            break;
                        }
                        h = (h + 1) & (kAdjSet - 1);
                    }
                    if (!placed) {
                        float* dst = dparams + 4 * P.vi;
#pragma unroll
                        for (int k = 0; k < 4; ++k) atomicAdd(dst + k, g4[k]);
                    }
                }
            }
        }
        if (GRAD) {
            __syncthreads();
            for (int e = threadIdx.x; e < kAdjSet; e += kAdjBlock) {
                const long long key = s_key[e];
                if (key == kAdjEmpty) continue;
                float* dst = dparams + 4 * key;
#pragma unroll
                for (int k = 0; k < 4; ++k) atomicAdd(dst + k, s_val[k][e]);
            }
            __syncthreads();
        }
    }
    // work-group sums in float64: wave shuffles, then one value per wave
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) {
        double x = (double)acc[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) s_red[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x < kAdjPart) {
        double x = 0.0;
        for (int w = 0; w < kAdjBlock / 64; ++w) x += s_red[threadIdx.x][w];
        partials[((size_t)kf * a.groups + blockIdx.x) * kAdjPart + threadIdx.x] = x;
    }
}

// One work-group per keyframe: fixed-order sum of the partials (256 threads
// stride over the work-groups, then a tree in LDS), then loss_out[kf] and
// (when asked) dxi = Jl(xi)^T (pose sums).
__global__ __launch_bounds__(256) void k_keyframe_finish(AdjArgs a, const double* __restrict__ xi,
                                                         const double* __restrict__ partials,
                                                         double* __restrict__ loss_out, double* __restrict__ dxi_out,
                                                         double* __restrict__ count_out) {
    __shared__ double s_part[kAdjPart][256];
    const int kf = blockIdx.x;
    double x[kAdjPart];
#pragma unroll
    for (int k = 0; k < kAdjPart; ++k) x[k] = 0.0;
    for (int g = threadIdx.x; g < a.groups; g += 256) {
        const double* p = partials + ((size_t)kf * a.groups + g) * kAdjPart;
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
    return (size_t)n_keyframes * adj_groups(*cam) * kAdjPart * sizeof(double);
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
    {
        TimedLaunch tl(map->timer, GSDF_K_LOSS, s);
        k_keyframe_loss<false><<<dim3(a.groups, n_keyframes), kAdjBlock, 0, s>>>(
            make_view(*map), a, depth_dev, T0_dev, xi_dev, reinterpret_cast<const float4*>(params_dev), nullptr,
            assoc_dev, nullptr, (double*)scratch);
    }
    k_keyframe_finish<<<n_keyframes, 256, 0, s>>>(a, xi_dev, (const double*)scratch, loss_dev, nullptr, count_dev);
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
    {
        TimedLaunch tl(map->timer, GSDF_K_BACKWARD, s);
        k_keyframe_loss<true><<<dim3(a.groups, n_keyframes), kAdjBlock, 0, s>>>(
            make_view(*map), a, depth_dev, T0_dev, xi_dev, reinterpret_cast<const float4*>(params_dev),
            grad_loss_dev, assoc_dev, dparams_dev, (double*)scratch);
    }
    k_keyframe_finish<<<n_keyframes, 256, 0, s>>>(a, xi_dev, (const double*)scratch, loss_dev, dxi_dev, nullptr);
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
