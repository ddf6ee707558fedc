// track_frame: direct SDF tracking with one voxel lookup per pixel
// (Gradient-SDF Sec. 4.1, Eq. (5) and (14)-(16)), Huber-weighted
// Gauss-Newton, and the damped 6x6 Cholesky solve with a left SE(3) update
// (Sec. 5.1), all on the device.
//
// Each Gauss-Newton iteration is one launch.  Every thread walks a strided
// set of pixels, accumulating the 21 upper entries of H = sum w J J^T, the
// 6 of b = sum w J r, the energy, the count of pixels used and the count of
// valid pixels in float32 registers; from there on every sum is float64:
// waves reduce with cross-lane shuffles, the 4 waves of a work-group through
// LDS, and the last work-group to finish (a device-scope ticket) adds all
// work-group partials, solves, updates the pose in place and records the
// statistics.  Float64 partial sums keep the rounding noise of b far below
// what a rank-deficient H (a lone sphere) would amplify through the damping.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "gsdf_common.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

constexpr int kNE = 30;          // 21 H + 6 b + energy + used + valid
constexpr int kPartStride = 32;  // doubles per work-group partial
constexpr int kTrackBlock = 256;
constexpr int kMaxGroups = 2048;
constexpr int kPixPerThread = 2;

struct TrackLevel {
    const float* depth;
    int W, H;
    double ifx, ify, cx, cy;
};

struct TrackArgs {
    float zmin, zmax, delta;
    double inv_vs, vs;
    double damping;
    float min_inlier_frac;
    int mode;            // 0: solve and update the pose; 1: write sums to out29
    int stat_slot;       // iteration index for stats, -1 for none
    int check_lost;      // 1 on the last iteration at the finest level
};

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Voxel values of the map at pool index vi: psi, gradient direction; false
// when unobserved.
template <int STORAGE>
__device__ inline bool read_voxel(const MapView& M, int64_t vi, float* psi, float gh[3]) {
    const float Wv = M.weight[vi];
    if (!(Wv > 0.0f)) return false;
    float g0, g1, g2;
    if (STORAGE == GSDF_FP32) {
        const float4 r = reinterpret_cast<const float4*>(M.vox)[vi];
        *psi = r.x / Wv;
        g0 = r.y;
        g1 = r.z;
        g2 = r.w;
    } else {
        const ushort4 p = reinterpret_cast<const ushort4*>(M.vox)[vi];
        *psi = unpack16(p.x, STORAGE) * M.truncation;
        g0 = unpack16(p.y, STORAGE);
        g1 = unpack16(p.z, STORAGE);
        g2 = unpack16(p.w, STORAGE);
    }
    const float n2 = g0 * g0 + g1 * g1 + g2 * g2;
    if (!(n2 > 0.0f)) return false;
    const float inv = 1.0f / sqrtf(n2);
    gh[0] = g0 * inv;
    gh[1] = g1 * inv;
    gh[2] = g2 * inv;
    return true;
}

// Cholesky solve of the damped 6x6 system and left update of the pose.
__device__ bool solve_and_update(const double* ne, double damping, double* pose) {
    double H[36];
    int k = 0;
    for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
            H[6 * i + j] = ne[k];
            H[6 * j + i] = ne[k];
            ++k;
        }
    double tr = 0;
    for (int i = 0; i < 6; ++i) tr += H[7 * i];
    const double mu = damping * tr / 6.0;
    for (int i = 0; i < 6; ++i) H[7 * i] += mu;
    double L[36];
    for (int i = 0; i < 36; ++i) L[i] = 0.0;
    for (int j = 0; j < 6; ++j) {
        double s = H[7 * j];
        for (int q = 0; q < j; ++q) s -= L[6 * j + q] * L[6 * j + q];
        if (!(s > 0.0)) return false;
        const double d = sqrt(s);
        L[7 * j] = d;
        for (int i = j + 1; i < 6; ++i) {
            double t = H[6 * i + j];
            for (int q = 0; q < j; ++q) t -= L[6 * i + q] * L[6 * j + q];
            L[6 * i + j] = t / d;
        }
    }
    double y[6], x[6];
    for (int i = 0; i < 6; ++i) {
        double s = -ne[21 + i];
        for (int q = 0; q < i; ++q) s -= L[6 * i + q] * y[q];
        y[i] = s / L[7 * i];
    }
    for (int i = 5; i >= 0; --i) {
        double s = y[i];
        for (int q = i + 1; q < 6; ++q) s -= L[6 * q + i] * x[q];
        x[i] = s / L[7 * i];
    }
    // exp of the twist (rho, phi) = (x[0..2], x[3..5])
    const double* rho = x;
    const double* phi = x + 3;
    const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-4) {
        A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
        B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
        C = 1.0 / 6.0 - th2 / 120.0 + th2 * th2 / 5040.0;
    } else {
        const double sn = sin(th), cs = cos(th);
        A = sn / th;
        B = (1.0 - cs) / th2;
        C = (th - sn) / (th2 * th);
    }
    const double K[9] = {0, -phi[2], phi[1], phi[2], 0, -phi[0], -phi[1], phi[0], 0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
    double Rd[9], V[9];
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        Rd[i] = I + A * K[i] + B * K2[i];
        V[i] = I + B * K[i] + C * K2[i];
    }
    double td[3];
    for (int i = 0; i < 3; ++i) td[i] = V[3 * i] * rho[0] + V[3 * i + 1] * rho[1] + V[3 * i + 2] * rho[2];
    double out[12];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 4; ++j) {
            double s = Rd[3 * i] * pose[j] + Rd[3 * i + 1] * pose[4 + j] + Rd[3 * i + 2] * pose[8 + j];
            if (j == 3) s += td[i];
            out[4 * i + j] = s;
        }
    }
    for (int i = 0; i < 12; ++i) pose[i] = out[i];
    return true;
}

template <int STORAGE>
__global__ __launch_bounds__(kTrackBlock) void k_track(MapView M, TrackLevel L, TrackArgs a,
                                                        double* pose, double* partials,
                                                        unsigned* ticket, double* out29,
                                                        float* stats, int32_t* status) {
    float acc[kNE];
#pragma unroll
    for (int k = 0; k < kNE; ++k) acc[k] = 0.0f;

    double R[9], t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) R[3 * i + j] = pose[4 * i + j];
        t[i] = pose[4 * i + 3];
    }
    const int N = L.W * L.H;
    for (int i = blockIdx.x * kTrackBlock + threadIdx.x; i < N; i += gridDim.x * kTrackBlock) {
        const float D = L.depth[i];
        if (!depth_ok(D, a.zmin, a.zmax)) continue;
        acc[29] += 1.0f;
        const int v = i / L.W;
        const int u = i - v * L.W;
        const double Dd = (double)D;
        const double x0 = Dd * (((double)u - L.cx) * L.ifx);
        const double x1 = Dd * (((double)v - L.cy) * L.ify);
        double q[3];
        int m[3];
        float qr[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            q[r] = R[3 * r] * x0 + R[3 * r + 1] * x1 + R[3 * r + 2] * Dd + t[r];
            m[r] = (int)floor(q[r] * a.inv_vs + 0.5);
            qr[r] = (float)(q[r] - a.vs * (double)m[r]);
        }
        const int32_t slot = hash_find(M, block_of(m[0]), block_of(m[1]), block_of(m[2]));
        if (slot < 0) continue;
        const int64_t vi = (int64_t)slot * kBlockVoxels + morton9(m[0] & 7, m[1] & 7, m[2] & 7);
        float psi, gh[3];
        if (!read_voxel<STORAGE>(M, vi, &psi, gh)) continue;
        const float r = psi + gh[0] * qr[0] + gh[1] * qr[1] + gh[2] * qr[2];
        const float qf[3] = {(float)q[0], (float)q[1], (float)q[2]};
        const float J[6] = {gh[0], gh[1], gh[2], qf[1] * gh[2] - qf[2] * gh[1],
                            qf[2] * gh[0] - qf[0] * gh[2], qf[0] * gh[1] - qf[1] * gh[0]};
        const float ar = fabsf(r);
        const float w = ar <= a.delta ? 1.0f : a.delta / ar;
        const float e = ar <= a.delta ? 0.5f * r * r : a.delta * (ar - 0.5f * a.delta);
        int k = 0;
#pragma unroll
        for (int p = 0; p < 6; ++p) {
            const float wj = w * J[p];
#pragma unroll
            for (int q2 = p; q2 < 6; ++q2) acc[k++] += wj * J[q2];
        }
#pragma unroll
        for (int p = 0; p < 6; ++p) acc[21 + p] += w * J[p] * r;
        acc[27] += e;
        acc[28] += 1.0f;
    }

    // ---- work-group reduction
    __shared__ double red[kTrackBlock / 64][kNE];
    __shared__ double fin[8][kNE];
    __shared__ int is_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < kNE; ++k) {
        const double s = wave_sum((double)acc[k]);
        if (lane == 0) red[wave][k] = s;
    }
    __syncthreads();
    if (threadIdx.x < kNE) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kTrackBlock / 64; ++w) s += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * kPartStride + threadIdx.x] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned prev = atomicAdd(ticket, 1u);
        is_last = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();

    // ---- last work-group: float64 total of all partials
    if (threadIdx.x < 8 * kNE) {
        const int k = threadIdx.x % kNE;
        const int part = threadIdx.x / kNE;
        double s = 0.0;
        for (int b = part; b < (int)gridDim.x; b += 8)
            s += __hip_atomic_load(&partials[(size_t)b * kPartStride + k], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        fin[part][k] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ne[kNE];
        for (int k = 0; k < kNE; ++k) {
            double s = 0.0;
            for (int p = 0; p < 8; ++p) s += fin[p][k];
            ne[k] = s;
        }
        if (a.mode == 1) {
            for (int k = 0; k < 29; ++k) out29[k] = ne[k];
        } else {
            if (a.stat_slot >= 0 && stats) {
                stats[2 * a.stat_slot] = (float)ne[27];
                stats[2 * a.stat_slot + 1] = (float)ne[28];
            }
            if (!solve_and_update(ne, a.damping, pose)) raise_status(status, GSDF_ENOTPD);
            if (a.check_lost && ne[28] < (double)a.min_inlier_frac * ne[29])
                raise_status(status, GSDF_ELOST);
        }
        *ticket = 0u;
    }
}

// 2x2 pyramid level in binary32: the mean of four valid depths whose spread
// is within the truncation, else 0.  Work-item (0,0) also clears the ticket.
__global__ void k_pyramid(const float* __restrict__ src, int Ws, float* __restrict__ dst, int Wd,
                          int Hd, float zmin, float zmax, float Tf, unsigned* ticket) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y * blockDim.y + threadIdx.y;
    if (ticket && u == 0 && v == 0) *ticket = 0u;
    if (u >= Wd || v >= Hd) return;
    const float a = src[(size_t)(2 * v) * Ws + 2 * u];
    const float b = src[(size_t)(2 * v) * Ws + 2 * u + 1];
    const float c = src[(size_t)(2 * v + 1) * Ws + 2 * u];
    const float e = src[(size_t)(2 * v + 1) * Ws + 2 * u + 1];
    bool ok = depth_ok(a, zmin, zmax) && depth_ok(b, zmin, zmax) && depth_ok(c, zmin, zmax) &&
              depth_ok(e, zmin, zmax);
    const float mx = fmaxf(fmaxf(a, b), fmaxf(c, e));
    const float mn = fminf(fminf(a, b), fminf(c, e));
    ok = ok && (sub_rn(mx, mn) <= Tf);
    dst[(size_t)v * Wd + u] = ok ? mul_rn(add_rn(add_rn(a, b), add_rn(c, e)), 0.25f) : 0.0f;
}

__global__ void k_zero_ticket(unsigned* ticket) {
    if (threadIdx.x == 0) *ticket = 0u;
}

struct ScratchLayout {
    size_t ticket, partials, level[4], total;
};

inline ScratchLayout scratch_layout(const gsdf_camera& c, int levels) {
    ScratchLayout s;
    size_t o = 0;
    s.ticket = o;   o = align256(o + 256);
    s.partials = o; o = align256(o + (size_t)kMaxGroups * kPartStride * 8);
    int W = c.width, H = c.height;
    s.level[0] = 0;
    for (int l = 1; l < 4; ++l) {
        W /= 2;
        H /= 2;
        s.level[l] = o;
        if (l < levels) o = align256(o + (size_t)W * H * 4);
    }
    s.total = o;
    return s;
}

inline int track_groups(int npx) {
    int g = ceil_div(npx, kTrackBlock * kPixPerThread);
    return g < 1 ? 1 : (g > kMaxGroups ? kMaxGroups : g);
}

template <int STORAGE>
void launch_track(int g, hipStream_t s, const MapView& M, const TrackLevel& L, const TrackArgs& a,
                  double* pose, double* partials, unsigned* ticket, double* out29, float* stats,
                  int32_t* status) {
    k_track<STORAGE><<<g, kTrackBlock, 0, s>>>(M, L, a, pose, partials, ticket, out29, stats, status);
}

void launch_track_any(int storage, int g, hipStream_t s, const MapView& M, const TrackLevel& L,
                      const TrackArgs& a, double* pose, double* partials, unsigned* ticket,
                      double* out29, float* stats, int32_t* status) {
    TimedLaunch tl(GSDF_K_TRACK, s);
    switch (storage) {
        case GSDF_FP32: launch_track<GSDF_FP32>(g, s, M, L, a, pose, partials, ticket, out29, stats, status); break;
        case GSDF_BF16: launch_track<GSDF_BF16>(g, s, M, L, a, pose, partials, ticket, out29, stats, status); break;
        default: launch_track<GSDF_FP16>(g, s, M, L, a, pose, partials, ticket, out29, stats, status); break;
    }
}

}  // namespace gsdf

using namespace gsdf;

extern "C" size_t gsdf_track_scratch_bytes(const gsdf_camera* cam, int32_t levels) {
    if (!valid_cam(cam) || levels < 1 || levels > 4) return 0;
    return scratch_layout(*cam, levels).total;
}

extern "C" int gsdf_track_frame(const gsdf_map* map, const float* depth_dev, const gsdf_camera* cam,
                                const gsdf_track_params* params, double* T_wc_inout_dev,
                                float* stats_dev, void* scratch_dev, size_t scratch_bytes,
                                int32_t* status_dev, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !params || !T_wc_inout_dev || !scratch_dev)
        return GSDF_EINVAL;
    const int levels = params->levels;
    if (levels < 1 || levels > 4) return GSDF_EINVAL;
    for (int l = 0; l < levels; ++l)
        if (params->iters[l] < 0 || params->iters[l] > 1000) return GSDF_EINVAL;
    if ((cam->width >> (levels - 1)) < 1 || (cam->height >> (levels - 1)) < 1) return GSDF_EINVAL;
    const ScratchLayout sl = scratch_layout(*cam, levels);
    if (scratch_bytes < sl.total) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch_dev;
    unsigned* ticket = (unsigned*)(base + sl.ticket);
    double* partials = (double*)(base + sl.partials);

    TrackLevel lv[4];
    lv[0].depth = depth_dev;
    lv[0].W = cam->width;
    lv[0].H = cam->height;
    double fx = cam->fx, fy = cam->fy, cx = cam->cx, cy = cam->cy;
    lv[0].ifx = 1.0 / fx;
    lv[0].ify = 1.0 / fy;
    lv[0].cx = cx;
    lv[0].cy = cy;
    for (int l = 1; l < levels; ++l) {
        fx /= 2;
        fy /= 2;
        cx = (cx + 0.5) / 2 - 0.5;
        cy = (cy + 0.5) / 2 - 0.5;
        lv[l].depth = (const float*)(base + sl.level[l]);
        lv[l].W = lv[l - 1].W / 2;
        lv[l].H = lv[l - 1].H / 2;
        lv[l].ifx = 1.0 / fx;
        lv[l].ify = 1.0 / fy;
        lv[l].cx = cx;
        lv[l].cy = cy;
    }
    {
        TimedLaunch tp(GSDF_K_PYRAMID, s);
        if (levels == 1) k_zero_ticket<<<1, 64, 0, s>>>(ticket);
        for (int l = 1; l < levels; ++l) {
            dim3 blk(16, 16), grd(ceil_div(lv[l].W, 16), ceil_div(lv[l].H, 16));
            k_pyramid<<<grd, blk, 0, s>>>(lv[l - 1].depth, lv[l - 1].W, (float*)lv[l].depth, lv[l].W,
                                          lv[l].H, cam->zmin, cam->zmax, (float)map->desc.truncation,
                                          l == 1 ? ticket : nullptr);
        }
    }
    const MapView M = make_view(*map);
    TrackArgs a;
    a.zmin = cam->zmin;
    a.zmax = cam->zmax;
    a.delta = params->huber_delta;
    a.inv_vs = 1.0 / map->desc.voxel_size;
    a.vs = map->desc.voxel_size;
    a.damping = params->damping;
    a.min_inlier_frac = params->min_inlier_frac;
    a.mode = 0;
    int slot = 0;
    for (int l = levels - 1; l >= 0; --l) {
        const int g = track_groups(lv[l].W * lv[l].H);
        for (int it = 0; it < params->iters[l]; ++it) {
            a.stat_slot = slot++;
            a.check_lost = (l == 0 && it == params->iters[0] - 1) ? 1 : 0;
            launch_track_any(map->desc.storage, g, s, M, lv[l], a, T_wc_inout_dev, partials, ticket,
                             nullptr, stats_dev, status_dev);
        }
    }
    return launch_status();
}

extern "C" int gsdf_normal_equations(const gsdf_map* map, const float* depth_dev,
                                     const gsdf_camera* cam, const double* T_wc_dev,
                                     float huber_delta, double* out29_dev, void* scratch_dev,
                                     size_t scratch_bytes, void* stream) {
    if (!valid_map(map) || !depth_dev || !valid_cam(cam) || !T_wc_dev || !out29_dev || !scratch_dev)
        return GSDF_EINVAL;
    const ScratchLayout sl = scratch_layout(*cam, 1);
    if (scratch_bytes < sl.total) return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    char* base = (char*)scratch_dev;
    unsigned* ticket = (unsigned*)(base + sl.ticket);
    double* partials = (double*)(base + sl.partials);
    TrackLevel L;
    L.depth = depth_dev;
    L.W = cam->width;
    L.H = cam->height;
    L.ifx = 1.0 / cam->fx;
    L.ify = 1.0 / cam->fy;
    L.cx = cam->cx;
    L.cy = cam->cy;
    TrackArgs a;
    a.zmin = cam->zmin;
    a.zmax = cam->zmax;
    a.delta = huber_delta;
    a.inv_vs = 1.0 / map->desc.voxel_size;
    a.vs = map->desc.voxel_size;
    a.damping = 0.0;
    a.min_inlier_frac = 0.0f;
    a.mode = 1;
    a.stat_slot = -1;
    a.check_lost = 0;
    k_zero_ticket<<<1, 64, 0, s>>>(ticket);
    launch_track_any(map->desc.storage, track_groups(L.W * L.H), s, make_view(*map), L, a,
                     const_cast<double*>(T_wc_dev), partials, ticket, out29_dev, nullptr, nullptr);
    return launch_status();
}
