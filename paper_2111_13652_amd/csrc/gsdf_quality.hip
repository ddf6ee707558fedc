// Gradient quality of the map against a known union of spheres (Sec. 5.2,
// App. A): the stored gradient and finite differences of the stored distance
// (forward, backward, central, step v_s along each axis), each as an angle to
// the true gradient of the distance.
//
// For the spheres (c, r) the nearest surface of a voxel centre v is the one
// minimising | |v - c| - r |; with psi > 0 inside, the true gradient there is
// (c - v)/|c - v|.  A voxel is evaluated when it is observed (W > 0, g != 0);
// the differences need the voxel's six face neighbours observed (W > 0),
// looked up across block borders through the hash table.
//
// One work-group per block slot (grid-stride).  The six face-neighbour slots
// are found once per block and kept in LDS; each thread takes two voxels in
// the order lx + 8 ly + 64 lz.  Differences and angles are formed in float64
// from the binary32 stored distances; results are written as float32 into 5
// planes of `stride` values: distance to the surface, then the angles in
// degrees of the stored gradient and of the forward, backward and central
// differences (NaN where undefined).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gsdf.h"
#include "gsdf_common.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

constexpr int kQualBlock = 256;
constexpr int kMaxSpheres = 64;

__device__ inline double angle_deg(const double a[3], const double b[3]) {
    const double x = a[1] * b[2] - a[2] * b[1];
    const double y = a[2] * b[0] - a[0] * b[2];
    const double z = a[0] * b[1] - a[1] * b[0];
    const double d = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    return atan2(sqrt(x * x + y * y + z * z), d) * (180.0 / M_PI);
}

__global__ __launch_bounds__(kQualBlock) void k_gradient_quality(MapView M, int storage,
                                                                 const double* __restrict__ spheres, int ns,
                                                                 float* __restrict__ out, int64_t stride) {
    __shared__ double s_sph[4 * kMaxSpheres];
    __shared__ int32_t s_nb[6];  // +x, -x, +y, -y, +z, -z
    for (int i = threadIdx.x; i < 4 * ns; i += kQualBlock) s_sph[i] = spheres[i];
    const int32_t nb_all = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    const int64_t slots_out = stride / kBlockVoxels;
    const int32_t nb = (int64_t)nb_all < slots_out ? nb_all : (int32_t)slots_out;
    const double vs = M.voxel_size_d;
    const float nanf = __int_as_float(0x7fc00000);
    for (int32_t slot = blockIdx.x; slot < nb; slot += gridDim.x) {
        int bx, by, bz;
        unpack_key(M.block_keys[slot], &bx, &by, &bz);
        __syncthreads();  // s_nb of the previous slot is no longer read
        if (threadIdx.x < 6) {
            const int axis = threadIdx.x >> 1, dir = (threadIdx.x & 1) ? -1 : 1;
            s_nb[threadIdx.x] = hash_find(M, bx + (axis == 0 ? dir : 0), by + (axis == 1 ? dir : 0),
                                          bz + (axis == 2 ? dir : 0));
        }
        __syncthreads();
        for (int half = 0; half < 2; ++half) {
            const int c = half * kQualBlock + threadIdx.x;
            const int l[3] = {c & 7, (c >> 3) & 7, c >> 6};
            const int64_t o = (int64_t)slot * kBlockVoxels + c;
            float res[5] = {nanf, nanf, nanf, nanf, nanf};
            float psi, g[3];
            const float Wv = load_voxel(M, storage, (int64_t)slot * kBlockVoxels + morton9(l[0], l[1], l[2]), &psi, g);
            if (Wv > 0.0f && (g[0] != 0.0f || g[1] != 0.0f || g[2] != 0.0f) && ns > 0) {
                const double v[3] = {vs * (8 * bx + l[0]), vs * (8 * by + l[1]), vs * (8 * bz + l[2])};
                int best = 0;
                double bd = INFINITY;
                for (int s = 0; s < ns; ++s) {
                    const double* S = s_sph + 4 * s;
                    const double r = sqrt((v[0] - S[0]) * (v[0] - S[0]) + (v[1] - S[1]) * (v[1] - S[1]) +
                                          (v[2] - S[2]) * (v[2] - S[2]));
                    if (fabs(r - S[3]) < bd) {
                        bd = fabs(r - S[3]);
                        best = s;
                    }
                }
                const double* S = s_sph + 4 * best;
                const double gt[3] = {S[0] - v[0], S[1] - v[1], S[2] - v[2]};
                const double gs[3] = {g[0], g[1], g[2]};
                res[0] = (float)bd;
                res[1] = (float)angle_deg(gs, gt);
                // the six face neighbours
                double pp[3], pm[3];
                bool ok = true;
                for (int k = 0; k < 3 && ok; ++k) {
                    for (int s = 0; s < 2 && ok; ++s) {
                        int q[3] = {l[0], l[1], l[2]};
                        q[k] += s == 0 ? 1 : -1;
                        int32_t nslot = slot;
                        if (q[k] < 0 || q[k] > 7) {
                            nslot = s_nb[2 * k + s];
                            q[k] &= 7;
                        }
                        float pn, gn[3];
                        ok = nslot >= 0 &&
                             load_voxel(M, storage, (int64_t)nslot * kBlockVoxels + morton9(q[0], q[1], q[2]), &pn,
                                        gn) > 0.0f;
                        if (ok) (s == 0 ? pp : pm)[k] = pn;
                    }
                }
                if (ok) {
                    double f[3], b[3], ce[3];
                    for (int k = 0; k < 3; ++k) {
                        f[k] = (pp[k] - (double)psi) / vs;
                        b[k] = ((double)psi - pm[k]) / vs;
                        ce[k] = (pp[k] - pm[k]) / (2.0 * vs);
                    }
                    res[2] = (float)angle_deg(f, gt);
                    res[3] = (float)angle_deg(b, gt);
                    res[4] = (float)angle_deg(ce, gt);
                }
            }
            for (int q = 0; q < 5; ++q) out[q * stride + o] = res[q];
        }
    }
}

}  // namespace gsdf

using namespace gsdf;

extern "C" {

int gsdf_gradient_quality(const gsdf_map* map, const double* spheres_dev, int32_t n_spheres, float* out_dev,
                          int64_t stride, void* stream) {
    if (!valid_map(map) || !has_gradients(map) || !spheres_dev || n_spheres < 1 || n_spheres > kMaxSpheres || !out_dev || stride < 0 ||
        stride % kBlockVoxels != 0)
        return GSDF_EINVAL;
    if (stride == 0) return GSDF_OK;
    const MapView M = make_view(*map);
    const int64_t slots = stride / kBlockVoxels;
    const unsigned grid = (unsigned)(slots < 2048 ? slots : 2048);
    k_gradient_quality<<<grid, kQualBlock, 0, (hipStream_t)stream>>>(M, map->desc.storage, spheres_dev, n_spheres,
                                                                     out_dev, stride);
    return launch_status();
}

}  // extern "C"
