// Oriented point cloud from the map (Sec. 4.3).
//
// Every observed voxel whose surface point lies inside its cell
// (|psi_j gh_jk| <= v_s/2 for each axis k) gives the point v_j - psi_j gh_j
// with normal -gh_j (gh points into the solid, so -gh faces free space).
// Upsampled (level 1): each voxel is split into 2x2x2 subvoxels with centres
// s = v_j + (v_s/4)(+-1, +-1, +-1); the Taylor expansion of the distance,
// psi(s) = psi_j + gh_j . (s - v_j), decides (|psi(s) gh_jk| <= v_s/4) and
// places the point s - psi(s) gh_j.  Selection is decided in float64 from the
// stored values; points and normals are written as float32.
//
// Three passes give a deterministic order (block slot, then voxel
// lx + 8 ly + 64 lz, then subvoxel sx + 2 sy + 4 sz): per-block counts, an
// exclusive scan over the blocks, and the write at the scanned offsets.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "gsdf.h"
#include "gsdf_common.hpp"
#include "gsdf_host.hpp"

namespace gsdf {

constexpr int kSurfBlock = 256;

// Stored distance and unit gradient of voxel vi; false when unobserved.
__device__ inline bool stored_voxel(const MapView& M, int storage, int64_t vi, double* psi, double gh[3]) {
    float p, g[3];
    if (!(load_voxel(M, storage, vi, &p, g) > 0.0f)) return false;
    const double ng = sqrt((double)g[0] * g[0] + (double)g[1] * g[1] + (double)g[2] * g[2]);
    if (!(ng > 0.0)) return false;
    for (int k = 0; k < 3; ++k) gh[k] = g[k] / ng;
    *psi = p;
    return true;
}

// Surfels of voxel (lx, ly, lz) of block (bx, by, bz): bit mask of the
// subvoxels taking part (bit 0 for level 0).
__device__ inline unsigned voxel_surfels(const MapView& M, int storage, int level, int64_t slot, int bx, int by,
                                         int bz, int c, double* psi, double gh[3], double v[3]) {
    const int lx = c & 7, ly = (c >> 3) & 7, lz = c >> 6;
    const int64_t vi = slot * kBlockVoxels + morton9(lx, ly, lz);
    if (!stored_voxel(M, storage, vi, psi, gh)) return 0u;
    const double vs = M.voxel_size_d;
    v[0] = vs * (8 * bx + lx);
    v[1] = vs * (8 * by + ly);
    v[2] = vs * (8 * bz + lz);
    if (level == 0) {
        bool in = true;
        for (int k = 0; k < 3; ++k) in = in && fabs(*psi * gh[k]) <= 0.5 * vs;
        return in ? 1u : 0u;
    }
    unsigned mask = 0u;
    for (int sub = 0; sub < 8; ++sub) {
        double ps = *psi;
        for (int k = 0; k < 3; ++k) ps += gh[k] * (((sub >> k) & 1) ? 0.25 * vs : -0.25 * vs);
        bool in = true;
        for (int k = 0; k < 3; ++k) in = in && fabs(ps * gh[k]) <= 0.25 * vs;
        if (in) mask |= 1u << sub;
    }
    return mask;
}

// Block-wide exclusive scan of one int per thread (256 threads).
__device__ inline int block_exclusive_scan(int x, int* total, int* s_warp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = x;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    if (lane == 63) s_warp[wave] = incl;
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += s_warp[w];
    *total = s_warp[0] + s_warp[1] + s_warp[2] + s_warp[3];
    __syncthreads();
    return base + incl - x;
}

// PASS 0: count per block; PASS 1: write at offsets[slot].
template <int PASS>
__global__ __launch_bounds__(kSurfBlock) void k_surfels(MapView M, int storage, int level, int32_t* __restrict__ counts,
                                                        const int64_t* __restrict__ offsets, int64_t capacity,
                                                        float* __restrict__ points, float* __restrict__ normals,
                                                        int32_t* __restrict__ ids) {
    __shared__ int s_warp[4];
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    for (int64_t slot = blockIdx.x; slot < nb; slot += gridDim.x) {
        int bx, by, bz;
        unpack_key(M.block_keys[slot], &bx, &by, &bz);
        int64_t base = PASS == 1 ? offsets[slot] : 0;
        int block_total = 0;
        // two voxels per thread, in voxel order lx + 8 ly + 64 lz
        for (int half = 0; half < 2; ++half) {
            const int c = half * kSurfBlock + threadIdx.x;
            double psi, gh[3], v[3];
            const unsigned mask = voxel_surfels(M, storage, level, slot, bx, by, bz, c, &psi, gh, v);
            const int n = __popc(mask);
            int total;
            const int off = block_exclusive_scan(n, &total, s_warp);
            if (PASS == 1 && mask) {
                int k = 0;
                for (int sub = 0; sub < (level == 0 ? 1 : 8); ++sub) {
                    if (!(mask & (1u << sub))) continue;
                    const int64_t o = base + off + k++;
                    if (o >= capacity) continue;
                    double s[3] = {v[0], v[1], v[2]}, ps = psi;
                    if (level == 1) {
                        for (int a = 0; a < 3; ++a) {
                            const double d = ((sub >> a) & 1) ? 0.25 * M.voxel_size_d : -0.25 * M.voxel_size_d;
                            s[a] += d;
                            ps += gh[a] * d;
                        }
                    }
                    for (int a = 0; a < 3; ++a) {
                        points[3 * o + a] = (float)(s[a] - ps * gh[a]);
                        normals[3 * o + a] = (float)(-gh[a]);
                    }
                    ids[4 * o] = 8 * bx + (c & 7);
                    ids[4 * o + 1] = 8 * by + ((c >> 3) & 7);
                    ids[4 * o + 2] = 8 * bz + (c >> 6);
                    ids[4 * o + 3] = level == 0 ? 0 : sub;
                }
            }
            base += total;
            block_total += total;
        }
        if (PASS == 0 && threadIdx.x == 0) counts[slot] = block_total;
    }
}

// Exclusive scan of the per-block counts (one work-group) and the total.
__global__ __launch_bounds__(1024) void k_surfel_scan(MapView M, const int32_t* __restrict__ counts,
                                                      int64_t* __restrict__ offsets, int64_t* __restrict__ total) {
    __shared__ int64_t s_part[1024];
    const int32_t nb = M.counters[kNumBlocks] < M.max_blocks ? M.counters[kNumBlocks] : M.max_blocks;
    const int per = (nb + 1023) / 1024;
    const int64_t lo = (int64_t)threadIdx.x * per;
    int64_t sum = 0;
    for (int64_t i = lo; i < lo + per && i < nb; ++i) sum += counts[i];
    s_part[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t y = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0;
        __syncthreads();
        s_part[threadIdx.x] += y;
        __syncthreads();
    }
    int64_t run = s_part[threadIdx.x] - sum;
    for (int64_t i = lo; i < lo + per && i < nb; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
    if (threadIdx.x == 1023) *total = s_part[1023];
}

}  // namespace gsdf

using namespace gsdf;

extern "C" {

size_t gsdf_surfel_scratch_bytes(const gsdf_map* map) {
    if (!valid_map(map)) return 0;
    return (size_t)map->desc.max_blocks * (sizeof(int32_t) + sizeof(int64_t)) + 256;
}

int gsdf_extract_surfels(const gsdf_map* map, int32_t level, float* points_dev, float* normals_dev, int32_t* ids_dev,
                         int64_t capacity, int64_t* count_dev, void* scratch_dev, size_t scratch_bytes, void* stream) {
    if (!valid_map(map) || !has_gradients(map) || (level != 0 && level != 1) || capacity < 0 || !count_dev ||
        !scratch_dev ||
        scratch_bytes < gsdf_surfel_scratch_bytes(map) ||
        (capacity > 0 && (!points_dev || !normals_dev || !ids_dev)))
        return GSDF_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const MapView M = make_view(*map);
    int64_t* offsets = (int64_t*)scratch_dev;
    int32_t* counts = (int32_t*)((char*)scratch_dev + (size_t)map->desc.max_blocks * sizeof(int64_t));
    const unsigned grid = 2048;
    k_surfels<0><<<grid, kSurfBlock, 0, s>>>(M, map->desc.storage, level, counts, nullptr, 0, nullptr, nullptr,
                                             nullptr);
    k_surfel_scan<<<1, 1024, 0, s>>>(M, counts, offsets, count_dev);
    if (capacity > 0)
        k_surfels<1><<<grid, kSurfBlock, 0, s>>>(M, map->desc.storage, level, counts, offsets, capacity, points_dev,
                                                 normals_dev, ids_dev);
    return launch_status();
}

}  // extern "C"
